"""Periodic Hermitisation and trace renormalisation of rho (FP64).

The paper evolves rho with Eq. (6) only; a density matrix is Hermitian with
unit trace, so the reduced-precision forms restore those two properties
every few steps:  rho <- (rho + rho^dag) / 2,  then  rho <- rho / Re Tr rho.
"""
from __future__ import annotations

import numpy as np


def hermitize_normalize(rho: np.ndarray) -> np.ndarray:
    h = 0.5 * (rho + rho.conj().T)
    return h / np.trace(h).real
