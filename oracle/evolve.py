"""Unitary evolution of the density matrix: exact and stepped references.

Sec. III.A, Eq. (6): rho(t+dt) = exp(-i H dt) rho(t) exp(+i H dt) (hbar = 1).
Stepping this S times gives rho(S dt) = exp(-i H S dt) rho(0) exp(+i H S dt)
exactly, which is the plain definition every route below computes:

  propagator        U = exp(-i H dt) from the Hermitian eigendecomposition
                    H = V diag(lam) V^T (V real because H is real symmetric)
  evolve_dense      rho <- U rho U^dag, step by step (Eq. (6))
  evolve_exact      rho(t) = W(t) rho0 W(t)^dag with W(t) = V e^{-i lam t} V^T
  evolve_sectors    the same for a pure state, block by block over the
                    excitation sectors of H (H commutes with N_exc)
  evolve_bruteforce state vector psi <- expm(-i H dt) psi with scipy's expm
  taylor_factors    Eq. (10)-(11): L and R as the Taylor series of the
                    exponentials truncated at k_max = 10, powers formed as
                    right-nested products (Eq. (9)); step rho <- L (rho R)
                    in the order of Eq. (12) with Eq. (9b)
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import model


def propagator(H: np.ndarray, t: float) -> np.ndarray:
    """exp(-i H t) for real symmetric H via numpy's eigh."""
    lam, V = np.linalg.eigh(H)
    return (V * np.exp(-1j * lam * t)) @ V.T


def step(U: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """One application of Eq. (6): U rho U^dag."""
    return U @ rho @ U.conj().T


def evolve_dense(U: np.ndarray, rho0: np.ndarray, steps: int, record_every: int = 1,
                 observe=None, renorm_every: int = 0):
    """Dense stepping of Eq. (6).  Returns (rho_final, records) where records
    holds observe(rho) after every record_every steps, starting with rho0."""
    from .renorm import hermitize_normalize
    rho = np.array(rho0, dtype=np.complex128, copy=True)
    records = []
    if observe is not None:
        records.append(observe(rho))
    for s in range(1, steps + 1):
        rho = step(U, rho)
        if renorm_every and s % renorm_every == 0:
            rho = hermitize_normalize(rho)
        if observe is not None and record_every and s % record_every == 0:
            records.append(observe(rho))
    return rho, records


def evolve_exact(H: np.ndarray, rho0: np.ndarray, t: float) -> np.ndarray:
    """rho(t) = W rho0 W^dag with W = exp(-i H t) (eigendecomposition)."""
    W = propagator(H, t)
    return W @ rho0 @ W.conj().T


class SectorPropagator:
    """Per-excitation-sector eigendecomposition of H for pure-state evolution.

    H is block diagonal over the sectors of N_exc = a^dag a + sum_i s_i^+ s_i^-.
    Each block is diagonalised once; psi(t) = sum_k V_k e^{-i lam_k t} V_k^T psi0_k.
    """

    def __init__(self, n, c, g, omega_a, omega_c=1.0):
        self.n, self.c = n, c
        Hs = model.hamiltonian_sparse(n, c, g, omega_a, omega_c)
        self.N = Hs.shape[0]
        self.blocks = []
        for k, idx in model.sectors(n, c).items():
            Hk = Hs[idx][:, idx].toarray()
            lam, V = np.linalg.eigh(Hk)
            self.blocks.append((k, idx, lam, V))

    def psi(self, psi0: np.ndarray, t: float) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.complex128)
        for _, idx, lam, V in self.blocks:
            x = psi0[idx]
            if not np.any(x):
                continue
            out[idx] = V @ (np.exp(-1j * lam * t) * (V.T @ x))
        return out


def evolve_sectors(n, c, g, omega_a, psi0, times, omega_c=1.0):
    """psi(t) for each t in times via the sector route."""
    P = SectorPropagator(n, c, g, omega_a, omega_c)
    return [P.psi(psi0, t) for t in times]


def evolve_bruteforce(n, c, g, omega_a, psi0, dt, steps, omega_c=1.0):
    """State-vector stepping with scipy.linalg.expm of the dense Kronecker H.
    Returns the list [psi_0, psi_1, ..., psi_steps]."""
    H = model.hamiltonian(n, c, g, omega_a, omega_c)
    U = sla.expm(-1j * dt * H)
    psi = np.array(psi0, dtype=np.complex128)
    out = [psi]
    for _ in range(steps):
        psi = U @ psi
        out.append(psi)
    return out


def taylor_series(A: np.ndarray, kmax: int = 10) -> np.ndarray:
    """sum_{k=0}^{kmax} A^k / k!, powers as right-nested products A (A (... A))."""
    N = A.shape[0]
    out = np.eye(N, dtype=np.complex128)
    P = np.eye(N, dtype=np.complex128)
    for k in range(1, kmax + 1):
        P = A @ P                      # A^k = A (A^{k-1})
        out = out + P / math.factorial(k)
    return out


def taylor_factors(H: np.ndarray, dt: float, kmax: int = 10):
    """Eq. (10): L = sum_k (-i H dt)^k / k!;  Eq. (11): R = sum_k (+i H dt)^k / k!."""
    L = taylor_series(-1j * dt * H.astype(np.complex128), kmax)
    R = taylor_series(+1j * dt * H.astype(np.complex128), kmax)
    return L, R


def taylor_step(L: np.ndarray, R: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """Eq. (12) with Eq. (9b): Cannon^3(L, rho, R) = L (rho R)."""
    return L @ (rho @ R)
