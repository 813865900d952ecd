"""Readouts of the density matrix.

Every population below is a diagonal sum  <O> = sum_s O_ss rho_ss  for a
diagonal operator O, which is the definition of the expectation Tr(O rho).

  excitation_total   sum_i <s_i^+ s_i^->, the per-step excited-atom
                     population of the paper's Sec. IV.A runs
  atom_populations   p_i = <s_i^+ s_i^->
  photon_distribution P(m) = prob(m photons)
  photon_state_probability  probability of the paper's {m> state, Eq. (13)
                     (sector reading: m photons AND n - m excited atoms)
  dicke_probability  the other reading of Eq. (13): overlap with the
                     normalised symmetric (Dicke) vector with m photons
  excitation_distribution P_k = prob(N_exc = k)
  invariants         Re/Im trace, purity sum |rho_ij|^2, max |rho - rho^dag|
"""
from __future__ import annotations

import numpy as np

from . import model


def diag_expect(rho: np.ndarray, odiag: np.ndarray) -> float:
    return float(np.sum(odiag * np.real(np.diagonal(rho))))


def excitation_total(rho, n, c) -> float:
    ops = sum(model.atom_excitation_diag(n, c, i) for i in range(n))
    return diag_expect(rho, ops)


def atom_populations(rho, n, c) -> np.ndarray:
    return np.array([diag_expect(rho, model.atom_excitation_diag(n, c, i))
                     for i in range(n)])


def photon_distribution(rho, n, c) -> np.ndarray:
    ph = np.rint(model.photon_number_diag(n, c)).astype(int)
    d = np.real(np.diagonal(rho))
    return np.array([float(np.sum(d[ph == m])) for m in range(c + 1)])


def photon_mean(rho, n, c) -> float:
    return diag_expect(rho, model.photon_number_diag(n, c))


def excitation_distribution(rho, n, c) -> np.ndarray:
    k = np.rint(model.total_excitation_diag(n, c)).astype(int)
    d = np.real(np.diagonal(rho))
    return np.array([float(np.sum(d[k == j])) for j in range(n + c + 1)])


def excitation_mean(rho, n, c) -> float:
    return diag_expect(rho, model.total_excitation_diag(n, c))


def photon_state_probability(rho, n, c) -> np.ndarray:
    """Eq. (13), sector reading: P({m>) = sum over basis states with m photons
    and exactly n - m excited atoms, for m = 0..min(n, c)."""
    ph = np.rint(model.photon_number_diag(n, c)).astype(int)
    ex = sum(model.atom_excitation_diag(n, c, i) for i in range(n))
    ex = np.rint(ex).astype(int)
    d = np.real(np.diagonal(rho))
    return np.array([float(np.sum(d[(ph == m) & (ex == n - m)]))
                     for m in range(min(n, c) + 1)])


def dicke_probability(rho, n, c) -> np.ndarray:
    """Eq. (13), symmetric reading: <v_m| rho |v_m> with v_m the equal-weight
    normalised sum of the basis states with m photons and n - m excitations."""
    ph = np.rint(model.photon_number_diag(n, c)).astype(int)
    ex = np.rint(sum(model.atom_excitation_diag(n, c, i) for i in range(n))).astype(int)
    out = []
    for m in range(min(n, c) + 1):
        v = ((ph == m) & (ex == n - m)).astype(np.float64)
        v /= np.linalg.norm(v)
        out.append(float(np.real(v @ rho @ v)))
    return np.array(out)


def invariants(rho) -> dict:
    tr = np.trace(rho)
    return {
        "trace_re": float(tr.real),
        "trace_im": float(tr.imag),
        "purity": float(np.sum(np.abs(rho) ** 2)),
        "herm_err": float(np.max(np.abs(rho - rho.conj().T))) if rho.size else 0.0,
    }


def psi_excitation_total(psi, n, c) -> float:
    ops = sum(model.atom_excitation_diag(n, c, i) for i in range(n))
    return float(np.sum(ops * np.abs(psi) ** 2))


def psi_photon_distribution(psi, n, c) -> np.ndarray:
    ph = np.rint(model.photon_number_diag(n, c)).astype(int)
    p = np.abs(psi) ** 2
    return np.array([float(np.sum(p[ph == m])) for m in range(c + 1)])
