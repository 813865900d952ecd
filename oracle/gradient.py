"""Gradient of the final atomic excitation with respect to g_i and delta_i.

Loss L = Tr(O rho(T)),  O = sum_i s_i^+ s_i^-,  rho(T) = W rho0 W^dag with
W = exp(-i H T), T = steps * dt (the S-fold product of the per-step
propagator of Eq. (6) is exactly W).  Parameters: the couplings g_i and the
detunings delta_i (w_a,i = 1 + delta_i) of Eq. (4).

Two independent routes:
  * Daleckii-Krein: with H = V diag(lam) V^T,
        dW/dtheta = V (F o (V^T dH/dtheta V)) V^T,
        F_kl = -i T exp(-i (lam_k + lam_l) T / 2) sinc((lam_k - lam_l) T / 2),
    the divided difference of exp(-i lam T) written in a form that stays
    exact at degenerate eigenvalues; then dL/dtheta = 2 Re Tr(O dW rho0 W^dag).
  * central finite differences of L with an absolute step h.
"""
from __future__ import annotations

import numpy as np

from . import model
from .evolve import propagator


def _sinc(x):
    return np.sinc(x / np.pi)     # numpy's sinc is sin(pi x)/(pi x)


def excitation_operator(n, c) -> np.ndarray:
    return sum(model.atom_excitation_diag(n, c, i) for i in range(n))


def support_indices(n, c, rho0) -> np.ndarray:
    """Union of the excitation sectors that carry rho0.  H, dH/dg_i, dH/ddelta_i
    and O all commute with N_exc, so restricting every operator to these rows
    and columns leaves L and its gradient unchanged (exact, not approximate)."""
    d = np.abs(np.asarray(rho0))
    live = np.nonzero((d.sum(axis=0) + d.sum(axis=1)) > 0)[0]
    keep = []
    for _, idx in model.sectors(n, c).items():
        if np.intersect1d(idx, live).size:
            keep.append(idx)
    return np.sort(np.concatenate(keep)) if keep else np.zeros(0, dtype=np.int64)


def _restricted(n, c, g, delta, rho0, omega_c, restrict):
    Hs = model.hamiltonian_sparse(n, c, g, 1.0 + np.asarray(delta), omega_c)
    O = excitation_operator(n, c)
    if restrict:
        idx = support_indices(n, c, rho0)
    else:
        idx = np.arange(Hs.shape[0])
    H = Hs[idx][:, idx].toarray()
    return idx, H, O[idx], np.asarray(rho0)[np.ix_(idx, idx)]


def loss(n, c, g, delta, rho0, T, omega_c=1.0, restrict=True) -> float:
    _, H, O, r0 = _restricted(n, c, g, delta, rho0, omega_c, restrict)
    W = propagator(H, T)
    rho = W @ r0 @ W.conj().T
    return float(np.sum(O * np.real(np.diagonal(rho))))


def grad_daleckii_krein(n, c, g, delta, rho0, T, omega_c=1.0, restrict=True):
    """Returns (loss, dL/dg [n], dL/ddelta [n])."""
    idx, H, O, r0 = _restricted(n, c, g, delta, rho0, omega_c, restrict)
    lam, V = np.linalg.eigh(H)
    W = (V * np.exp(-1j * lam * T)) @ V.T
    rho_T = W @ r0 @ W.conj().T
    L = float(np.sum(O * np.real(np.diagonal(rho_T))))
    F = (-1j * T * np.exp(-0.5j * np.add.outer(lam, lam) * T)
         * _sinc(0.5 * np.subtract.outer(lam, lam) * T))
    # Tr(O dW rho0 W^dag) = sum_ij O_i [dW]_ij [rho0 W^dag]_ji
    B = r0 @ W.conj().T
    dgs, dds = model.derivative_operators(n, c)

    def one(dH):
        dH = dH[idx][:, idx].toarray()
        dHe = V.T @ (dH @ V)
        dW = V @ (F * dHe) @ V.T
        return 2.0 * float(np.real(np.sum(O[:, None] * dW * B.T)))

    gg = np.array([one(d) for d in dgs])
    gd = np.array([one(d) for d in dds])
    return L, gg, gd


def grad_fd(n, c, g, delta, rho0, T, h=1e-6, omega_c=1.0, restrict=True):
    """Central finite differences with absolute step h; returns (dL/dg, dL/ddelta)."""
    g = np.asarray(g, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    gg = np.zeros_like(g)
    gd = np.zeros_like(delta)
    for i in range(len(g)):
        e = np.zeros_like(g)
        e[i] = h
        gg[i] = (loss(n, c, g + e, delta, rho0, T, omega_c, restrict)
                 - loss(n, c, g - e, delta, rho0, T, omega_c, restrict)) / (2 * h)
        gd[i] = (loss(n, c, g, delta + e, rho0, T, omega_c, restrict)
                 - loss(n, c, g, delta - e, rho0, T, omega_c, restrict)) / (2 * h)
    return gg, gd
