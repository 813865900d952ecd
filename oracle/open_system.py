"""Open-system stepping: the Lindblad term of Eq. (5), restored (test
infrastructure; only the tests, the smoke check and the benchmark's CPU
baseline may use it).

Sec. III.A writes the master equation i drho/dt = [H, rho] + i L(rho) and then
drops L(rho).  The paper names no jump operators; the reading taken here is
the standard Tavis-Cummings dissipation at zero temperature,

    L(rho) = kappa D[a] rho + gamma sum_i D[s_i^-] rho,
    D[A] rho = A rho A^dag - (A^dag A rho + rho A^dag A) / 2,

cavity leakage at rate kappa and spontaneous emission of every atom at rate
gamma (hbar = 1, so drho/dt = -i [H, rho] + L(rho)).

Plain definition (small N only): the Liouvillian as an N^2 x N^2 matrix on
row-major vec(rho), vec(A X B) = (A (x) B^T) vec(X), and
rho(t) = expm(t Liouvillian) vec(rho(0)).

The stepped method keeps Eq. (6) for the Hamiltonian part and follows each
unitary step by the exact dissipation over dt (Lie splitting, first order in
dt):  rho <- Diss_dt(U rho U^dag),  Diss_dt = exp(dt L).  The dissipators of
the cavity and of the atoms act on different factors of the Kronecker
product, so exp(dt L) is the composition of one amplitude-damping channel per
factor, each written with its Kraus operators:
  atom i:  K0 = |g><g| + sqrt(1 - p)|e><e|,  K1 = sqrt(p) |g><e|,
           p = 1 - exp(-gamma dt);
  cavity:  E_l = sum_{m >= l} sqrt(binom(m, l)) eta^{(m-l)/2} (1-eta)^{l/2} |m-l><m|,
           eta = exp(-kappa dt), l = 0..c
(a lowers the photon number, so the cutoff space is invariant and the channel
on it is the untruncated one restricted).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import model


def jump_operators(n: int, c: int, kappa: float, gamma: float):
    """[(rate, A)] for L: (kappa, a) and (gamma, s_i^-) for each atom, sparse."""
    ops = [(kappa, model._embed(model.annihilation(c), {}, n))]
    for i in range(n):
        ops.append((gamma, model._embed(np.eye(c + 1), {i: model.SIGMA_MINUS}, n)))
    return ops


def liouvillian(H: np.ndarray, jumps) -> np.ndarray:
    """Dense N^2 x N^2 generator of drho/dt = -i[H, rho] + sum_k r_k D[A_k] rho
    acting on the row-major vec(rho)."""
    N = H.shape[0]
    Id = np.eye(N)
    Lv = -1j * (np.kron(H, Id) - np.kron(Id, H.T))
    for r, A in jumps:
        if r == 0.0:
            continue
        A = A.toarray() if sp.issparse(A) else np.asarray(A)
        AdA = A.conj().T @ A
        Lv = Lv + r * (np.kron(A, A.conj()) - 0.5 * np.kron(AdA, Id) - 0.5 * np.kron(Id, AdA.T))
    return Lv


def evolve_lindblad_exact(rho0: np.ndarray, H: np.ndarray, jumps, t: float) -> np.ndarray:
    """rho(t) = expm(t Liouvillian) rho(0) (scipy's expm; N up to ~32)."""
    N = rho0.shape[0]
    v = sla.expm(t * liouvillian(H, jumps)) @ rho0.reshape(-1)
    return v.reshape(N, N)


def atom_kraus(n: int, c: int, i: int, p: float):
    """Kraus operators of the amplitude damping of atom i with probability p."""
    k0 = np.array([[1.0, 0.0], [0.0, math.sqrt(1.0 - p)]])
    k1 = math.sqrt(p) * model.SIGMA_MINUS
    return [model._embed(np.eye(c + 1), {i: k0}, n), model._embed(np.eye(c + 1), {i: k1}, n)]


def cavity_kraus(n: int, c: int, eta: float):
    """Kraus operators E_l (l = 0..c) of the cavity damping with eta = exp(-kappa dt)."""
    out = []
    for l in range(c + 1):
        E = np.zeros((c + 1, c + 1))
        for m in range(l, c + 1):
            E[m - l, m] = math.sqrt(math.comb(m, l)) * eta ** ((m - l) / 2) * (1 - eta) ** (l / 2)
        out.append(model._embed(E, {}, n))
    return out


def apply_channel(rho: np.ndarray, kraus) -> np.ndarray:
    """sum_k K rho K^dag with sparse K."""
    out = np.zeros_like(rho)
    for K in kraus:
        KR = K @ rho
        out += (K.conj() @ KR.T).T          # (K rho) K^dag = ((K^*) (K rho)^T)^T
    return out


def dissipation(rho: np.ndarray, n: int, c: int, kappa: float, gamma: float,
                dt: float) -> np.ndarray:
    """exp(dt L) rho: the cavity channel and one channel per atom."""
    if gamma != 0.0:
        p = 1.0 - math.exp(-gamma * dt)
        for i in range(n):
            rho = apply_channel(rho, atom_kraus(n, c, i, p))
    if kappa != 0.0:
        rho = apply_channel(rho, cavity_kraus(n, c, math.exp(-kappa * dt)))
    return rho


def evolve_open_split(rho0: np.ndarray, U: np.ndarray, n: int, c: int, kappa: float,
                      gamma: float, dt: float, steps: int, observe=None):
    """The stepped method: rho <- exp(dt L)(U rho U^dag), steps times.  observe
    (optional) is called on rho(0) and after each step; returns (rho, records)."""
    rho = np.array(rho0, dtype=np.complex128)
    Ud = U.conj().T
    rec = [observe(rho)] if observe else []
    for _ in range(steps):
        rho = U @ rho @ Ud
        rho = dissipation(rho, n, c, kappa, gamma, dt)
        if observe:
            rec.append(observe(rho))
    return rho, rec
