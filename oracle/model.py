"""Tavis-Cummings Hamiltonian, written out from its operator definition.

Sec. II, Eq. (4): with hbar = 1,
    H = w_c a^dag a + sum_i [ w_a,i s_i^+ s_i^- + g_i (a^dag s_i^- + a s_i^+) ].
The paper writes sigma_i for the relaxation operator (s^-) and sigma_i^dag for
excitation (s^+), a single cavity frequency w = w_a = w_c, and a per-atom
photon qubit in Eq. (1) that it then drops (Eq. (2)).  Readings taken here:
  * one bosonic cavity mode with photon cutoff c, a = sum_{m=1..c} sqrt(m)|m-1><m|
    (so a^dag|c> = 0 and the truncated H stays Hermitian);
  * per-atom frequencies w_a,i = 1 + delta_i (delta_i = 0 is the paper's
    resonance);
  * real couplings g_i, so H is real symmetric;
  * photon-major Kronecker order |m> (x) |l_1> (x) ... (x) |l_n>, atom 1 most
    significant, atom basis (|ground>, |excited>).

The matrix is assembled with Kronecker products of the single-site operators
(scipy.sparse.kron for the large sizes), which is independent of any
bit-index formula.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Single-atom operators in the basis (|ground>, |excited>).
SIGMA_MINUS = np.array([[0.0, 1.0], [0.0, 0.0]])   # |g><e|
SIGMA_PLUS = SIGMA_MINUS.T.copy()                   # |e><g|
NUM_ATOM = SIGMA_PLUS @ SIGMA_MINUS                 # |e><e|


def annihilation(c: int) -> np.ndarray:
    """Truncated cavity annihilation operator on photon numbers 0..c."""
    a = np.zeros((c + 1, c + 1))
    for m in range(1, c + 1):
        a[m - 1, m] = np.sqrt(m)
    return a


def number_operator(c: int) -> np.ndarray:
    """a^dag a on photon numbers 0..c: diag(0, 1, ..., c).  Written as its
    eigen-definition (a^dag a |m> = m |m>) so the diagonal is exact rather than
    the rounded products sqrt(m) * sqrt(m)."""
    return np.diag(np.arange(c + 1, dtype=np.float64))


def _embed(op_photon, atom_ops, n):
    """op_photon (x) A_1 (x) ... (x) A_n with A_i = atom_ops.get(i, I2), sparse."""
    out = sp.csr_matrix(op_photon)
    for i in range(n):
        A = atom_ops.get(i, np.eye(2))
        out = sp.kron(out, sp.csr_matrix(A), format="csr")
    return out


def hamiltonian_sparse(n: int, c: int, g, omega_a, omega_c: float = 1.0):
    """Eq. (4) with cutoff c and per-atom frequencies, as a scipy CSR matrix."""
    g = np.asarray(g, dtype=np.float64)
    omega_a = np.asarray(omega_a, dtype=np.float64)
    a = annihilation(c)
    ad = a.T.copy()
    Ip = np.eye(c + 1)
    H = omega_c * _embed(number_operator(c), {}, n)
    for i in range(n):
        H = H + omega_a[i] * _embed(Ip, {i: NUM_ATOM}, n)
        H = H + g[i] * (_embed(ad, {i: SIGMA_MINUS}, n)
                        + _embed(a, {i: SIGMA_PLUS}, n))
    return H.tocsr()


def hamiltonian(n: int, c: int, g, omega_a, omega_c: float = 1.0) -> np.ndarray:
    """Dense real FP64 Hamiltonian (N x N), N = (c+1) 2^n."""
    return hamiltonian_sparse(n, c, g, omega_a, omega_c).toarray()


def derivative_operators(n: int, c: int):
    """dH/dg_i = a^dag s_i^- + a s_i^+  and  dH/ddelta_i = s_i^+ s_i^-  (sparse)."""
    a = annihilation(c)
    ad = a.T.copy()
    Ip = np.eye(c + 1)
    dg = [(_embed(ad, {i: SIGMA_MINUS}, n) + _embed(a, {i: SIGMA_PLUS}, n)).tocsr()
          for i in range(n)]
    dd = [_embed(Ip, {i: NUM_ATOM}, n).tocsr() for i in range(n)]
    return dg, dd


# --- diagonal operators (photon number, atom excitation) via Kronecker too ---

def photon_number_diag(n: int, c: int) -> np.ndarray:
    """Diagonal of a^dag a."""
    return _embed(number_operator(c), {}, n).diagonal().real.copy()


def atom_excitation_diag(n: int, c: int, i: int) -> np.ndarray:
    """Diagonal of s_i^+ s_i^- (atom i, 0-based)."""
    return _embed(np.eye(c + 1), {i: NUM_ATOM}, n).diagonal().real.copy()


def total_excitation_diag(n: int, c: int) -> np.ndarray:
    """Diagonal of N_exc = a^dag a + sum_i s_i^+ s_i^- (conserved by Eq. (4))."""
    out = photon_number_diag(n, c)
    for i in range(n):
        out = out + atom_excitation_diag(n, c, i)
    return out


def sectors(n: int, c: int):
    """Basis indices grouped by total excitation k = m + |l| (H is block
    diagonal in k because N_exc commutes with Eq. (4))."""
    kdiag = np.rint(total_excitation_diag(n, c)).astype(np.int64)
    return {int(k): np.nonzero(kdiag == k)[0] for k in np.unique(kdiag)}


def paper_model_hamiltonian(n: int, g, omega_a, omega_c: float = 1.0) -> np.ndarray:
    """The paper's atom-only model (Sec. II, Eq. (2) with the Hamiltonian of
    Eq. (4)): the 2^n atom patterns l (atom i on bit n - 1 - i, 1 = excited),
    each carrying the n - |l| photons that the all-excited start (Sec. IV)
    leaves.  Written out element by element on those 2^n states, ordered by
    the integer value of l:
      H[l][l]   = w_c (n - |l|) + sum_i w_a,i l_i
      H[l'][l]  = H[l][l'] = g_i sqrt(n - |l| + 1)  for l_i = 1, l' = l - e_i
    (a^dag s_i^- takes |m, l> to sqrt(m + 1) |m + 1, l - e_i>, m = n - |l|)."""
    g = np.asarray(g, dtype=np.float64)
    omega_a = np.asarray(omega_a, dtype=np.float64)
    D = 1 << n
    H = np.zeros((D, D))
    for l in range(D):
        bits = [(l >> (n - 1 - i)) & 1 for i in range(n)]
        m = n - sum(bits)
        H[l, l] = omega_c * m + sum(omega_a[i] for i in range(n) if bits[i])
        for i in range(n):
            if bits[i]:
                lp = l ^ (1 << (n - 1 - i))
                H[lp, l] = H[l, lp] = g[i] * np.sqrt(m + 1)
    return H
