"""Pins of the oracle's Hamiltonian (Eq. (4) with cavity cutoff and detuning)
against constructions and closed forms that do not share its code."""
import math

import numpy as np
import pytest

import tcm_inputs as ti
from oracle import model

pytestmark = pytest.mark.filterwarnings("ignore")


def ket_hamiltonian(n, c, g, omega_a, omega_c=1.0):
    """Independent route: apply each term of Eq. (4) to every basis ket
    (m, l_1..l_n) and place <s'|H|s> with the index formula s = m 2^n + ..."""
    N = ti.hilbert_dim(n, c)
    H = np.zeros((N, N))
    for m in range(c + 1):
        for code in range(2 ** n):
            bits = [(code >> (n - 1 - i)) & 1 for i in range(n)]
            s = ti.basis_index(n, m, bits)
            H[s, s] += omega_c * m + sum(omega_a[i] * bits[i] for i in range(n))
            for i in range(n):
                # a^dag s_i^-: atom i excited -> ground, one more photon
                if bits[i] == 1 and m < c:
                    nb = list(bits)
                    nb[i] = 0
                    t = ti.basis_index(n, m + 1, nb)
                    H[t, s] += g[i] * math.sqrt(m + 1)
                # a s_i^+: atom i ground -> excited, one photon fewer
                if bits[i] == 0 and m > 0:
                    nb = list(bits)
                    nb[i] = 1
                    t = ti.basis_index(n, m - 1, nb)
                    H[t, s] += g[i] * math.sqrt(m)
    return H


@pytest.mark.parametrize("n,c,seed", [(1, 1, 0), (1, 4, 1), (2, 3, 2), (3, 3, 3), (4, 2, 4), (3, 0, 5)])
def test_kron_equals_ket_construction(n, c, seed):
    inst = ti.random_model(n, c, seed)
    H1 = model.hamiltonian(n, c, inst.g, inst.omega_a)
    H2 = ket_hamiltonian(n, c, inst.g, inst.omega_a)
    assert H1.shape == (ti.hilbert_dim(n, c),) * 2
    # diagonal sums are added in a different order: a few ulp of max |H|
    assert np.max(np.abs(H1 - H2)) <= 4 * np.finfo(float).eps * np.max(np.abs(H1))
    # real symmetric and the sparsity pattern is exactly the ket one
    assert np.array_equal(H1, H1.T)
    assert np.array_equal(H1 != 0, H2 != 0)


@pytest.mark.parametrize("c", [1, 3, 6])
@pytest.mark.parametrize("delta", [0.0, 0.013])
def test_jc_spectrum_closed_form(c, delta):
    """n = 1 (Jaynes-Cummings): each doublet {|m,e>, |m+1,g>} has eigenvalues
    (w_c(2m+1) + w_a)/2 +- sqrt(((w_a - w_c)/2)^2 + g^2 (m+1)); plus |0,g> at 0
    and the uncoupled top state |c,e> at w_c c + w_a."""
    g, wc, wa = 0.0173, 1.0, 1.0 + delta
    H = model.hamiltonian(1, c, [g], [wa], wc)
    ev = np.sort(np.linalg.eigvalsh(H))
    expect = [0.0, wc * c + wa]
    for m in range(c):
        mid = (wc * (2 * m + 1) + wa) / 2
        r = math.sqrt(((wa - wc) / 2) ** 2 + g * g * (m + 1))
        expect += [mid - r, mid + r]
    assert np.allclose(ev, np.sort(expect), atol=1e-14, rtol=0)


def test_sector_sizes_closed_form():
    """d_k = sum_{m=0}^{min(k,c)} C(n, k-m); n=11, c=5 gives the 17 sizes
    1, 12, 67, 232, 562, 1024, 1485, 1804, 1914, 1804, ... summing to 12288."""
    n, c = 11, 5
    secs = model.sectors(n, c)
    sizes = [len(secs[k]) for k in sorted(secs)]
    expect = [sum(math.comb(n, k - m) for m in range(0, min(k, c) + 1) if 0 <= k - m <= n)
              for k in range(n + c + 1)]
    assert sizes == expect
    assert sizes[:9] == [1, 12, 67, 232, 562, 1024, 1485, 1804, 1914]
    assert sum(sizes) == 12288


def test_excitation_number_commutes():
    inst = ti.random_model(3, 4, 7)
    H = model.hamiltonian(3, 4, inst.g, inst.omega_a)
    k = model.total_excitation_diag(3, 4)
    # [H, N_exc]_ij = H_ij (k_j - k_i): every nonzero entry joins equal k
    i, j = np.nonzero(H)
    assert np.all(k[i] == k[j])


def test_paper_2n_sector_embedding():
    """The paper's atom-only space (Eq. (2), N = 2^n) is the excitation-n sector
    when c >= n: it has exactly 2^n states and starts from |0 photons>|1..1>."""
    for n in (2, 3, 4):
        secs = model.sectors(n, n)
        assert len(secs[n]) == 2 ** n
        assert ti.basis_index(n, 0, [1] * n) in set(secs[n].tolist())


def test_c_zero_is_diagonal():
    inst = ti.random_model(3, 0, 9)
    H = model.hamiltonian(3, 0, inst.g, inst.omega_a)
    assert np.count_nonzero(H - np.diag(np.diagonal(H))) == 0


def test_paper_model_is_the_excitation_n_sector():
    """The paper's 2^n model written on atom patterns equals the excitation-n
    block of the (c >= n) Kronecker-built H, state for state (each pattern l
    is the basis state (n - |l|) 2^n + l); n = 1 is the Jaynes-Cummings 2 x 2
    block [[w_c, g], [g, w_a]] in the order (|1 photon, g>, |0, e>)."""
    for n, c, seed in [(1, 1, 0), (2, 2, 1), (3, 4, 2), (4, 4, 3), (5, 6, 4)]:
        inst = ti.random_model(n, c, seed)
        Hp = model.paper_model_hamiltonian(n, inst.g, inst.omega_a, 1.3)
        H = model.hamiltonian(n, c, inst.g, inst.omega_a, 1.3)
        idx = [(n - bin(l).count("1")) * (1 << n) + l for l in range(1 << n)]
        assert sorted(idx) == sorted(model.sectors(n, c)[n].tolist())
        assert np.max(np.abs(Hp - H[np.ix_(idx, idx)])) < 1e-15
    g, wa = 0.013, 1.02
    Hp = model.paper_model_hamiltonian(1, [g], [wa], 0.97)
    assert np.allclose(Hp, [[0.97, g], [g, wa]], rtol=0, atol=1e-17)


def test_paper_model_equal_g_dicke_chain():
    """Equal g at resonance: the all-excited start stays in the symmetric
    states |m>|D_{n-m}>, whose chain couplings are g (m + 1) sqrt(n - m); the
    chain's eigenvalues are eigenvalues of the paper's 2^n model."""
    n, g = 4, 0.02
    Hp = model.paper_model_hamiltonian(n, [g] * n, [1.0] * n, 1.0)
    chain = np.diag([float(n)] * (n + 1))
    for m in range(n):
        chain[m, m + 1] = chain[m + 1, m] = g * (m + 1) * np.sqrt(n - m)
    ev = np.linalg.eigvalsh(Hp)
    for lam in np.linalg.eigvalsh(chain):
        assert np.min(np.abs(ev - lam)) < 1e-14
