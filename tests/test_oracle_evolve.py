"""Pins of the oracle's evolution (Eq. (6)), readouts (Eq. (13)) and the
truncated Taylor factors (Eq. (10)-(11)) against closed forms, invariants and
independent routes."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import tcm_inputs as ti
from oracle import evolve, model, observables as obs, renorm


@pytest.mark.parametrize("m", [0, 1, 3])
def test_jc_resonant_closed_form(m):
    """n=1 on resonance, psi0 = |m>|e>:  P_e(t) = cos^2(g sqrt(m+1) t)."""
    g, c, dt, steps = 0.02, m + 2, 0.37, 60
    n = 1
    H = model.hamiltonian(n, c, [g], [1.0])
    U = evolve.propagator(H, dt)
    rho0 = np.outer(ti.basis_state(n, c, m, [1]), ti.basis_state(n, c, m, [1]))
    _, rec = evolve.evolve_dense(U, rho0, steps, 1, lambda r: obs.excitation_total(r, n, c))
    t = dt * np.arange(steps + 1)
    assert np.max(np.abs(np.array(rec) - np.cos(g * math.sqrt(m + 1) * t) ** 2)) < 1e-12


@pytest.mark.parametrize("m,delta", [(0, 0.011), (2, -0.03)])
def test_jc_detuned_closed_form(m, delta):
    """P_e(t) = 1 - (4 g^2 (m+1) / W^2) sin^2(W t / 2),  W = sqrt(D^2 + 4 g^2 (m+1)),
    D = w_a - w_c."""
    g, c, dt, steps = 0.02, m + 1, 0.5, 80
    H = model.hamiltonian(1, c, [g], [1.0 + delta])
    U = evolve.propagator(H, dt)
    psi0 = ti.basis_state(1, c, m, [1])
    _, rec = evolve.evolve_dense(U, np.outer(psi0, psi0), steps, 1,
                                 lambda r: obs.excitation_total(r, 1, c))
    t = dt * np.arange(steps + 1)
    W = math.sqrt(delta ** 2 + 4 * g * g * (m + 1))
    pe = 1 - (4 * g * g * (m + 1) / W ** 2) * np.sin(W * t / 2) ** 2
    assert np.max(np.abs(np.array(rec) - pe)) < 1e-12


def test_collective_rabi():
    """psi0 = |1 photon>|all ground>, resonant, unequal g: the photon couples
    to the bright state with g_eff = sqrt(sum g_i^2) (g sqrt(n) for equal g):
    <a^dag a> = cos^2(g_eff t), sum p_i = sin^2(g_eff t),
    p_i = (g_i^2 / g_eff^2) sin^2(g_eff t)."""
    n, c, dt, steps = 4, 2, 0.8, 50
    inst = ti.random_model(n, c, 11)
    g = inst.g
    H = model.hamiltonian(n, c, g, np.ones(n))
    U = evolve.propagator(H, dt)
    psi0 = ti.basis_state(n, c, 1, [0] * n)
    geff = math.sqrt(float(np.sum(g ** 2)))
    rho = np.outer(psi0, psi0)
    for s in range(steps + 1):
        t = s * dt
        assert abs(obs.photon_mean(rho, n, c) - math.cos(geff * t) ** 2) < 1e-12
        assert abs(obs.excitation_total(rho, n, c) - math.sin(geff * t) ** 2) < 1e-12
        assert np.max(np.abs(obs.atom_populations(rho, n, c)
                             - g ** 2 / geff ** 2 * math.sin(geff * t) ** 2)) < 1e-12
        rho = evolve.step(U, rho)


def dicke_chain(n, c, g, m0=0):
    """Equal-g chain of |m, D_{n-m}> states starting from |0>|1^n>: the coupling
    between |m, D_j> and |m+1, D_{j-1}> (j = n - m) is g sqrt(m+1) sqrt(j (n-j+1)),
    i.e. g (m+1) sqrt(n-m); truncated at m = min(n, c)."""
    mmax = min(n, c)
    K = mmax + 1
    Hc = np.zeros((K, K))
    for m in range(mmax):
        Hc[m, m + 1] = Hc[m + 1, m] = g * (m + 1) * math.sqrt(n - m)
    return Hc


@pytest.mark.parametrize("n,c", [(3, 3), (4, 2), (5, 5)])
def test_equal_g_dicke_chain(n, c):
    """Equal g, resonant, psi0 = |0>|1^n>: the dynamics stay in the symmetric
    chain, so P(m photons) = |chain amplitude m|^2 and the total excitation is
    sum_m (n - m) |a_m|^2 (the common energy n w only adds a phase)."""
    g, dt, steps = 0.01, 0.7, 120
    H = model.hamiltonian(n, c, [g] * n, [1.0] * n)
    U = evolve.propagator(H, dt)
    psi0 = ti.basis_state(n, c, 0, [1] * n)
    Hc = dicke_chain(n, c, g)
    Uc = sla.expm(-1j * dt * Hc)
    a = np.zeros(Hc.shape[0], dtype=complex)
    a[0] = 1
    rho = np.outer(psi0, psi0).astype(complex)
    for s in range(steps + 1):
        pm = np.abs(a) ** 2
        tot = float(np.sum((n - np.arange(len(a))) * pm))
        assert abs(obs.excitation_total(rho, n, c) - tot) < 1e-12
        assert np.max(np.abs(obs.photon_state_probability(rho, n, c) - pm)) < 1e-12
        # with equal g the two readings of Eq. (13) coincide
        assert np.max(np.abs(obs.dicke_probability(rho, n, c) - pm)) < 1e-12
        rho = evolve.step(U, rho)
        a = Uc @ a


def test_routes_agree_and_invariants():
    """Dense stepping, exact eigendecomposition, the sector route and
    brute-force state-vector stepping (scipy expm) agree; trace, purity,
    Hermiticity and the excitation distribution P_k are conserved."""
    n, c, dt, steps = 3, 3, 0.05, 40
    inst = ti.random_model(n, c, 21, state="gaussian")
    H = model.hamiltonian(n, c, inst.g, inst.omega_a)
    U = evolve.propagator(H, dt)
    rho0 = inst.rho0()
    Pk0 = obs.excitation_distribution(rho0, n, c)
    rho = rho0
    bf = evolve.evolve_bruteforce(n, c, inst.g, inst.omega_a, inst.psi0, dt, steps)
    sec = evolve.SectorPropagator(n, c, inst.g, inst.omega_a)
    for s in range(1, steps + 1):
        rho = evolve.step(U, rho)
        if s % 10 == 0:
            t = s * dt
            ex = evolve.evolve_exact(H, rho0, t)
            psi_s = sec.psi(inst.psi0, t)
            assert np.max(np.abs(rho - ex)) < 1e-12
            assert np.max(np.abs(rho - np.outer(bf[s], bf[s].conj()))) < 1e-12
            assert np.max(np.abs(rho - np.outer(psi_s, psi_s.conj()))) < 1e-12
            inv = obs.invariants(rho)
            assert abs(inv["trace_re"] - 1) < 1e-13 and abs(inv["trace_im"]) < 1e-13
            assert abs(inv["purity"] - 1) < 1e-12
            assert inv["herm_err"] < 1e-14
            assert np.max(np.abs(obs.excitation_distribution(rho, n, c) - Pk0)) < 1e-13


def test_reversibility():
    n, c = 2, 3
    inst = ti.random_model(n, c, 5)
    U = evolve.propagator(model.hamiltonian(n, c, inst.g, inst.omega_a), 0.3)
    rho0 = inst.rho0()
    rho = rho0
    for _ in range(25):
        rho = evolve.step(U, rho)
    for _ in range(25):
        rho = evolve.step(U.conj().T, rho)
    assert np.max(np.abs(rho - rho0)) < 1e-13


def test_permutation_covariance():
    """Relabelling the atoms (g_i, delta_i and the state's qubit order) permutes p_i."""
    n, c, dt = 3, 2, 0.4
    rng = np.random.default_rng(3)
    g = np.array([0.011, 0.017, 0.006])
    w = 1 + np.array([0.002, -0.004, 0.001])
    qs = [np.array([0.6, 0.8]), np.array([1.0, 0.0]), np.array([0.0, 1.0])]
    perm = [2, 0, 1]
    psi_a = ti.product_state(n, c, 1, qs)
    psi_b = ti.product_state(n, c, 1, [qs[p] for p in perm])
    Ha = model.hamiltonian(n, c, g, w)
    Hb = model.hamiltonian(n, c, g[perm], w[perm])
    ra = evolve.evolve_exact(Ha, np.outer(psi_a, psi_a.conj()), 30 * dt)
    rb = evolve.evolve_exact(Hb, np.outer(psi_b, psi_b.conj()), 30 * dt)
    pa = obs.atom_populations(ra, n, c)
    pb = obs.atom_populations(rb, n, c)
    assert np.max(np.abs(pa[perm] - pb)) < 1e-13


def test_sector_readout_basis_state():
    """On a basis state the readouts are one-hot."""
    n, c = 3, 4
    psi = ti.basis_state(n, c, 2, [1, 0, 1])
    rho = np.outer(psi, psi)
    assert obs.excitation_total(rho, n, c) == 2
    assert np.array_equal(obs.atom_populations(rho, n, c), [1, 0, 1])
    assert np.array_equal(obs.photon_distribution(rho, n, c), [0, 0, 1, 0, 0])
    assert obs.excitation_mean(rho, n, c) == 4
    assert obs.photon_state_probability(rho, n, c)[1] == 0  # needs n-m = 2 excited with m=1
    psi = ti.basis_state(n, c, 1, [1, 0, 1])
    assert obs.photon_state_probability(np.outer(psi, psi), n, c)[1] == 1


@pytest.mark.parametrize("dt", [0.01, 0.05])
def test_taylor10_remainder_bound(dt):
    """Eq. (10): the truncated series differs from exp(-i H dt) by at most the
    tail sum_{k>10} ||A||^k / k! <= ||A||^11 / 11! e^||A||, A = -i H dt."""
    inst = ti.random_model(3, 3, 31)
    H = model.hamiltonian(3, 3, inst.g, inst.omega_a)
    L, R = evolve.taylor_factors(H, dt)
    E = sla.expm(-1j * dt * H)
    a = np.linalg.norm(H, 2) * dt
    bound = a ** 11 / math.factorial(11) * math.exp(a)
    assert np.linalg.norm(L - E, 2) <= bound + 1e-14
    # Eq. (11) is the adjoint of Eq. (10) for Hermitian H
    assert np.max(np.abs(R - L.conj().T)) < 1e-15
    # one step of Eq. (12) matches Eq. (6) within the same bound
    rho = inst.rho0()
    assert np.max(np.abs(evolve.taylor_step(L, R, rho) - E @ rho @ E.conj().T)) <= 3 * bound + 1e-14


def test_taylor10_large_norm_error_is_visible():
    """With ||H dt|| ~ 0.9 (the N=5120 workload's scale) ten terms leave an
    error far above 1e-10 per step: Eq. (10) alone cannot meet an FP64 contract."""
    H = np.diag(np.linspace(0, 18, 40))
    L, _ = evolve.taylor_factors(H, 0.05)
    E = sla.expm(-1j * 0.05 * H)
    err = np.max(np.abs(L - E))
    assert 1e-9 < err < 1e-7


def test_renorm():
    rng = np.random.default_rng(0)
    rho = ti.random_density(12, 3, rank=2) * 1.37
    rho = rho + 1e-3 * (rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)))
    out = renorm.hermitize_normalize(rho)
    assert np.array_equal(out, out.conj().T)
    assert abs(np.trace(out).real - 1) < 1e-15
    good = ti.random_density(12, 4)
    good = 0.5 * (good + good.conj().T)
    assert np.max(np.abs(renorm.hermitize_normalize(good) - good)) < 1e-15
