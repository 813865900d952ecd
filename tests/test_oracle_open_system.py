"""Pins of the open-system oracle (the Lindblad term of Eq. (5) restored):
the Kraus channels against the exponential of the dissipative Liouvillian,
pure-decay closed forms, first-order convergence of the split step to the
exact master-equation solution, and the density-matrix invariants."""
import math

import numpy as np
import pytest

import tcm_inputs as ti
from oracle import evolve as oev
from oracle import model as omodel
from oracle import open_system as oos


def _excitations(rho, n, c):
    return float(np.real(np.sum(np.diag(rho) * sum(omodel.atom_excitation_diag(n, c, i)
                                                   for i in range(n)))))


def _photons(rho, n, c):
    return float(np.real(np.sum(np.diag(rho) * omodel.photon_number_diag(n, c))))


@pytest.mark.parametrize("n,c,kappa,gamma,dt", [(2, 2, 0.3, 0.0, 0.4), (2, 2, 0.0, 0.2, 0.4),
                                                (2, 3, 0.25, 0.15, 0.7), (1, 4, 1.3, 0.6, 0.9)])
def test_channels_equal_exponential_of_dissipator(n, c, kappa, gamma, dt):
    """exp(dt L) with L built from D[A] = A.A^dag - {A^dag A, .}/2 (no Hamiltonian)
    equals the composition of the Kraus channels, on a random mixed state."""
    N = (c + 1) << n
    rho = ti.random_density(N, 3, rank=3)
    jumps = oos.jump_operators(n, c, kappa, gamma)
    ref = oos.evolve_lindblad_exact(rho, np.zeros((N, N)), jumps, dt)
    got = oos.dissipation(rho, n, c, kappa, gamma, dt)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_liouvillian_hamiltonian_part_is_the_unitary_step():
    """No jumps: expm(t L) vec(rho) = W rho W^dag with W = exp(-i H t)."""
    inst = ti.random_model(2, 2, 41, state="gaussian")
    H = omodel.hamiltonian(inst.n, inst.c, inst.g, inst.omega_a)
    rho = inst.rho0()
    W = oev.propagator(H, 3.0)
    got = oos.evolve_lindblad_exact(rho, H, [], 3.0)
    assert np.max(np.abs(got - W @ rho @ W.conj().T)) < 1e-13


@pytest.mark.parametrize("m0", [1, 3])
def test_pure_decay_closed_forms(m0):
    """g = 0: the dissipation commutes with the free evolution, so the split
    step is exact: <a^dag a>(t) = m0 exp(-kappa t), every excited atom decays as
    exp(-gamma t)."""
    n, c, kappa, gamma, dt, steps = 3, 4, 0.07, 0.03, 0.25, 80
    g = np.zeros(n)
    wa = np.array([1.0, 1.01, 0.99])
    H = omodel.hamiltonian(n, c, g, wa)
    U = oev.propagator(H, dt)
    psi0 = ti.basis_state(n, c, m0, [1, 0, 1])
    rho0 = np.outer(psi0, psi0.conj())
    _, rec = oos.evolve_open_split(rho0, U, n, c, kappa, gamma, dt, steps,
                                   lambda r: (_photons(r, n, c), _excitations(r, n, c)))
    t = dt * np.arange(steps + 1)
    ph = np.array([x[0] for x in rec])
    ex = np.array([x[1] for x in rec])
    assert np.max(np.abs(ph - m0 * np.exp(-kappa * t))) < 1e-13
    assert np.max(np.abs(ex - 2 * np.exp(-gamma * t))) < 1e-13


def test_split_step_converges_first_order():
    """Jaynes-Cummings with loss: the split step approaches the exact
    master-equation solution with error proportional to dt."""
    n, c, g, kappa, gamma, T = 1, 3, 0.3, 0.2, 0.1, 4.0
    H = omodel.hamiltonian(n, c, [g], [1.0])
    jumps = oos.jump_operators(n, c, kappa, gamma)
    psi0 = ti.basis_state(n, c, 2, [1])
    rho0 = np.outer(psi0, psi0.conj())
    exact = oos.evolve_lindblad_exact(rho0, H, jumps, T)
    errs = []
    for steps in (40, 80, 160):
        dt = T / steps
        rho, _ = oos.evolve_open_split(rho0, oev.propagator(H, dt), n, c, kappa, gamma, dt, steps)
        errs.append(float(np.max(np.abs(rho - exact))))
    assert errs[0] < 1e-2
    for a, b in zip(errs, errs[1:]):
        assert 1.8 < a / b < 2.2


def test_invariants_and_ground_state_limit():
    """Trace one, Hermitian, positive semidefinite after every step; at long
    times everything relaxes into |0>|0...0>."""
    inst = ti.random_model(3, 2, 43, state="gaussian")
    n, c = inst.n, inst.c
    H = omodel.hamiltonian(n, c, inst.g * 20, inst.omega_a)
    dt = 0.5
    U = oev.propagator(H, dt)
    worst = [0.0, 0.0, 0.0]

    def obs(r):
        worst[0] = max(worst[0], abs(np.trace(r) - 1))
        worst[1] = max(worst[1], float(np.max(np.abs(r - r.conj().T))))
        worst[2] = min(worst[2], float(np.min(np.linalg.eigvalsh(0.5 * (r + r.conj().T)))))
        return None

    rho, _ = oos.evolve_open_split(inst.rho0(), U, n, c, 0.4, 0.3, dt, 120, obs)
    assert worst[0] < 1e-13 and worst[1] < 1e-14 and worst[2] > -1e-14
    assert abs(rho[0, 0] - 1) < 1e-6


def test_no_dissipation_is_the_unitary_step():
    inst = ti.random_model(3, 2, 44, state="gaussian")
    H = omodel.hamiltonian(inst.n, inst.c, inst.g, inst.omega_a)
    U = oev.propagator(H, 0.3)
    rho, _ = oos.evolve_open_split(inst.rho0(), U, inst.n, inst.c, 0.0, 0.0, 0.3, 25)
    ref, _ = oev.evolve_dense(U, inst.rho0(), 25)
    assert np.max(np.abs(rho - ref)) < 1e-14
