"""The GPU stepper against closed forms of the model (no oracle in between):
Jaynes-Cummings Rabi oscillations (n = 1), the collective single-excitation
oscillation at g_eff = sqrt(sum g_i^2), the uncoupled c = 0 model (pure
phases) and the equal-g Dicke chain, in every precision and frame."""
import math

import numpy as np
import pytest
import torch

import tcm_inputs as ti

pytestmark = pytest.mark.gpu

tcm = pytest.importorskip("paper_2403_06937_amd")
from paper_2403_06937_amd import pipeline  # noqa: E402

MODES = [
    (tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB, torch.complex128, 1e-10),
    (tcm.TC_GEMM_F64, tcm.TC_FRAME_ROTATING, torch.complex128, 1e-10),
    (tcm.TC_GEMM_F32, tcm.TC_FRAME_ROTATING, torch.complex64, 2e-5),
    (tcm.TC_GEMM_SPLIT_BF16, tcm.TC_FRAME_ROTATING, torch.complex64, 2e-5),
]


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tcm.lib()


def run(inst, dt, steps, mode, frame, dtype, record_photons=False):
    m = pipeline.model_of(inst)
    _, U = pipeline.propagator(m, dt)
    rho = torch.from_numpy(inst.rho0()).to("cuda").to(dtype)
    pop, pd, _ = pipeline.evolve(m, U, rho, steps, dt, mode, frame, 0, 1,
                                 record_photons=record_photons)
    torch.cuda.synchronize()
    return (rho.cpu().numpy().astype(np.complex128), pop.cpu().numpy(),
            None if pd is None else pd.cpu().numpy())


@pytest.mark.parametrize("mode,frame,dtype,tol", MODES)
@pytest.mark.parametrize("m_photons,detuning", [(0, 0.0), (2, 0.0), (1, 0.03)])
def test_jaynes_cummings(mode, frame, dtype, tol, m_photons, detuning):
    """n = 1, start |m>|e>: P_e(t) = 1 - (4 g^2 (m+1) / W^2) sin^2(W t / 2) with
    W = sqrt(delta^2 + 4 g^2 (m+1)) (cos^2(g sqrt(m+1) t) on resonance), as
    long as the cutoff keeps |m+1> (c = 4 here)."""
    g, c, dt, steps = 0.05, 4, 0.1, 300
    inst = ti.Instance(n=1, c=c, g=np.array([g]), omega_a=np.array([1.0 + detuning]),
                       psi0=ti.basis_state(1, c, m_photons, [1]))
    _, pop, _ = run(inst, dt, steps, mode, frame, dtype)
    t = dt * np.arange(steps + 1)
    W = math.sqrt(detuning ** 2 + 4 * g * g * (m_photons + 1))
    ref = 1 - (4 * g * g * (m_photons + 1) / W ** 2) * np.sin(W * t / 2) ** 2
    assert np.max(np.abs(pop - ref)) < tol


@pytest.mark.parametrize("mode,frame,dtype,tol", MODES)
def test_collective_single_excitation(mode, frame, dtype, tol):
    """One photon, all atoms ground, uneven g_i, no detuning: the photon
    oscillates with the bright state at g_eff = sqrt(sum g_i^2):
    <a^dag a> = cos^2(g_eff t) and sum_i <s_i^+ s_i^-> = sin^2(g_eff t)."""
    n, c, dt, steps = 5, 2, 0.2, 250
    g = np.array([0.01, 0.02, 0.015, 0.005, 0.012])
    inst = ti.Instance(n=n, c=c, g=g, omega_a=np.ones(n), psi0=ti.basis_state(n, c, 1, [0] * n))
    _, pop, pd = run(inst, dt, steps, mode, frame, dtype, record_photons=True)
    t = dt * np.arange(steps + 1)
    geff = math.sqrt(float(np.sum(g * g)))
    assert np.max(np.abs(pop - np.sin(geff * t) ** 2)) < tol
    # P(m = 1), the one-photon probability (here only |1>|0...0> has a photon)
    assert np.max(np.abs(pd[:, 1] - np.cos(geff * t) ** 2)) < tol


@pytest.mark.parametrize("mode,frame,dtype,tol", MODES)
def test_uncoupled_model_is_pure_phase(mode, frame, dtype, tol):
    """c = 0 (no photons, H diagonal with energies sum_i w_i l_i): every entry
    of rho only turns by exp(-i (E_r - E_s) t)."""
    n, dt, steps = 6, 0.05, 120
    rng = np.random.default_rng(11)
    w = 1.0 + rng.normal(0, 0.01, n)
    inst = ti.Instance(n=n, c=0, g=np.full(n, 0.01), omega_a=w,
                       psi0=ti.gaussian_state(1 << n, rng))
    rho, pop, _ = run(inst, dt, steps, mode, frame, dtype)
    bits = (np.arange(1 << n)[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1
    E = bits @ w
    T = dt * steps
    rho0 = inst.rho0()
    ref = rho0 * np.exp(-1j * (E[:, None] - E[None, :]) * T)
    assert np.max(np.abs(rho - ref)) < tol
    assert np.max(np.abs(pop - pop[0])) < tol


@pytest.mark.parametrize("mode,frame,dtype,tol", MODES)
def test_equal_g_dicke_chain(mode, frame, dtype, tol):
    """Equal g, start |0>|1^n>: the state stays in the chain |m>|D_{n-m}> with
    couplings g (m+1) sqrt(n-m) (truncated at c); the excited-atom population
    follows the chain's own 4 x 4 evolution (n = 3, c = 3)."""
    n, c, g, dt, steps = 3, 3, 0.02, 0.1, 400
    inst = ti.Instance(n=n, c=c, g=np.full(n, g), omega_a=np.ones(n),
                       psi0=ti.basis_state(n, c, 0, [1] * n))
    _, pop, _ = run(inst, dt, steps, mode, frame, dtype)
    Hc = np.zeros((c + 1, c + 1))
    for mm in range(c):
        Hc[mm, mm + 1] = Hc[mm + 1, mm] = g * (mm + 1) * math.sqrt(n - mm)
    lam, V = np.linalg.eigh(Hc)
    t = dt * np.arange(steps + 1)
    amp = (V[None, :, :] * np.exp(-1j * lam[None, None, :] * t[:, None, None])) @ V[0]
    ref = np.abs(amp) ** 2 @ (n - np.arange(c + 1))
    assert np.max(np.abs(pop - ref)) < tol
