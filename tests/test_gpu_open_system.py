"""The open-system step (Lindblad term of Eq. (5), cavity leakage kappa and
atomic emission gamma) on the GPU: against the oracle's split step in every
precision and frame, against the pure-decay closed forms at the full N = 12288
shape, batched against single runs, and the invariants."""
import numpy as np
import pytest
import torch

import tcm_inputs as ti
from oracle import evolve as oev
from oracle import model as omodel
from oracle import open_system as oos

pytestmark = pytest.mark.gpu

tcm = pytest.importorskip("paper_2403_06937_amd")
from paper_2403_06937_amd import pipeline  # noqa: E402

MODES = [
    (tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB, torch.complex128, 1e-12),
    (tcm.TC_GEMM_F64, tcm.TC_FRAME_ROTATING, torch.complex128, 1e-12),
    (tcm.TC_GEMM_F32, tcm.TC_FRAME_ROTATING, torch.complex64, 1e-5),
    (tcm.TC_GEMM_SPLIT_BF16, tcm.TC_FRAME_ROTATING, torch.complex64, 1e-5),
]


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tcm.lib()


def _open(n, c, seed, kappa, gamma, state="gaussian"):
    inst = ti.random_model(n, c, seed, state=state)
    inst.g = inst.g * 10          # couplings comparable with the losses
    inst.kappa, inst.gamma = kappa, gamma
    return inst


def _oracle(inst, dt, steps):
    n, c = inst.n, inst.c
    H = omodel.hamiltonian(n, c, inst.g, inst.omega_a)
    U = oev.propagator(H, dt)
    O = sum(omodel.atom_excitation_diag(n, c, i) for i in range(n))
    ph = omodel.photon_number_diag(n, c)
    per = 1 << n

    def obs(r):
        d = np.real(np.diag(r))
        return float(np.sum(O * d)), np.array([d[m * per:(m + 1) * per].sum() for m in range(c + 1)]), \
            float(np.sum(ph * d))
    rho, rec = oos.evolve_open_split(inst.rho0(), U, n, c, inst.kappa, inst.gamma, dt, steps, obs)
    return rho, np.array([r[0] for r in rec]), np.array([r[1] for r in rec])


def _gpu(inst, dt, steps, mode, frame, dtype, full=False):
    m = pipeline.model_of(inst)
    _, U = pipeline.propagator(m, dt)
    rho = torch.from_numpy(inst.rho0()).to("cuda").to(dtype)
    pop, pd, _ = pipeline.evolve(m, U, rho, steps, dt, mode, frame, 0, 1, record_photons=True,
                                 full_product=full)
    torch.cuda.synchronize()
    return rho.cpu().numpy().astype(np.complex128), pop.cpu().numpy(), pd.cpu().numpy()


@pytest.mark.parametrize("mode,frame,dtype,tol", MODES)
@pytest.mark.parametrize("n,c", [(4, 3), (5, 2), (6, 4)])
def test_against_oracle_split_step(mode, frame, dtype, tol, n, c):
    """N = 128, 96 and 320 (ragged against the 128 tiles), 60 steps with
    kappa = 0.05, gamma = 0.03: every population and photon-number record and
    the final rho."""
    inst = _open(n, c, 60 + n, 0.05, 0.03)
    dt, steps = 0.1, 60
    rho_ref, pop_ref, pd_ref = _oracle(inst, dt, steps)
    rho, pop, pd = _gpu(inst, dt, steps, mode, frame, dtype)
    e_pop, e_pd = np.max(np.abs(pop - pop_ref)), np.max(np.abs(pd - pd_ref))
    e_rho = np.max(np.abs(rho - rho_ref))
    print(f"open n={n} c={c} mode={mode}: max-entry {e_rho:.3e}, population {e_pop:.3e}, "
          f"photon distribution {e_pd:.3e}", flush=True)
    assert e_pop <= tol and e_pd <= tol and e_rho <= tol


@pytest.mark.parametrize("mode,frame,dtype,tol", MODES)
def test_invariants(mode, frame, dtype, tol):
    """Trace one, Hermitian and positive semidefinite after 150 lossy steps."""
    inst = _open(4, 3, 70, 0.3, 0.2)
    rho, _, _ = _gpu(inst, 0.2, 150, mode, frame, dtype)
    e_tr = abs(np.trace(rho) - 1)
    e_h = np.max(np.abs(rho - rho.conj().T))
    e_min = np.min(np.linalg.eigvalsh(0.5 * (rho + rho.conj().T)))
    print(f"open invariants mode={mode}: |Tr - 1| {e_tr:.3e}, herm {e_h:.3e}, "
          f"min eigenvalue {e_min:.3e}", flush=True)
    assert e_tr <= tol and e_h <= tol and e_min >= -tol


@pytest.mark.parametrize("mode,frame,dtype,tol", [MODES[0], MODES[3]])
def test_pure_decay_at_full_size(mode, frame, dtype, tol):
    """n = 11, c = 5 (N = 12288), g = 0, the workload's initial state: the
    photon number decays as 2 e^{-kappa t} and the excitation as
    E(0) e^{-gamma t}, every step (the split step is exact without coupling)."""
    w = ti.get("n11")
    inst = w.instances[0]
    inst = ti.Instance(n=inst.n, c=inst.c, g=np.zeros(inst.n), omega_a=inst.omega_a,
                       psi0=inst.psi0, kappa=0.08, gamma=0.05)
    steps = 10 if mode == tcm.TC_GEMM_F64 else 40
    dt = 0.05
    _, pop, pd = _gpu(inst, dt, steps, mode, frame, dtype)
    t = dt * np.arange(steps + 1)
    photons = pd @ np.arange(inst.c + 1)
    e_ph = np.max(np.abs(photons - 2 * np.exp(-0.08 * t)))
    e_pop = np.max(np.abs(pop - pop[0] * np.exp(-0.05 * t)))
    print(f"pure decay N=12288 mode={mode}: photon number {e_ph:.3e}, excitation {e_pop:.3e} "
          f"(of {pop[0]:.3f})", flush=True)
    # a sum of N rounded diagonal entries weighted by up to n (c): its error is
    # relative to its size, so the bar scales with the readout once it exceeds 1
    assert e_ph <= tol * max(1.0, 2.0) and e_pop <= tol * max(1.0, float(pop[0]))


@pytest.mark.parametrize("pad", [0, 1])
def test_damping_alone_n10_against_oracle(pad):
    """n = 10, c = 1 (N = 2048), complex FP32, U = I: one step is the damping
    channels alone (the FP32 products with the identity are exact).  With the
    row stride N the three-atom passes (atoms 0-2, 3-5, 6-8) take the 512-column
    coalesced windows; with the odd stride N + 1 the per-block kernel.  Every
    element against the oracle's Kraus channels applied to the same FP32-rounded
    state.  Bar: the ten atom channels and the cavity channel each round every
    entry a few times in FP32 (unit roundoff 6e-8), so 4e-6 of the largest entry."""
    n, c = 10, 1
    inst = _open(n, c, 91, 0.03, 0.07)
    m = pipeline.model_of(inst)
    N = m.N
    dt = 0.5
    rho0 = inst.rho0().astype(np.complex64)
    U = torch.eye(N, dtype=torch.complex128, device="cuda")
    buf = torch.zeros((N, N + pad), dtype=torch.complex64, device="cuda")
    rho = buf[:, :N]
    rho.copy_(torch.from_numpy(rho0))
    pipeline.evolve(m, U, rho, 1, dt, tcm.TC_GEMM_F32, tcm.TC_FRAME_LAB, 0, 1)
    torch.cuda.synchronize()
    ref = oos.dissipation(rho0.astype(np.complex128), n, c, 0.03, 0.07, dt)
    got = rho.cpu().numpy().astype(np.complex128)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref))
    change = np.max(np.abs(ref - rho0))
    print(f"damping alone n=10 stride {N + pad}: max-entry {err:.3e} of {scale:.3e} "
          f"(largest change {change:.3e})", flush=True)
    assert change > 0.05 * scale                         # the channels do act
    assert err <= 4e-6 * scale
    if pad:
        assert torch.all(buf[:, N:] == 0)                # the padding column is untouched


@pytest.mark.parametrize("mode,dtype", [(tcm.TC_GEMM_F32, torch.complex64),
                                        (tcm.TC_GEMM_F64, torch.complex128)])
def test_batched_equals_single(mode, dtype):
    """Lossy instances stepped together (grouped launches) equal their single
    runs bit for bit when every tile is formed."""
    insts = [_open(n, c, 80 + n, 0.04 * (k + 1), 0.02 * (k + 1))
             for k, (n, c) in enumerate([(3, 2), (5, 1), (4, 3)])]
    dt, steps = 0.1, 30
    models = [pipeline.model_of(i) for i in insts]
    Us = [pipeline.propagator(m, dt)[1] for m in models]
    rhos = [torch.from_numpy(i.rho0()).to("cuda").to(dtype) for i in insts]
    pops = [torch.zeros(steps + 1, dtype=torch.float64, device="cuda") for _ in insts]
    rdt = tcm.TC_C128 if dtype == torch.complex128 else tcm.TC_C64
    opts = tcm.make_opts(steps, dt, mode, rdt, tcm.TC_FRAME_ROTATING, 0, 1, 0, 1, 1)
    tcm.tc_evolve([tcm.make_instance(m, U, r, p) for m, U, r, p in zip(models, Us, rhos, pops)],
                  opts)
    torch.cuda.synchronize()
    for k, inst in enumerate(insts):
        rho, pop, _ = _gpu(inst, dt, steps, mode, tcm.TC_FRAME_ROTATING, dtype, full=True)
        assert np.array_equal(rhos[k].cpu().numpy().astype(np.complex128), rho)
        assert np.array_equal(pops[k].cpu().numpy(), pop)
