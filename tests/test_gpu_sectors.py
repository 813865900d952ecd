"""Excitation-sector block stepping (tc_evolve with opts.sectors = 1) on the
GPU: against the oracle's dense evolution and against the dense GPU products,
on ragged sizes, both frames, with records, checkpoints,
renormalisation and the Lindblad term, in FP64, FP32 and split-BF16; plus
the degenerate cases (no cavity photons, one atom, zero steps)."""
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
    (tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB, torch.complex128, 1e-10),
    (tcm.TC_GEMM_F64, tcm.TC_FRAME_ROTATING, torch.complex128, 1e-10),
    (tcm.TC_GEMM_F32, tcm.TC_FRAME_LAB, torch.complex64, 1e-5),
    (tcm.TC_GEMM_F32, tcm.TC_FRAME_ROTATING, torch.complex64, 1e-5),
    (tcm.TC_GEMM_SPLIT_BF16, tcm.TC_FRAME_ROTATING, torch.complex64, 1e-5),
]


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tcm.lib()


def _oracle(inst, dt, steps):
    """Dense oracle: rho(s dt) = U^s rho0 U^dag^s with U from eigh, plus the
    per-step population and photon-number records."""
    n, c = inst.n, inst.c
    H = omodel.hamiltonian(n, c, inst.g, inst.omega_a)
    U = oev.propagator(H, dt)
    O = sum(omodel.atom_excitation_diag(n, c, i) for i in range(n))
    per = 1 << n
    rho = inst.rho0()
    pops, pds = [], []
    for s in range(steps + 1):
        d = np.real(np.diag(rho))
        pops.append(float(np.sum(O * d)))
        pds.append([d[m * per:(m + 1) * per].sum() for m in range(c + 1)])
        if s < steps:
            rho = U @ rho @ U.conj().T
    return rho, np.array(pops), np.array(pds)


def _gpu(inst, dt, steps, mode, frame, dtype, sectors, renorm=0, checkpoint_every=0):
    m = pipeline.model_of(inst)
    _, U = pipeline.propagator(m, dt)
    rho = torch.from_numpy(inst.rho0()).to("cuda").to(dtype)
    pop, pd, ck = pipeline.evolve(m, U, rho, steps, dt, mode, frame, renorm, 1,
                                  checkpoint_every, record_photons=True, sectors=sectors)
    torch.cuda.synchronize()
    ckn = None if ck is None else ck.cpu().numpy().astype(np.complex128)
    return rho.cpu().numpy().astype(np.complex128), pop.cpu().numpy(), pd.cpu().numpy(), ckn


@pytest.mark.parametrize("mode,frame,dtype,tol", MODES)
@pytest.mark.parametrize("n,c,seed", [(3, 3, 0), (5, 2, 1), (6, 4, 2), (7, 1, 3), (1, 6, 4),
                                      (4, 0, 5)])
def test_against_oracle(mode, frame, dtype, tol, n, c, seed):
    """Dense random pure state (every sector block populated), 40 steps,
    renormalised every 10: final rho, every population and photon-number
    record within the precision's bar.  N = 32, 96, 320, 256, 14 and 16,
    none a multiple of the 128 tile except through its sector blocks."""
    inst = ti.random_model(n, c, seed)
    inst.g = inst.g * 20                    # visible dynamics within 40 steps
    dt, steps = 0.05, 40
    ref, rpop, rpd = _oracle(inst, dt, steps)
    rho, pop, pd, _ = _gpu(inst, dt, steps, mode, frame, dtype, True, renorm=10)
    err = float(np.max(np.abs(rho - ref)))
    perr = float(np.max(np.abs(pop - rpop)))
    derr = float(np.max(np.abs(pd - rpd)))
    print(f"sectors n={n} c={c} mode={mode} frame={frame}: max-entry {err:.2e}, "
          f"population {perr:.2e}, photon distribution {derr:.2e}")
    assert err < tol and perr < tol and derr < tol


@pytest.mark.parametrize("mode,frame,dtype,tol", MODES)
def test_equals_dense_products(mode, frame, dtype, tol):
    """Sector blocks and the dense N x N products reach the same state (the
    cross-sector entries of U are exact zeros): FP64 to rounding (1e-13),
    FP32 to its bar."""
    inst = ti.random_model(6, 3, 7)          # N = 256
    inst.g = inst.g * 20
    a, pa, _, _ = _gpu(inst, 0.05, 30, mode, frame, dtype, False, renorm=10)
    b, pb, _, _ = _gpu(inst, 0.05, 30, mode, frame, dtype, True, renorm=10)
    bar = 1e-13 if dtype == torch.complex128 else tol
    assert float(np.max(np.abs(a - b))) < bar
    assert float(np.max(np.abs(pa - pb))) < bar


def test_checkpoints_and_hermiticity():
    """Checkpoints of a sector run are the dense oracle's states at those steps,
    in the basis order and lab frame, exactly Hermitian off the diagonal
    blocks (the lower block triangle is the mirror of the upper)."""
    inst = ti.random_model(5, 3, 11)          # N = 128
    inst.g = inst.g * 20
    dt, steps, every = 0.05, 30, 10
    n, c = inst.n, inst.c
    U = oev.propagator(omodel.hamiltonian(n, c, inst.g, inst.omega_a), dt)
    rho, _, _, ck = _gpu(inst, dt, steps, tcm.TC_GEMM_F64, tcm.TC_FRAME_ROTATING,
                         torch.complex128, True, checkpoint_every=every)
    assert ck.shape == (steps // every + 1, inst.N, inst.N)
    r = inst.rho0()
    for s in range(steps + 1):
        if s % every == 0:
            assert np.max(np.abs(ck[s // every] - r)) < 1e-12, s
        if s < steps:
            r = U @ r @ U.conj().T
    assert np.max(np.abs(rho - r)) < 1e-12
    lab, _, _, _ = _gpu(inst, dt, steps, tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB, torch.complex128,
                        True)
    k = omodel.total_excitation_diag(n, c)
    off = k[:, None] != k[None, :]
    assert np.array_equal(lab[off], lab.conj().T[off])


@pytest.mark.parametrize("mode,frame,dtype,tol", [
    (tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB, torch.complex128, 1e-12),
    (tcm.TC_GEMM_F32, tcm.TC_FRAME_ROTATING, torch.complex64, 2e-5),
    (tcm.TC_GEMM_SPLIT_BF16, tcm.TC_FRAME_ROTATING, torch.complex64, 2e-5)])
def test_open_system(mode, frame, dtype, tol):
    """With the Lindblad term (kappa = 0.05, gamma = 0.03) each sector step is
    followed by the damping channels in the basis order: equal to the oracle's
    split step."""
    inst = ti.random_model(5, 2, 12)          # N = 96
    inst.g = inst.g * 10
    inst.kappa, inst.gamma = 0.05, 0.03
    dt, steps = 0.05, 40
    n, c = inst.n, inst.c
    U = oev.propagator(omodel.hamiltonian(n, c, inst.g, inst.omega_a), dt)
    O = sum(omodel.atom_excitation_diag(n, c, i) for i in range(n))
    ref, rec = oos.evolve_open_split(inst.rho0(), U, n, c, inst.kappa, inst.gamma, dt, steps,
                                     lambda r: float(np.sum(O * np.real(np.diag(r)))))
    rho, pop, _, _ = _gpu(inst, dt, steps, mode, frame, dtype, True)
    err = float(np.max(np.abs(rho - ref)))
    perr = float(np.max(np.abs(pop - np.array(rec))))
    print(f"sectors open system mode={mode}: max-entry {err:.2e}, population {perr:.2e}")
    assert err < tol and perr < tol


def test_zero_steps_and_single_step():
    """steps = 0 returns an exactly Hermitian rho(0) bitwise (permute and
    unpermute are exact copies, and the mirrored lower block triangle equals
    what was there); one step matches U rho U^dag."""
    inst = ti.random_model(4, 2, 13)          # N = 48
    rho0 = inst.rho0()
    rho0 = 0.5 * (rho0 + rho0.conj().T)      # bitwise Hermitian
    m = pipeline.model_of(inst)
    _, Ug = pipeline.propagator(m, 0.05)
    r = torch.from_numpy(rho0).to("cuda")
    pop, _, _ = pipeline.evolve(m, Ug, r, 0, 0.05, sectors=True)
    assert np.array_equal(r.cpu().numpy(), rho0)
    assert pop.shape == (1,)
    U = oev.propagator(omodel.hamiltonian(inst.n, inst.c, inst.g, inst.omega_a), 0.05)
    b, _, _, _ = _gpu(inst, 0.05, 1, tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB, torch.complex128, True)
    assert np.max(np.abs(b - U @ rho0 @ U.conj().T)) < 1e-14


def test_workload_n9_sectors():
    """The N = 5120 FP64 workload (|0>|1^9>, 100 steps) by sector blocks: every
    population record and the final rho within 1e-10 of the oracle."""
    w = ti.get("n9")
    inst = w.instances[0]
    n, c = inst.n, inst.c
    P = oev.SectorPropagator(n, c, inst.g, inst.omega_a)
    O = sum(omodel.atom_excitation_diag(n, c, i) for i in range(n))
    rho, pop, _, _ = _gpu(inst, w.dt, w.steps, tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB,
                          torch.complex128, True)
    ref = np.array([float(np.sum(O * np.abs(P.psi(inst.psi0, s * w.dt)) ** 2))
                    for s in range(w.steps + 1)])
    assert np.max(np.abs(pop - ref)) < 1e-10
    psiT = P.psi(inst.psi0, w.steps * w.dt)
    err = 0.0
    for r0 in range(0, inst.N, 1024):
        err = max(err, float(np.max(np.abs(rho[r0:r0 + 1024] - np.outer(psiT[r0:r0 + 1024],
                                                                          psiT.conj())))))
    print(f"n9 sectors fp64: max-entry {err:.2e}")
    assert err < 1e-10


def test_split_lab_frame_runs():
    """Split-BF16 by sectors in the lab frame (the rounded operand is U_k, not
    D_k): same result as the dense split products in the lab frame to the
    lab frame's error level."""
    inst = ti.random_model(5, 3, 15)          # N = 128
    inst.g = inst.g * 20
    dt, steps = 0.05, 40
    ref, _, _ = _oracle(inst, dt, steps)
    a, _, _, _ = _gpu(inst, dt, steps, tcm.TC_GEMM_SPLIT_BF16, tcm.TC_FRAME_LAB,
                      torch.complex64, True, renorm=10)
    b, _, _, _ = _gpu(inst, dt, steps, tcm.TC_GEMM_SPLIT_BF16, tcm.TC_FRAME_LAB,
                      torch.complex64, False, renorm=10)
    ea, eb = float(np.max(np.abs(a - ref))), float(np.max(np.abs(b - ref)))
    print(f"split lab frame: sectors {ea:.2e}, dense {eb:.2e}")
    assert ea < 1e-3 and eb < 1e-3


def _run_batch(insts, dt, steps, mode, frame, dtype, use_graph, sectors, renorm=10):
    models = [pipeline.model_of(i) for i in insts]
    Us = [pipeline.propagator(m, dt)[1] for m in models]
    rhos = [torch.from_numpy(i.rho0()).to("cuda").to(dtype) for i in insts]
    pops = [torch.zeros(steps + 1, dtype=torch.float64, device="cuda") for _ in insts]
    pds = [torch.zeros((steps + 1, m.c + 1), dtype=torch.float64, device="cuda") for m in models]
    rdt = tcm.TC_C128 if dtype == torch.complex128 else tcm.TC_C64
    opts = tcm.make_opts(steps, dt, mode, rdt, frame, renorm, 1, 0, use_graph, 0,
                         sectors=int(sectors))
    tcm.tc_evolve([tcm.make_instance(m, U, r, p, d)
                   for m, U, r, p, d in zip(models, Us, rhos, pops, pds)], opts)
    torch.cuda.synchronize()
    return ([r.cpu().numpy().astype(np.complex128) for r in rhos], [p.cpu().numpy() for p in pops],
            [d.cpu().numpy() for d in pds])


@pytest.mark.parametrize("mode,frame,dtype,tol", MODES)
def test_batched_sectors(mode, frame, dtype, tol):
    """Uneven instances stepped together by sector blocks (one grouped launch
    per product over the blocks of all instances; eager and hipGraph chunks):
    bitwise equal to each instance's own sector run (the same block tiles),
    and within the precision's bar of the oracle."""
    shapes = [(3, 2), (5, 1), (7, 4), (4, 6), (6, 3)]
    insts = [ti.random_model(n, c, 400 + k, state="gaussian") for k, (n, c) in enumerate(shapes)]
    for i in insts:
        i.g = i.g * 20
    dt, steps = 0.05, 30
    a = _run_batch(insts, dt, steps, mode, frame, dtype, 0, True)
    b = _run_batch(insts, dt, steps, mode, frame, dtype, 1, True)
    for k, inst in enumerate(insts):
        assert np.array_equal(a[0][k], b[0][k]) and np.array_equal(a[1][k], b[1][k])
        single = _run_batch([inst], dt, steps, mode, frame, dtype, 0, True)
        assert np.array_equal(single[0][0], a[0][k])
        assert np.array_equal(single[1][0], a[1][k])
        ref, rpop, _ = _oracle(inst, dt, steps)
        err = float(np.max(np.abs(a[0][k] - ref)))
        perr = float(np.max(np.abs(a[1][k] - rpop)))
        assert err < tol and perr < tol, (k, err, perr)
