"""Batched stepping (tc_evolve with count > 1): grouped persistent launches,
hipGraph-captured step chunks and the tile autotuner, against single-instance
runs and the oracle, including the 64-instance uneven workload."""
import json
import os
import time

import numpy as np
import pytest
import torch

import tcm_inputs as ti
from oracle import evolve as oev
from oracle import model as omodel

pytestmark = pytest.mark.gpu

tcm = pytest.importorskip("paper_2403_06937_amd")
from paper_2403_06937_amd import pipeline  # noqa: E402


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tcm.lib()


def _run_batch(insts, dt, steps, mode, frame, dtype, use_graph, record_every=1, renorm=0, full=0):
    models = [pipeline.model_of(i) for i in insts]
    Us = [pipeline.propagator(m, dt)[1] for m in models]
    rhos = [torch.from_numpy(i.rho0()).to("cuda").to(dtype) for i in insts]
    R = steps // record_every + 1
    pops = [torch.zeros(R, dtype=torch.float64, device="cuda") for _ in insts]
    pds = [torch.zeros((R, m.c + 1), dtype=torch.float64, device="cuda") for m in models]
    rdt = tcm.TC_C128 if dtype == torch.complex128 else tcm.TC_C64
    # singles take the same product kernels as batches (not the LDS-resident one)
    opts = tcm.make_opts(steps, dt, mode, rdt, frame, renorm, record_every, 0, use_graph, full,
                         no_resident=1)
    tcm.tc_evolve([tcm.make_instance(m, U, r, p, d) for m, U, r, p, d in zip(models, Us, rhos, pops, pds)],
                  opts)
    torch.cuda.synchronize()
    return ([r.cpu().numpy().astype(np.complex128) for r in rhos], [p.cpu().numpy() for p in pops],
            [d.cpu().numpy() for d in pds])


@pytest.mark.parametrize("mode,dtype", [(tcm.TC_GEMM_F32, torch.complex64),
                                        (tcm.TC_GEMM_F64, torch.complex128)])
@pytest.mark.parametrize("full", [0, 1])
def test_graph_equals_eager_and_single(mode, dtype, full):
    """Uneven instances (N = 24 .. 640): graph replay equals eager launches bit
    for bit.  Single and batch agree to rounding: the N = 256 and 640
    instances run on their own have too few tiles to fill the CUs, so their
    products split their K sums into ranges added in order (the grouped
    launch does not), and with the mirrored triangle (full = 0) the elements
    that are mirrored depend on the tile shape.  In FP64 the instances of a
    single tile row, stepped on their own with every tile (full = 1), equal
    their batch members bit for bit."""
    shapes = [(3, 2), (5, 1), (7, 4), (4, 6), (6, 3)]
    insts = [ti.random_model(n, c, 300 + k, state="gaussian") for k, (n, c) in enumerate(shapes)]
    dt, steps = 0.03, 37
    a = _run_batch(insts, dt, steps, mode, tcm.TC_FRAME_ROTATING, dtype, 0, 1, 10, full)
    b = _run_batch(insts, dt, steps, mode, tcm.TC_FRAME_ROTATING, dtype, 1, 1, 10, full)
    for k in range(len(insts)):
        assert np.array_equal(a[0][k], b[0][k]) and np.array_equal(a[1][k], b[1][k])
        assert np.array_equal(a[2][k], b[2][k])
        single = _run_batch([insts[k]], dt, steps, mode, tcm.TC_FRAME_ROTATING, dtype, 0, 1, 10,
                            full)
        if full and mode == tcm.TC_GEMM_F64 and insts[k].N <= 128:
            assert np.array_equal(single[0][0], a[0][k])
        tol = 1e-14 if mode == tcm.TC_GEMM_F64 else 2e-6
        assert np.max(np.abs(single[0][0] - a[0][k])) <= tol


def test_record_every_and_graph_chunks():
    """record_every = 3 with 50 steps: records 0..16 hold the readout after 3r
    steps, also when a graph chunk covers 15 steps and 5 steps run eagerly."""
    insts = [ti.random_model(3, 3, 310 + k, state="gaussian") for k in range(3)]
    dt, steps = 0.05, 50
    rhos, pops, _ = _run_batch(insts, dt, steps, tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB,
                               torch.complex128, 1, 3)
    for k, inst in enumerate(insts):
        P = oev.SectorPropagator(inst.n, inst.c, inst.g, inst.omega_a)
        O = sum(omodel.atom_excitation_diag(inst.n, inst.c, i) for i in range(inst.n))
        assert pops[k].shape == (17,)
        for r in range(17):
            ref = float(np.sum(O * np.abs(P.psi(inst.psi0, 3 * r * dt)) ** 2))
            assert abs(pops[k][r] - ref) < 1e-12


def test_autotune_table_and_cache(tmp_path):
    path = tmp_path / "tune.json"
    os.environ["TC_AUTOTUNE_CACHE"] = str(path)
    try:
        tcm.tc_autotune(tcm.TC_GEMM_F32, 1024)
        v = [tcm.tc_autotune_query(tcm.TC_GEMM_F32, N) for N in (64, 512, 2048, 8192)]
        assert all(x in (1, 2) for x in v)
        d = json.loads(path.read_text())
        assert d["f32"][:2] == v[:2]
    finally:
        del os.environ["TC_AUTOTUNE_CACHE"]


def test_batch64_workload_parity():
    """The 64-instance uneven workload (n in 4..10, c in 1..6, N = 32 .. 6144,
    complex64, dt = 0.02, rotating frame) for all 500 steps in one grouped,
    graph-captured call: every element of every instance's final rho and
    every 25th population record against the oracle's exact evolution."""
    w = ti.get("batch64")
    insts = w.instances
    steps = w.steps
    models = [pipeline.model_of(i) for i in insts]
    Us = [pipeline.propagator(m, w.dt)[1] for m in models]
    rhos = [torch.from_numpy(i.rho0()).to("cuda").to(torch.complex64) for i in insts]
    pops = [torch.zeros(steps + 1, dtype=torch.float64, device="cuda") for _ in insts]
    opts = tcm.make_opts(steps, w.dt, tcm.TC_GEMM_F32, tcm.TC_C64, tcm.TC_FRAME_ROTATING, 0, 1, 0, 1)
    torch.cuda.synchronize()
    t0 = time.time()
    tcm.tc_evolve([tcm.make_instance(m, U, r, p) for m, U, r, p in zip(models, Us, rhos, pops)],
                  opts)
    torch.cuda.synchronize()
    print(f"gpu batch64 {steps} steps {time.time() - t0:.2f}s", flush=True)
    del Us
    worst, worst_pop, at = 0.0, 0.0, None
    for k, inst in enumerate(insts):
        P = oev.SectorPropagator(inst.n, inst.c, inst.g, inst.omega_a)
        psi = P.psi(inst.psi0, steps * w.dt)
        rho = rhos[k].cpu().numpy()
        err = 0.0
        for r0 in range(0, inst.N, 1024):
            blk = rho[r0:r0 + 1024].astype(np.complex128)
            err = max(err, float(np.max(np.abs(blk - np.outer(psi[r0:r0 + 1024], psi.conj())))))
        O = sum(omodel.atom_excitation_diag(inst.n, inst.c, i) for i in range(inst.n))
        popn = pops[k].cpu().numpy()
        perr = max(abs(popn[s] - float(np.sum(O * np.abs(P.psi(inst.psi0, s * w.dt)) ** 2)))
                   for s in range(0, steps + 1, 25))
        if err > worst:
            at = (k, inst.n, inst.c, inst.N)
        worst, worst_pop = max(worst, err), max(worst_pop, perr)
    print(f"batch64 ({steps} steps): worst max-entry error {worst:.2e} (instance, n, c, N = {at}), "
          f"worst population error {worst_pop:.2e}", flush=True)
    assert worst <= 1e-5 and worst_pop <= 1e-5
