"""Benchmark of the Tavis-Cummings density-matrix stepper on one MI355X.

Workload: n = 11 atoms, photon cutoff 5 (N = 12288), seeded g_i ~ U(0.005,
0.02) and delta_i ~ N(0, 0.005), rho0 = |2 photons> (x) Haar product state,
dt = 0.05, renormalised every 20 steps, excited-atom population recorded
every step.  A step is one pass of the whole path: rho <- U rho U^dag (two
complex N x N x N products; the second one's result is Hermitian, so its upper
tile triangle is multiplied and mirrored), the per-step readout and (every
20th step) the FP64 renormalisation.  U = exp(-i H dt) is formed before the timed region
and timed on its own.

The headline value is the split-BF16 form (hi/lo 3-term products on BF16
MFMA, FP32 accumulation, rotating frame) in steps/s; the FP64 and complex
FP32 forms are measured on the same workload and reported beside it.
`roofline.mfma_probe` gives what the product kernels' MFMA instructions
sustain with no memory traffic (zero and random operand bits), the practical
ceiling against which `roofline.issued_frac` reads.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ρ←UρU† steps/s + TFLOP/s at N=12288: FP64 vs split-BF16 at ≤1e-5 error"
PEAK_BF16 = 2.5e15       # dense BF16 MFMA, FLOP/s
PEAK_F64 = 78.6e12       # FP64 MFMA
PEAK_F32 = 157.3e12      # FP32 MFMA


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_entry(kernel, workload, src):
    """HBM bytes per product measured with rocprofv3 counters (profiles/traffic.json),
    only if recorded for the kernel source as it is now."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(f"{kernel}@{workload}")
        if e and e.get("source_sha") == kernel_source_hash(src):
            return e.get("bytes_per_launch")
    except Exception:
        return None
    return None


TILE = 128                # output tile edge of the product kernels at this size


def executed_flop_per_step(N, full=False, tile=TILE):
    """Flops (8 per complex multiply-add) the two products of one step execute:
    the first product in full; the second, whose result is Hermitian, on the
    T(T+1)/2 tiles on and above the tile diagonal of its T x T tile grid."""
    T = -(-N // tile)
    frac = 1.0 if full else T * (T + 1) / 2.0 / (T * T)
    return 8.0 * float(N) ** 3 * (1.0 + frac)


def run_mode(tcm, pipeline, model, U, rho0_np, mode, frame, dtype, steps, warmup, dt, renorm):
    import torch
    rho = torch.from_numpy(rho0_np).to("cuda").to(dtype)
    rdt = tcm.TC_C128 if dtype == torch.complex128 else tcm.TC_C64
    # warmup (same call shape)
    if warmup:
        w = rho.clone()
        pipeline.evolve(model, U, w, warmup, dt, mode, frame, renorm, 1)
        del w
    pop = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
    opts = tcm.make_opts(steps, dt, mode, rdt, frame, renorm, 1)
    inst = tcm.make_instance(model, U, rho, pop)
    ws = torch.empty(tcm.tc_evolve_workspace_size([inst], opts), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    kind = {tcm.TC_GEMM_F64: tcm.TC_KERNEL_GEMM_F64, tcm.TC_GEMM_F32: tcm.TC_KERNEL_GEMM_F32,
            tcm.TC_GEMM_SPLIT_BF16: tcm.TC_KERNEL_SPLIT_BF16}[mode]
    tcm.tc_profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    tcm.tc_evolve([inst], opts, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    kms, klaunch = tcm.tc_profile_read(kind)
    tcm.tc_profile_enable(False)
    return {"ms_total": ms_total, "wall_s": wall, "kernel_ms": kms, "kernel_launches": klaunch,
            "rho": rho, "pop": pop}


def bench_n9(tcm, pipeline, ti, steps=100):
    """n=9, c=9 (N=5120) FP64 workload: steps/s and TFLOP/s of its full 100-step run."""
    import torch
    w = ti.get("n9")
    inst = w.instances[0]
    m = pipeline.model_of(inst)
    _, U = pipeline.propagator(m, w.dt)
    rho = torch.from_numpy(inst.rho0()).to("cuda")
    pipeline.evolve(m, U, rho.clone(), 2, w.dt)                   # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    pipeline.evolve(m, U, rho, steps, w.dt)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fx = executed_flop_per_step(inst.N)
    return {"workload": w.name, "N": inst.N, "dtype": "f64", "steps": steps,
            "steps_per_s": 1000.0 / ms, "ms_per_step": ms,
            "tflops": 16.0 * inst.N ** 3 / (ms * 1e-3) / 1e12,
            "tflops_executed": fx / (ms * 1e-3) / 1e12,
            "executed_frac_of_peak": fx / (ms * 1e-3) / PEAK_F64}


def mfma_probe(tcm):
    """What the MFMA instructions of the product kernels sustain with no memory
    traffic: one 512-thread workgroup per CU issuing them back to back on
    register operands, zero and random bits, as fractions of the datasheet
    peak.  Random-operand BF16 issue draws enough power to lower the clock, so
    its fraction is the practical ceiling of the split-BF16 product's
    issued_frac."""
    kinds = {"bf16_16x16x32": (tcm.TC_PROBE_BF16_16X16X32, PEAK_BF16, 100000),
             "bf16_32x32x16": (tcm.TC_PROBE_BF16_32X32X16, PEAK_BF16, 100000),
             "f64_16x16x4": (tcm.TC_PROBE_F64_16X16X4, PEAK_F64, 10000)}
    out = {}
    for name, (kind, peak, iters) in kinds.items():
        tcm.tc_mfma_probe(kind, True, iters // 10)
        r = {}
        for label, rnd in (("zero_operands_frac", False), ("random_operands_frac", True)):
            ms, fl = tcm.tc_mfma_probe(kind, rnd, iters)
            r[label] = fl / (ms * 1e-3) / peak
        out[name] = r
    return out


def mfma_probe_or_none(tcm):
    """The probe is context for the roofline; a failure of it must not cost the
    benchmark line (reported as null with the error)."""
    try:
        return mfma_probe(tcm)
    except Exception as e:  # noqa: BLE001 - any failure is reported, not raised
        log(f"mfma probe failed: {e}")
        return None


def bench_jc3(tcm, pipeline, ti):
    """n = 3, c = 3 (N = 32), FP64, dt = 0.01 x 1000 steps with the excited-atom
    population recorded every step: launch-bound.  Timed in the LDS-resident
    kernel (all steps in one launch, the default at this size) and with the
    launches of every step issued eagerly or as hipGraph-captured chunks."""
    import torch
    w = ti.get("jc3")
    inst = w.instances[0]
    m = pipeline.model_of(inst)
    _, U = pipeline.propagator(m, w.dt)
    rho0 = torch.from_numpy(inst.rho0()).to("cuda")
    out = {"workload": w.name, "N": inst.N, "dtype": "f64", "steps": w.steps}
    for key, graph, nores in (("resident", False, False), ("eager", False, True),
                              ("graph", True, True)):
        pipeline.evolve(m, U, rho0.clone(), 50, w.dt, use_graph=graph, no_resident=nores)
        rho = rho0.clone()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        pop, _, _ = pipeline.evolve(m, U, rho, w.steps, w.dt, use_graph=graph, no_resident=nores)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        out[key] = {"ms_total": ms, "wall_ms": 1e3 * wall, "steps_per_s": w.steps / (ms * 1e-3),
                    "us_per_step": 1e3 * ms / w.steps, "final_excitation": float(pop[-1].item())}
    return out


def bench_batch64(tcm, pipeline, ti, steps=50):
    """64 uneven instances (N = 32..7168, complex64) stepped together: grouped
    persistent launches with autotuned tile shapes, hipGraph-captured chunks."""
    import torch
    w = ti.get("batch64")
    models = [pipeline.model_of(i) for i in w.instances]
    Us = [pipeline.propagator(m, w.dt)[1] for m in models]
    maxN = max(m.N for m in models)
    t0 = time.perf_counter()
    tcm.tc_autotune(tcm.TC_GEMM_F32, maxN)
    tune_s = time.perf_counter() - t0
    rho0 = [torch.from_numpy(i.rho0()).to("cuda").to(torch.complex64) for i in w.instances]

    def run(k, mode=tcm.TC_GEMM_F32, sectors=0):
        rhos = [r.clone() for r in rho0]
        pops = [torch.zeros(k + 1, dtype=torch.float64, device="cuda") for _ in models]
        opts = tcm.make_opts(k, w.dt, mode, tcm.TC_C64, tcm.TC_FRAME_ROTATING, 0, 1, 0, 1,
                             sectors=sectors)
        insts = [tcm.make_instance(m, U, r, p) for m, U, r, p in zip(models, Us, rhos, pops)]
        ws = torch.empty(tcm.tc_evolve_workspace_size(insts, opts), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        tcm.tc_evolve(insts, opts, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    run(16)                                                      # warm-up
    ms = run(steps)
    flop = 16.0 * sum(float(m.N) ** 3 for m in models) * steps
    edge = {b: 128 if tcm.tc_autotune_query(tcm.TC_GEMM_F32, b) == 1 else 64
            for b in (256, 1024, 4096, 1 << 30)}

    def tile_edge(N):
        return edge[min(b for b in edge if N <= b)]
    fx = sum(executed_flop_per_step(m.N, tile=tile_edge(m.N)) for m in models) * steps
    out = {"workload": w.name, "instances": len(models), "N_min": min(m.N for m in models),
           "N_max": maxN, "dtype": "f32", "steps": steps, "steps_per_s": steps / (ms * 1e-3),
           "ms_per_step": ms / steps, "tflops": flop / (ms * 1e-3) / 1e12,
           "tflops_executed": fx / (ms * 1e-3) / 1e12,
           "executed_frac_of_peak": fx / (ms * 1e-3) / PEAK_F32,
           "autotune_s": tune_s,
           "tile_variants": {str(b): tcm.tc_autotune_query(tcm.TC_GEMM_F32, b)
                             for b in (256, 1024, 4096, 7168)}}
    # the same batch by excitation-sector blocks (all instances' blocks in one
    # grouped launch per product), complex FP32 and split-BF16
    for key, mode in (("sectors_fp32", tcm.TC_GEMM_F32), ("sectors_split", tcm.TC_GEMM_SPLIT_BF16)):
        run(8, mode, 1)
        ms = run(steps, mode, 1)
        sflop = sum(sector_flop_per_step(m.n, m.c) for m in models) * steps
        out[key] = {"steps_per_s": steps / (ms * 1e-3), "ms_per_step": ms / steps,
                    "tflops": sflop / (ms * 1e-3) / 1e12,
                    "dense_equivalent_tflops": flop / (ms * 1e-3) / 1e12}
    return out


def bench_grad8(tcm, pipeline, ti):
    """n=8, c=8 (N=2304): complex64 forward with checkpoints every 50 (500 steps,
    rotating frame) and the adjoint sweep (FP32 products, FP64 Frechet), with
    dense products and by excitation sectors."""
    import torch
    w = ti.get("grad8")
    inst = w.instances[0]
    m = pipeline.model_of(inst)
    H, U = pipeline.propagator(m, w.dt)
    rho0 = torch.from_numpy(inst.rho0()).to("cuda").to(torch.complex64)
    out = {"workload": w.name, "N": inst.N, "steps": w.steps, "dtype": "f32"}
    for key, sec in (("dense", False), ("sectors", True)):
        rho = rho0.clone()
        pipeline.evolve(m, U, rho.clone(), 4, w.dt, tcm.TC_GEMM_F32, tcm.TC_FRAME_ROTATING,
                        sectors=sec)                                         # warm-up
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        ev[0].record()
        _, _, ck = pipeline.evolve(m, U, rho, w.steps, w.dt, tcm.TC_GEMM_F32,
                                   tcm.TC_FRAME_ROTATING, 0, w.steps, w.checkpoint_every,
                                   sectors=sec)
        ev[1].record()
        opts = tcm.make_opts(w.steps, w.dt, tcm.TC_GEMM_F32, tcm.TC_C64, tcm.TC_FRAME_LAB, 0, 1,
                             w.checkpoint_every, sectors=int(sec))
        gg = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        gd = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        ws = torch.empty(tcm.tc_evolve_backward_workspace_size(m, opts), dtype=torch.uint8,
                         device="cuda")
        torch.cuda.synchronize()
        ev[2].record()
        tcm.tc_evolve_backward(m, H, U, opts, ck, loss, gg, gd, ws=ws)
        ev[3].record()
        torch.cuda.synchronize()
        fwd = ev[0].elapsed_time(ev[1])
        bwd = ev[2].elapsed_time(ev[3])
        out[key] = {"forward_s": fwd / 1000.0, "backward_s": bwd / 1000.0,
                    "backward_over_forward": bwd / fwd, "loss": float(loss.item())}
        del ck, ws
    return out


def bench_open11(tcm, pipeline, ti, steps=20):
    """The N = 12288 workload with the Lindblad term of Eq. (5) switched on
    (kappa = 0.01, gamma = 0.005): split-BF16 rotating-frame steps followed by
    the exact damping channels, against the same steps without them."""
    import torch
    w = ti.get("n11")
    inst = w.instances[0]
    m0 = pipeline.model_of(inst)
    m1 = tcm.Model(m0.n, m0.c, m0.g, m0.omega_a, m0.omega_c, kappa=0.01, gamma=0.005)
    _, U = pipeline.propagator(m0, w.dt)
    out = {"workload": "tcm_n11_c5_N12288_open", "N": inst.N, "dtype": "bf16", "steps": steps,
           "kappa": 0.01, "gamma": 0.005}
    for key, m in (("unitary", m0), ("open", m1)):
        rho = torch.from_numpy(inst.rho0()).to("cuda").to(torch.complex64)
        pipeline.evolve(m, U, rho.clone(), 2, w.dt, tcm.TC_GEMM_SPLIT_BF16, tcm.TC_FRAME_ROTATING)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        pop, _, _ = pipeline.evolve(m, U, rho, steps, w.dt, tcm.TC_GEMM_SPLIT_BF16,
                                    tcm.TC_FRAME_ROTATING, w.renorm_every)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[key + "_ms_per_step"] = ms
        out[key + "_final_excitation"] = float(pop[-1].item())
    out["steps_per_s"] = 1000.0 / out["open_ms_per_step"]
    out["dissipation_ms_per_step"] = out["open_ms_per_step"] - out["unitary_ms_per_step"]
    del U
    return out


def bench_dense12(tcm, pipeline, ti, steps=20, steps64=2):
    """Dense control at N = 12288: U from a dense random real symmetric H with
    ||H dt|| ~ 0.8 and a dense random pure rho, against the TCM workload's own
    U and rho0, both in the lab frame (the rotating frame is exact only for a
    U that commutes with the excitation number), split-BF16 and FP64.  The
    product kernels do the same work on any values; this shows what the exact
    zeros of the TCM operands do to their time (clocks, power)."""
    import torch
    w = ti.get("n11")
    inst = w.instances[0]
    m = pipeline.model_of(inst)
    N, dt = inst.N, w.dt
    Hn, psi = ti.dense_control(N, dt)
    H = torch.from_numpy(Hn).to("cuda")
    del Hn
    # Gershgorin interval of the control H (any valid bound sets the scaling)
    off = H.abs().sum(dim=1) - H.diagonal().abs()
    lo = float((H.diagonal() - off).min().item())
    hi = float((H.diagonal() + off).max().item())
    Ud = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    tcm.tc_expm(H, dt, lo, hi, Ud)
    del H, off
    psi_t = torch.from_numpy(psi).to("cuda")
    rho_d = torch.outer(psi_t, psi_t.conj())
    _, Ut = pipeline.propagator(m, dt)
    rho_t = torch.from_numpy(inst.rho0()).to("cuda")
    out = {"workload": "dense_control_N12288", "N": N, "norm_H_dt": 0.8, "steps": steps,
           "steps_fp64": steps64, "frame": "lab"}
    cases = (("dense", Ud, rho_d), ("tcm", Ut, rho_t))
    for mode, key, dtype, K in ((tcm.TC_GEMM_SPLIT_BF16, "split", torch.complex64, steps),
                                (tcm.TC_GEMM_F64, "fp64", torch.complex128, steps64)):
        kind = {tcm.TC_GEMM_F64: tcm.TC_KERNEL_GEMM_F64,
                tcm.TC_GEMM_SPLIT_BF16: tcm.TC_KERNEL_SPLIT_BF16}[mode]
        for name, U, rho0 in cases:
            r = rho0.to(dtype)
            pipeline.evolve(m, U, r.clone(), 1, dt, mode, tcm.TC_FRAME_LAB, w.renorm_every)
            torch.cuda.synchronize()
            tcm.tc_profile_enable(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pipeline.evolve(m, U, r, K, dt, mode, tcm.TC_FRAME_LAB, w.renorm_every)
            e1.record()
            torch.cuda.synchronize()
            kms, kl = tcm.tc_profile_read(kind)
            tcm.tc_profile_enable(False)
            out[f"{key}_{name}_ms_per_step"] = e0.elapsed_time(e1) / K
            out[f"{key}_{name}_product_ms"] = kms / max(1, kl)
            del r
        out[f"{key}_dense_over_tcm"] = (out[f"{key}_dense_ms_per_step"]
                                        / out[f"{key}_tcm_ms_per_step"])
    del Ud, Ut, rho_d, rho_t
    return out


def sector_flop_per_step(n, c):
    """Flops (8 per complex multiply-add) of one sector-block step: for every
    excitation sector k (size d_k, first sorted position o_k) the first
    product X_{k,k:} = U_k rho_{k,k:} is d_k x d_k x (N - o_k) and the second
    rho'_{:k,k} = X_{:k,k} U_k^dag is (o_k + d_k) x d_k x d_k."""
    from math import comb
    d = [sum(comb(n, k - m) for m in range(min(k, c) + 1) if k - m <= n)
         for k in range(n + c + 1)]
    N = sum(d)
    o = [sum(d[:k]) for k in range(len(d))]
    return sum(8.0 * dk * dk * (N - ok) + 8.0 * dk * dk * (ok + dk) for dk, ok in zip(d, o))


def sector_executed_flop_per_step(n, c, q):
    """Flops the sector-block products execute: each sector padded to D_k, a
    multiple of the tile edge q, so the products are 8 sum_k D_k^2 (N_p + D_k)."""
    from math import comb
    d = [sum(comb(n, k - m) for m in range(min(k, c) + 1) if k - m <= n)
         for k in range(n + c + 1)]
    D = [-(-x // q) * q for x in d]
    Np = sum(D)
    return sum(8.0 * x * x * (Np + x) for x in D)


def bench_sectors11(tcm, pipeline, ti, steps=40):
    """The N = 12288 workload stepped by excitation-sector blocks (opts.sectors):
    FP64 (lab frame) and complex FP32 (rotating frame), renormalised every 20
    steps.  Same result as the dense products (cross-sector entries of U are
    exact zeros); 15.3x fewer flops per step."""
    import torch
    w = ti.get("n11")
    inst = w.instances[0]
    m = pipeline.model_of(inst)
    N, dt = inst.N, w.dt
    _, U = pipeline.propagator(m, dt)
    fl = sector_flop_per_step(inst.n, inst.c)
    out = {"workload": "tcm_n11_c5_N12288_sectors", "N": N, "steps": steps,
           "flop_per_step": fl, "dense_flop_per_step": 16.0 * N ** 3}
    for key, mode, frame, dtype, kind in (
            ("fp64", tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB, torch.complex128, tcm.TC_KERNEL_GEMM_F64),
            ("fp32", tcm.TC_GEMM_F32, tcm.TC_FRAME_ROTATING, torch.complex64,
             tcm.TC_KERNEL_GEMM_F32),
            ("split", tcm.TC_GEMM_SPLIT_BF16, tcm.TC_FRAME_ROTATING, torch.complex64,
             tcm.TC_KERNEL_SPLIT_BF16)):
        rho = torch.from_numpy(inst.rho0()).to("cuda").to(dtype)
        pipeline.evolve(m, U, rho.clone(), 2, dt, mode, frame, w.renorm_every, sectors=True)
        torch.cuda.synchronize()
        tcm.tc_profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        pipeline.evolve(m, U, rho, steps, dt, mode, frame, w.renorm_every, sectors=True)
        e1.record()
        torch.cuda.synchronize()
        kms, kl = tcm.tc_profile_read(kind)
        tcm.tc_profile_enable(False)
        ms = e0.elapsed_time(e1) / steps
        peak = {"fp64": PEAK_F64, "fp32": PEAK_F32, "split": PEAK_BF16}[key]
        # tile edge the sector blocks are padded to: 128 for split-BF16 and for
        # FP64 blocks above 1024 states, else the autotuner's table
        from math import comb
        maxd = max(sum(comb(inst.n, k - m) for m in range(min(k, inst.c) + 1) if k - m <= inst.n)
                   for k in range(inst.n + inst.c + 1))
        q = 128 if (key == "split" or (key == "fp64" and maxd > 1024)
                    or tcm.tc_autotune_query(mode, N) == 1) else 64
        fx = sector_executed_flop_per_step(inst.n, inst.c, q)
        out[key] = {"ms_per_step": ms, "steps_per_s": 1000.0 / ms,
                    "tflops": fl / (ms * 1e-3) / 1e12,
                    "tflops_executed": fx / (ms * 1e-3) / 1e12,
                    "dense_equivalent_tflops": 16.0 * N ** 3 / (ms * 1e-3) / 1e12,
                    "product_launches": kl, "product_ms": kms / max(1, kl),
                    "product_frac_of_peak": (fl / 2.0) / (kms / max(1, kl) * 1e-3) / peak,
                    "product_executed_frac_of_peak":
                        (fx / 2.0) / (kms / max(1, kl) * 1e-3) / peak,
                    "product_issued_frac_of_peak":
                        (3.0 if key == "split" else 1.0) * (fx / 2.0)
                        / (kms / max(1, kl) * 1e-3) / peak,
                    "final_excitation": float(torch.real(torch.diagonal(rho)).sum().item())}
        del rho
    del U
    return out


def bench_share(tcm, pipeline, ti, reps=4):
    """One GPU's share of the step distributed over P GPUs by row blocks (rho
    in blocks of N/P rows, U on every GPU): the two local products of a step,
    Y_r = rho_r conj(U) ((N/P) x N x N) and U Y_c (N x (N/P) x N, Y_c a block
    of N/P columns after the all-to-all), in split-BF16 at N = 12288 on the
    TCM operands, timed by the product kernel's own events.  The all-to-all
    between them is not run here (one GPU)."""
    import torch
    w = ti.get("n11")
    inst = w.instances[0]
    m = pipeline.model_of(inst)
    N, dt = inst.N, w.dt
    _, U = pipeline.propagator(m, dt)
    rho = torch.from_numpy(inst.rho0()).to("cuda")
    kind = tcm.TC_KERNEL_SPLIT_BF16
    out = {"workload": "tcm_n11_c5_N12288_share", "N": N, "dtype": "bf16",
           "products": "Y_r = rho_r conj(U), then U Y_c", "shares": []}

    def timed(A, B, C, op_b):
        tcm.tc_zgemm(A, B, C, 0, op_b, 1.0, 0.0, tcm.TC_GEMM_SPLIT_BF16)
        torch.cuda.synchronize()
        tcm.tc_profile_enable(True)
        for _ in range(reps):
            tcm.tc_zgemm(A, B, C, 0, op_b, 1.0, 0.0, tcm.TC_GEMM_SPLIT_BF16)
        torch.cuda.synchronize()
        kms, kl = tcm.tc_profile_read(kind)
        tcm.tc_profile_enable(False)
        return kms / max(1, kl)

    for P in (1, 2, 4, 8):
        r = N // P
        rho_r = rho[:r].contiguous()
        C1 = torch.empty((r, N), dtype=torch.complex128, device="cuda")
        ms1 = timed(rho_r, U, C1, 1)
        B2 = rho[:, :r].contiguous()
        C2 = torch.empty((N, r), dtype=torch.complex128, device="cuda")
        ms2 = timed(U, B2, C2, 0)
        fl = 8.0 * r * N * N
        out["shares"].append({"gpus": P, "rows": r, "rows_product_ms": ms1,
                              "cols_product_ms": ms2,
                              "rows_product_tflops": fl / (ms1 * 1e-3) / 1e12,
                              "cols_product_tflops": fl / (ms2 * 1e-3) / 1e12,
                              "local_products_ms_per_step": ms1 + ms2})
        del rho_r, C1, B2, C2
        torch.cuda.empty_cache()
    base = out["shares"][0]["local_products_ms_per_step"]
    for e in out["shares"]:
        e["compute_speedup_vs_1"] = base / e["local_products_ms_per_step"]
    del U, rho
    return out


def bench_paper_sweep(tcm, pipeline, ti, ns=range(8, 16)):
    """The paper's own model (the 2^n states of all-excited atoms, Sec. II and
    IV) at N = 2^8 .. 2^15 on one GPU: the time to form L by Eq. (10)'s
    ten-term series (the counterpart of Table I) and the time per step
    rho <- L rho L^dag (of Table II, whose totals are over unstated step
    counts), in FP64 and in split-BF16 (rotating frame)."""
    import torch
    rows = []
    for n in ns:
        w = ti.workload_paper(n)
        inst = w.instances[0]
        m = pipeline.model_of(inst)
        k, dt, D = n, w.dt, 1 << n
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = pipeline.sector_hamiltonian(m, k)
        torch.cuda.synchronize()
        t_h = time.perf_counter() - t0
        L = torch.empty((D, D), dtype=torch.complex128, device="cuda")
        ws = torch.empty(tcm.tc_expm_workspace_size(D, tcm.TC_EXPM_TAYLOR10),
                         dtype=torch.uint8, device="cuda")
        tcm.tc_expm(H, dt, 0.0, 0.0, L, tcm.TC_EXPM_TAYLOR10, ws=ws)     # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tcm.tc_expm(H, dt, 0.0, 0.0, L, tcm.TC_EXPM_TAYLOR10, ws=ws)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - t0
        del ws, H
        row = {"n": n, "N": D, "hamiltonian_ms": 1e3 * t_h, "taylor10_ms": 1e3 * t_l}
        for key, mode, frame, dtype in (
                ("fp64", tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB, torch.complex128),
                ("split", tcm.TC_GEMM_SPLIT_BF16, tcm.TC_FRAME_ROTATING, torch.complex64)):
            steps = max(1, min(20, int(3e14 / (12.0 * D ** 3) if key == "fp64"
                                       else 3e15 / (36.0 * D ** 3))))
            rho = torch.zeros((D, D), dtype=dtype, device="cuda")
            rho[0, 0] = 1.0                  # all excited: first state of the sector
            pipeline.evolve_sector(m, k, L, rho.clone(), 1, dt, mode, frame)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pop, _, _ = pipeline.evolve_sector(m, k, L, rho, steps, dt, mode, frame)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            row[key + "_ms_per_step"] = ms
            row[key + "_steps"] = steps
            row[key + "_tflops"] = 16.0 * D ** 3 / (ms * 1e-3) / 1e12
            fx = executed_flop_per_step(D, tile=128)
            row[key + "_tflops_executed"] = fx / (ms * 1e-3) / 1e12
            row[key + "_executed_frac_of_peak"] = (
                fx / (ms * 1e-3) / (PEAK_F64 if key == "fp64" else PEAK_BF16 / 3.0))
            row[key + "_final_excitation"] = float(pop[-1].item())
            del rho
        del L
        torch.cuda.empty_cache()
        rows.append(row)
        log(f"paper model n={n}: {row}")
    return {"workload": "tcm_paper_2n_sweep", "method": "Taylor-10 L (Eq. (10)), R = L^dag",
            "rows": rows}


def _host_cpu():
    """The host CPU as the OS names it: /proc/cpuinfo's model name, with the
    vendor, family, model and stepping numbers (a short model name alone may
    not say which part it is)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if info:
                        break
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("model name", "vendor_id", "cpu family", "model", "stepping") \
                        and k not in info:
                    info[k] = v
    except OSError:
        pass
    name = info.get("model name", "unknown")
    return (f"{name} ({info.get('vendor_id', '?')} family {info.get('cpu family', '?')} "
            f"model {info.get('model', '?')} stepping {info.get('stepping', '?')})")


def cpu_baseline(U_np, rho_np, min_s=20.0):
    """The oracle's dense step (rho <- U rho U^dag, numpy complex128 products on
    the host BLAS) on the N = 12288 matrices of the timed workload: whole steps,
    after a warm-up product on a row slab, until at least min_s seconds have
    passed (two steps on 16 threads).  One host thread is timed on a row slab
    of one step, scaled by N / rows, and labelled so."""
    from oracle import linalg as olin
    blas, threads = "numpy BLAS", None
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max((d.get("num_threads", 0) for d in info if d.get("user_api") == "blas"),
                      default=None)
        libs = [f"{d.get('internal_api', '')} {d.get('version', '')}".strip()
                for d in info if d.get("user_api") == "blas"]
        if libs:
            blas = ", ".join(libs)
    except Exception:
        pass
    affinity = len(os.sched_getaffinity(0))
    N = U_np.shape[0]
    olin.gemm(U_np[:512], rho_np)                       # warm-up: BLAS threads up
    steps, t0 = 0, time.perf_counter()
    rho = rho_np
    while True:
        X = olin.gemm(U_np, rho)
        rho = olin.gemm(X, U_np, op_b="h")
        del X
        steps += 1
        elapsed = time.perf_counter() - t0
        if elapsed >= min_s:
            break
    out = {"value": steps / elapsed, "unit": "steps/s",
           "cores": int(threads) if threads else affinity, "kind": "oracle",
           "sample": f"{steps} whole steps of the N={N} workload (U rho U^dag, numpy complex128 "
                     f"products, 16 N^3 = {16.0 * N ** 3:.3g} flop each) after a 512-row "
                     f"warm-up product, {elapsed:.2f} s",
           "s_per_step": elapsed / steps,
           "gflops": 16.0 * N ** 3 * steps / elapsed / 1e9,
           "blas_threads": threads, "affinity_cpus": affinity,
           "cpu": _host_cpu(), "blas": blas}
    del rho
    # one thread, on a row slab of one step sized to about 8 s
    try:
        from threadpoolctl import threadpool_limits

        def slab(rows):
            t = time.perf_counter()
            X = olin.gemm(U_np[:rows], rho_np)
            olin.gemm(X, U_np, op_b="h")
            return time.perf_counter() - t
        with threadpool_limits(limits=1):
            r1 = 64
            t1 = slab(r1)
            r1 = int(min(N, max(64, r1 * 8.0 / t1 // 64 * 64)))
            t1 = slab(r1)
        out["single_core"] = {"value": 1.0 / (t1 * N / r1), "unit": "steps/s",
                              "sample": f"rows 0..{r1 - 1} of one step, {t1:.2f} s on 1 thread, "
                                        f"scaled by N/rows (extrapolated, not a whole step)"}
    except Exception as e:   # threadpoolctl missing or unable to limit the BLAS
        out["single_core"] = {"value": None, "note": f"not measured: {e}"}
    return out


def parity_errors(inst, dt, runs):
    """Max-entry and population error of each timed run against the oracle's
    exact evolution of the same pure state (per-sector eigendecomposition of
    H), after the same number of steps: max_ij |rho_ij - psi_i conj(psi_j)|
    over the whole final matrix and max over every record of
    |sum_i <s_i^+ s_i^-> - oracle|."""
    import numpy as np
    from oracle import evolve as oev
    from oracle import model as omodel
    P = oev.SectorPropagator(inst.n, inst.c, inst.g, inst.omega_a)
    O = sum(omodel.atom_excitation_diag(inst.n, inst.c, i) for i in range(inst.n))
    out = {}
    for key, (rho_dev, pop_dev, steps) in runs.items():
        psi = P.psi(inst.psi0, steps * dt)
        rho = rho_dev.cpu().numpy()
        err = 0.0
        for r0 in range(0, psi.size, 1024):
            blk = rho[r0:r0 + 1024].astype(np.complex128)
            err = max(err, float(np.max(np.abs(blk - np.outer(psi[r0:r0 + 1024], psi.conj())))))
        del rho
        pop = pop_dev.cpu().numpy()
        perr = max(abs(pop[k] - float(np.sum(O * np.abs(P.psi(inst.psi0, k * dt)) ** 2)))
                   for k in range(steps + 1))
        out[key] = {"steps": steps, "max_entry": err, "population": perr,
                    "bar": 1e-10 if key == "fp64" else 1e-5}
        log(f"{key}: max-entry error {err:.3e}, population error {perr:.3e} after {steps} steps")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--modes", default="split,fp64,fp32")
    ap.add_argument("--extras", default="jc3,n9,batch64,grad8,open11,dense12,sectors11,paper,share",
                    help="other workloads measured after the headline one ('' for none)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the "
                         "reference kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 1 << 30, "bytes_written": 1 << 30}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design, not a run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import tcm_inputs as ti
    import paper_2403_06937_amd as tcm
    from paper_2403_06937_amd import pipeline

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tcm.lib()
    w = ti.get("n11")
    inst = w.instances[0]
    N, dt, renorm = inst.N, w.dt, w.renorm_every
    model = pipeline.model_of(inst)
    rho0 = inst.rho0()
    flop_alg = 16.0 * float(N) ** 3           # two complex N^3 products per step

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H, U = pipeline.propagator(model, dt)
    torch.cuda.synchronize()
    expm_s = time.perf_counter() - t0
    del H
    torch.cuda.empty_cache()
    log(f"U formed in {expm_s:.2f} s")

    K, W = args.steps, args.warmup
    res = {}
    modes = args.modes.split(",")
    if "split" in modes:
        res["split"] = run_mode(tcm, pipeline, model, U, rho0, tcm.TC_GEMM_SPLIT_BF16,
                                tcm.TC_FRAME_ROTATING, torch.complex64, K, W, dt, renorm)
        log(f"split-bf16: {res['split']['ms_total'] / K:.2f} ms/step")
    if "fp64" in modes:
        K64 = max(2, K // 8)
        res["fp64"] = run_mode(tcm, pipeline, model, U, rho0, tcm.TC_GEMM_F64, tcm.TC_FRAME_LAB,
                               torch.complex128, K64, 1, dt, renorm)
        res["fp64"]["steps"] = K64
        log(f"fp64: {res['fp64']['ms_total'] / K64:.2f} ms/step")
    if "fp32" in modes:
        K32 = max(4, K // 4)
        res["fp32"] = run_mode(tcm, pipeline, model, U, rho0, tcm.TC_GEMM_F32,
                               tcm.TC_FRAME_ROTATING, torch.complex64, K32, 1, dt, renorm)
        res["fp32"]["steps"] = K32
        log(f"fp32: {res['fp32']['ms_total'] / K32:.2f} ms/step")

    flop_exec = executed_flop_per_step(N)

    def summary(r, steps):
        ms = r["ms_total"] / steps
        return {"steps_per_s": 1000.0 / ms, "ms_per_step": ms,
                "tflops": flop_alg / (ms * 1e-3) / 1e12,
                "tflops_executed": flop_exec / (ms * 1e-3) / 1e12,
                "product_kernel_ms": r["kernel_ms"] / max(1, r["kernel_launches"]),
                "product_launches": r["kernel_launches"], "steps": steps}

    out = {"metric": METRIC, "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": W,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    head = "split" if "split" in res else list(res)[0]
    hs = summary(res[head], K if head == "split" else res[head]["steps"])
    out["value"] = hs["steps_per_s"]
    out["ms_per_step"] = hs["ms_per_step"]
    out["dtype"] = {"split": "bf16", "fp64": "f64", "fp32": "f32"}[head]
    out["config"] = {"workload": w.name, "N": N, "n_atoms": inst.n, "photon_cutoff": inst.c,
                     "dt": dt, "renorm_every": renorm, "record_every": 1,
                     "products": {"split": "split-BF16 hi/lo 3-term, FP32 accumulate, rotating frame",
                                  "fp64": "complex FP64", "fp32": "complex FP32"}[head],
                     "parallelism": "single GPU"}
    # tflops counts 16 N^3 per step (two full complex products, the method's
    # count); tflops_executed counts what the kernels multiply (the second
    # product's result is Hermitian, so only its upper tile triangle is formed)
    out["tflops"] = hs["tflops"]
    out["tflops_executed"] = hs["tflops_executed"]
    for k in ("fp64", "fp32", "split"):
        if k in res and k != head:
            out[k] = summary(res[k], res[k]["steps"])
    out["expm_s"] = expm_s

    # roofline of the dominant kernel (the complex product), from live events:
    # a "launch" here is one complex N x N x N product, 8 N^3 flop on the
    # method's count (for the upper tile triangle of the second product: its
    # main launch and the split-K pair of its last round, timed together); the
    # products alternate between the full first product and that triangle, so
    # a product executes flop_exec / 2 on average, and the split form issues
    # three BF16 products per real product
    kern_ms = hs["product_kernel_ms"]
    per_launch_alg = 8.0 * float(N) ** 3
    per_launch_exec = flop_exec / 2.0
    achieved = per_launch_alg / (kern_ms * 1e-3)
    peak = {"split": PEAK_BF16, "fp64": PEAK_F64, "fp32": PEAK_F32}[head]
    src = os.path.join(ROOT, "paper_2403_06937_amd", "csrc",
                       "gemm_bf16.hip" if head == "split" else "gemm_mfma.hip")
    kname = "split_gemm_kernel" if head == "split" else "gemm_kernel"
    exec_frac = per_launch_exec / (kern_ms * 1e-3) / peak
    out["roofline"] = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                       "unit": "TFLOP/s", "frac": achieved / peak,
                       "traffic": traffic_entry(kname, w.name, src),
                       "kernel": kname, "kernel_ms": kern_ms,
                       "algorithmic_flop_per_launch": per_launch_alg,
                       "executed_flop_per_launch": per_launch_exec,
                       "executed_frac": exec_frac,
                       "issued_frac": (3.0 if head == "split" else 1.0) * exec_frac,
                       "mfma_probe": mfma_probe_or_none(tcm)}

    if not args.no_cpu:
        # the CPU leg, the one part of the benchmark that runs the oracle: first
        # the errors of the timed runs against its exact evolution, then its own
        # dense step timed on the host cores
        out["error"] = parity_errors(inst, dt, {k: (res[k]["rho"], res[k]["pop"],
                                                    K if k == "split" else res[k]["steps"])
                                                for k in res})
        for k in list(res):
            del res[k]["rho"], res[k]["pop"]
        torch.cuda.empty_cache()
        U_np = U.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(U_np, rho0)
        del U_np
    res.clear()
    del U
    torch.cuda.empty_cache()
    extras = [e for e in args.extras.split(",") if e]
    if extras:
        out["other_workloads"] = {}
    for e in extras:
        fn = {"jc3": bench_jc3, "n9": bench_n9, "batch64": bench_batch64, "grad8": bench_grad8,
              "open11": bench_open11, "dense12": bench_dense12,
              "sectors11": bench_sectors11, "paper": bench_paper_sweep,
              "share": bench_share}[e]
        out["other_workloads"][e] = fn(tcm, pipeline, ti)
        log(f"{e}: {out['other_workloads'][e]}")
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
