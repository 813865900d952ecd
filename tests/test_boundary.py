"""Boundary tests that need no GPU: the C-ABI library loads, exports every
entry point include/tcm.h declares, and its host-only calls validate
arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import tcm_inputs as ti
from oracle import model as omodel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

tcm = pytest.importorskip("paper_2403_06937_amd")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tcm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(tc_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = tcm.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(tcm.EXPORTED)


def test_version_and_dim():
    assert tcm.tc_version() == 120
    assert tcm.tc_dim(3, 3) == 32
    assert tcm.tc_dim(11, 5) == 12288
    assert tcm.tc_dim(1, 0) == 2


@pytest.mark.parametrize("n,c", [(0, 3), (-1, 1), (25, 1), (3, -1), (24, 20)])
def test_dim_rejects(n, c):
    with pytest.raises(tcm.TcmError) as e:
        tcm.tc_dim(n, c)
    assert e.value.code == tcm.TC_ERR_INVALID_ARGUMENT
    assert "invalid argument" in str(e.value)


@pytest.mark.parametrize("n,c,seed", [(1, 3, 0), (3, 3, 1), (5, 2, 2), (2, 0, 3)])
def test_spectral_bounds_contain_spectrum(n, c, seed):
    """Gershgorin interval from the host call contains every eigenvalue of the
    oracle's H and equals the row-wise centre -/+ radius bounds."""
    inst = ti.random_model(n, c, seed)
    m = tcm.Model(n, c, inst.g, inst.omega_a)
    lo, hi = tcm.tc_spectral_bounds(m)
    H = omodel.hamiltonian(n, c, inst.g, inst.omega_a)
    ev = np.linalg.eigvalsh(H)
    assert lo <= ev.min() + 1e-12 and ev.max() <= hi + 1e-12
    d = np.diagonal(H)
    rad = np.sum(np.abs(H), axis=1) - np.abs(d)
    assert abs(lo - np.min(d - rad)) < 1e-12 and abs(hi - np.max(d + rad)) < 1e-12


def test_argument_errors_before_device_work():
    L = tcm.lib()
    m = tcm.Model(2, 1, [0.01, 0.02], [1.0, 1.0])
    # NULL H
    assert L.tc_build_hamiltonian(ctypes.byref(m.struct), None, 8, None) == tcm.TC_ERR_INVALID_ARGUMENT
    # ld < N
    assert L.tc_build_hamiltonian(ctypes.byref(m.struct), 0x1000, 4, None) == tcm.TC_ERR_INVALID_ARGUMENT
    assert b"ldh" in L.tc_last_error()
    # unknown expm method
    sz = ctypes.c_size_t()
    assert L.tc_expm_workspace_size(8, 7, ctypes.byref(sz)) == tcm.TC_ERR_INVALID_ARGUMENT
    # workspace too small
    assert L.tc_expm_workspace_size(8, tcm.TC_EXPM_SS_TAYLOR, ctypes.byref(sz)) == 0
    assert sz.value > 0
    rc = L.tc_expm(0x1000, 8, 8, 0.1, 0.0, 1.0, tcm.TC_EXPM_SS_TAYLOR, 0x2000, 8, 0x3000,
                   sz.value - 1, None)
    assert rc == tcm.TC_ERR_WORKSPACE
    # non-finite dt, inverted bounds
    assert L.tc_expm(0x1000, 8, 8, float("nan"), 0.0, 1.0, 0, 0x2000, 8, 0x3000, sz.value,
                     None) == tcm.TC_ERR_INVALID_ARGUMENT
    assert L.tc_expm(0x1000, 8, 8, 0.1, 1.0, 0.0, 0, 0x2000, 8, 0x3000, sz.value,
                     None) == tcm.TC_ERR_INVALID_ARGUMENT


def test_evolve_argument_errors():
    m = tcm.Model(2, 1, [0.01, 0.02], [1.0, 1.0])
    N = m.N

    class Fake:
        def __init__(self, p, ld):
            self.p, self.ld = p, ld

        def data_ptr(self):
            return self.p

        def stride(self, i):
            return self.ld

    U, rho = Fake(0x1000, N), Fake(0x2000, N)
    inst = tcm.make_instance(m, U, rho)
    for bad in [dict(steps=-1), dict(gemm_mode=9), dict(rho_dtype=7), dict(frame=3),
                dict(renorm_every=-2), dict(record_every=-1)]:
        kw = dict(steps=10, dt=0.1)
        kw.update(bad)
        with pytest.raises(tcm.TcmError) as e:
            tcm.tc_evolve_workspace_size([inst], tcm.make_opts(**kw))
        assert e.value.code == tcm.TC_ERR_INVALID_ARGUMENT
    # records requested with record_every = 0
    inst2 = tcm.make_instance(m, U, rho, pop_out=Fake(0x3000, 1))
    with pytest.raises(tcm.TcmError):
        tcm.tc_evolve_workspace_size([inst2], tcm.make_opts(10, 0.1, record_every=0))
    # wrong N
    inst3 = tcm.make_instance(m, U, rho)
    inst3.N = N + 1
    with pytest.raises(tcm.TcmError):
        tcm.tc_evolve_workspace_size([inst3], tcm.make_opts(10, 0.1))
    # workspace too small -> TC_ERR_WORKSPACE, nothing launched
    need = tcm.tc_evolve_workspace_size([inst], tcm.make_opts(10, 0.1))
    arr = (tcm.tc_instance * 1)(inst)
    opts = tcm.make_opts(10, 0.1)
    rc = tcm.lib().tc_evolve(arr, 1, ctypes.byref(opts), 0x4000, need - 1, None)
    assert rc == tcm.TC_ERR_WORKSPACE


def test_workspace_sizes_scale():
    a = tcm.tc_expm_workspace_size(1024)
    b = tcm.tc_expm_workspace_size(2048)
    assert 3.9 < b / a < 4.1
    assert tcm.tc_gemm_workspace_size(64, 64, 64, tcm.TC_GEMM_F64) == 0
    assert tcm.tc_gemm_workspace_size(64, 64, 64, tcm.TC_GEMM_SPLIT_BF16) > 0


def test_dissipation_rates_checked_before_device_work():
    """Negative or non-finite kappa / gamma are argument errors; the adjoint
    rejects a model with a Lindblad term (it covers the unitary step only)."""
    class Fake:
        def __init__(self, p, ld):
            self.p, self.ld = p, ld

        def data_ptr(self):
            return self.p

        def stride(self, i):
            return self.ld

    for kappa, gamma in [(-0.1, 0.0), (0.0, -1e-3), (float("nan"), 0.0), (0.0, float("inf"))]:
        m = tcm.Model(2, 1, [0.01, 0.02], [1.0, 1.0], kappa=kappa, gamma=gamma)
        inst = tcm.make_instance(m, Fake(0x1000, m.N), Fake(0x2000, m.N))
        with pytest.raises(tcm.TcmError) as e:
            tcm.tc_evolve_workspace_size([inst], tcm.make_opts(10, 0.1))
        assert e.value.code == tcm.TC_ERR_INVALID_ARGUMENT
    ok = tcm.Model(2, 1, [0.01, 0.02], [1.0, 1.0], kappa=0.1, gamma=0.2)
    inst = tcm.make_instance(ok, Fake(0x1000, ok.N), Fake(0x2000, ok.N))
    assert tcm.tc_evolve_workspace_size([inst], tcm.make_opts(10, 0.1)) > 0
    sz = ctypes.c_size_t()
    opts = tcm.make_opts(10, 0.1, checkpoint_every=5)
    rc = tcm.lib().tc_evolve_backward_workspace_size(ctypes.byref(ok.struct), ok.N,
                                                     ctypes.byref(opts), ctypes.byref(sz))
    assert rc == tcm.TC_ERR_UNSUPPORTED


def test_sector_option_validation_and_workspace():
    """opts.sectors: only 0 / 1; the workspace holds rho and X in the padded
    sorted order, the padded U blocks (sum_k D_k^2 elements) and the three
    index maps."""
    from math import comb
    n, c = 5, 2
    m = tcm.Model(n, c, [0.01] * n, [1.0] * n)
    N = m.N

    class Fake:
        def __init__(self, p, ld):
            self.p, self.ld = p, ld

        def data_ptr(self):
            return self.p

        def stride(self, i):
            return self.ld

    inst = tcm.make_instance(m, Fake(0x1000, N), Fake(0x2000, N))
    with pytest.raises(tcm.TcmError) as e:
        tcm.tc_evolve_workspace_size([inst], tcm.make_opts(10, 0.1, sectors=2))
    assert e.value.code == tcm.TC_ERR_INVALID_ARGUMENT
    # split-BF16 by sectors pads every sector to the 128 tile
    wsp = tcm.tc_evolve_workspace_size([inst], tcm.make_opts(10, 0.1, tcm.TC_GEMM_SPLIT_BF16,
                                                             tcm.TC_C64, sectors=1))
    assert wsp > 0
    ws = tcm.tc_evolve_workspace_size([inst], tcm.make_opts(10, 0.1, sectors=1))
    d = [sum(comb(n, k - mm) for mm in range(min(k, c) + 1) if k - mm <= n)
         for k in range(n + c + 1)]
    assert sum(d) == N
    # each sector padded to a multiple of the product tile edge (64 at this N)
    q = 128 if tcm.tc_autotune_query(tcm.TC_GEMM_F64, N) == 1 else 64
    D = [-(-x // q) * q for x in d]
    Np = sum(D)
    need = 2 * Np * Np * 16 + sum(x * x for x in D) * 16 + 2 * Np * 4 + N * 4
    assert need <= ws <= need + 64 * 1024


def test_sector_entry_points_host_side():
    """tc_sector_dim / tc_sector_states against the oracle's sectors; the
    one-sector workspace query refuses a Lindblad model, a wrong N and
    opts.sectors, and sizes the block's buffers plus the state map."""
    from oracle import model as omodel
    n, c = 4, 3
    m = tcm.Model(n, c, [0.01] * n, [1.0] * n)
    secs = omodel.sectors(n, c)
    for k in range(n + c + 1):
        assert tcm.tc_sector_dim(m, k) == secs[k].size
        assert np.array_equal(tcm.tc_sector_states(m, k), secs[k])
    for k in (-1, n + c + 1):
        with pytest.raises(tcm.TcmError):
            tcm.tc_sector_dim(m, k)

    class Fake:
        def __init__(self, p, ld):
            self.p, self.ld = p, ld

        def data_ptr(self):
            return self.p

        def stride(self, i):
            return self.ld

    d = secs[3].size
    inst = tcm.make_instance(m, Fake(0x1000, d), Fake(0x2000, d))
    inst.N = d
    ws = tcm.tc_evolve_sector_workspace_size(inst, 3, tcm.make_opts(10, 0.1))
    assert ws >= d * d * 16 + m.N * 4
    inst.N = d + 1
    with pytest.raises(tcm.TcmError) as e:
        tcm.tc_evolve_sector_workspace_size(inst, 3, tcm.make_opts(10, 0.1))
    assert e.value.code == tcm.TC_ERR_INVALID_ARGUMENT
    inst.N = d
    with pytest.raises(tcm.TcmError) as e:
        tcm.tc_evolve_sector_workspace_size(inst, 3, tcm.make_opts(10, 0.1, sectors=1))
    assert e.value.code == tcm.TC_ERR_INVALID_ARGUMENT
    mo = tcm.Model(n, c, [0.01] * n, [1.0] * n, kappa=0.1)
    inst2 = tcm.make_instance(mo, Fake(0x1000, d), Fake(0x2000, d))
    inst2.N = d
    with pytest.raises(tcm.TcmError) as e:
        tcm.tc_evolve_sector_workspace_size(inst2, 3, tcm.make_opts(10, 0.1))
    assert e.value.code == tcm.TC_ERR_UNSUPPORTED


def test_noalloc_observables_rejects_before_device_work():
    """The allocation-free readout refuses a matrix whose partial sums exceed
    its device array, and bad arguments, before it touches a device (no GPU
    needed: the pointers are never dereferenced)."""
    L = tcm.lib()
    N = ctypes.c_int64()
    assert L.tc_observables_noalloc_max_dim(ctypes.byref(N)) == tcm.TC_OK
    assert N.value == 37120
    big = tcm.Model(12, 9, [0.01] * 12, [1.0] * 12)          # N = 40960
    rc = L.tc_observables_noalloc(ctypes.byref(big.struct), 0x1000, tcm.TC_C64, big.N, big.N,
                                  0x2000, None, None, None, None, None, None)
    assert rc == tcm.TC_ERR_UNSUPPORTED
    assert b"use tc_observables" in L.tc_last_error()
    m = tcm.Model(3, 2, [0.01] * 3, [1.0] * 3)
    assert L.tc_observables_noalloc(ctypes.byref(m.struct), 0x1000, tcm.TC_C64, m.N, m.N - 1,
                                    0x2000, None, None, None, None, None,
                                    None) == tcm.TC_ERR_INVALID_ARGUMENT
    assert L.tc_observables_noalloc(ctypes.byref(m.struct), 0x1000, 9, m.N, m.N, 0x2000, None,
                                    None, None, None, None, None) == tcm.TC_ERR_INVALID_ARGUMENT
    assert L.tc_observables_noalloc(ctypes.byref(m.struct), 0x1000, tcm.TC_C64, m.N, m.N, None,
                                    None, None, None, None, None,
                                    None) == tcm.TC_ERR_INVALID_ARGUMENT


def test_mfma_probe_rejects_before_device_work():
    """Argument errors of the MFMA rate probe come back before any HIP call."""
    L = tcm.lib()
    ms, fl = ctypes.c_double(), ctypes.c_double()
    assert L.tc_mfma_probe(7, 1, 100, None, 0, ctypes.byref(ms), ctypes.byref(fl),
                           None) == tcm.TC_ERR_INVALID_ARGUMENT
    assert L.tc_mfma_probe(tcm.TC_PROBE_F64_16X16X4, 1, 0, None, 0, ctypes.byref(ms),
                           ctypes.byref(fl), None) == tcm.TC_ERR_INVALID_ARGUMENT
    assert L.tc_mfma_probe(tcm.TC_PROBE_F64_16X16X4, 1, 10, None, 0, ctypes.byref(ms),
                           ctypes.byref(fl), None) == tcm.TC_ERR_INVALID_ARGUMENT
    assert b"iters" in L.tc_last_error() or b"NULL" in L.tc_last_error()
