"""tc_observables_noalloc (the readout for callers that cannot allocate: its
partial sums live in the library's own device array) against tc_observables
with a caller workspace: the same kernels in the same order, so every output
is bitwise equal, on two calls in a row, the second on a smaller matrix, and
with a matrix too large for the array rejected before any device work."""
import numpy as np
import pytest
import torch

import tcm_inputs as ti

pytestmark = pytest.mark.gpu

tcm = pytest.importorskip("paper_2403_06937_amd")


def _outputs(model, device="cuda"):
    ns = min(model.n, model.c) + 1
    z = lambda k: torch.full((k,), -7.0, dtype=torch.float64, device=device)  # noqa: E731
    return [z(8), z(model.n), z(model.c + 1), z(model.n + model.c + 1), z(ns), z(ns)]


def _both(model, rho):
    a = _outputs(model)
    tcm.tc_observables(model, rho, *a)
    b = _outputs(model)
    tcm.tc_observables_noalloc(model, rho, *b)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in a], [x.cpu().numpy() for x in b]


def test_noalloc_equals_workspace_readout():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert tcm.tc_observables_noalloc_max_dim() == 37120
    # first call: the N = 12288 shape (n = 11, c = 5) in complex64; second: a
    # smaller ragged one (n = 5, c = 2, N = 96) in complex128, so the second
    # call reads partials that the first one left larger
    cases = [(11, 5, torch.complex64, 3), (5, 2, torch.complex128, 2)]
    for n, c, dtype, rank in cases:
        inst = ti.random_model(n, c, 40 + n)
        m = tcm.Model(n, c, inst.g, inst.omega_a)
        rho = torch.from_numpy(ti.random_density(m.N, 41 + n, rank=rank)).to("cuda").to(dtype)
        a, b = _both(m, rho)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), (n, c)
        assert np.all(b[0][:7] != -7.0) and b[0][7] == 0.0
        print(f"noalloc n={n} c={c}: trace {b[0][0]:.15f}, purity {b[0][2]:.6f}", flush=True)
    # beyond the array: refused with a clear error before any device work
    # (the matrix pointer is never dereferenced), the outputs untouched
    import ctypes
    big = tcm.Model(12, 9, [0.01] * 12, [1.0] * 12)          # N = 40960 > 37120
    s = torch.full((8,), -7.0, dtype=torch.float64, device="cuda")
    rc = tcm.lib().tc_observables_noalloc(ctypes.byref(big.struct), 0x1000, tcm.TC_C64, big.N,
                                          big.N, s.data_ptr(), None, None, None, None, None,
                                          None)
    assert rc == tcm.TC_ERR_UNSUPPORTED
    assert b"use tc_observables" in tcm.lib().tc_last_error()
    torch.cuda.synchronize()
    assert torch.all(s == -7.0)
