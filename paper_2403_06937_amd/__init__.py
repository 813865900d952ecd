"""Python binding of libtcm, the MI355X Tavis-Cummings density-matrix stepper.

Thin ctypes layer over the C ABI in include/tcm.h: every function below has
the name of the C entry point it marshals to and does no arithmetic of its
own.  Device memory and streams come from PyTorch (torch tensors on a ROCm
device); all work runs in the library's HIP kernels.  If libtcm.so has not
been built, every call raises TcmUnavailable -- there is no fallback path.

Model of the paper (arXiv 2403.06937, Sec. II, Eq. (4)): n two-level atoms
in one cavity mode with photon cutoff c, hbar = 1, basis order photon-major
|m>|l_1..l_n> with atom 1 the most significant bit.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtcm.so")

TC_OK = 0
TC_ERR_INVALID_ARGUMENT = 1
TC_ERR_UNSUPPORTED = 2
TC_ERR_WORKSPACE = 3
TC_ERR_HIP = 4
TC_ERR_NONFINITE = 5

TC_C64 = 1
TC_C128 = 2
TC_GEMM_F64 = 0
TC_GEMM_F32 = 1
TC_GEMM_SPLIT_BF16 = 2
TC_EXPM_SS_TAYLOR = 0
TC_EXPM_TAYLOR10 = 1
TC_FRAME_LAB = 0
TC_FRAME_ROTATING = 1
TC_OBS_EXCITED_TOTAL = 0

EXPORTED = [
    "tc_version", "tc_last_error", "tc_dim", "tc_spectral_bounds", "tc_build_hamiltonian",
    "tc_expm_workspace_size", "tc_expm", "tc_evolve_workspace_size", "tc_evolve",
    "tc_observables_workspace_size", "tc_observables", "tc_evolve_backward_workspace_size",
    "tc_evolve_backward", "tc_gemm_workspace_size", "tc_zgemm", "tc_split_bf16",
    "tc_profile_enable", "tc_profile_read", "tc_autotune_workspace_size", "tc_autotune",
    "tc_autotune_query", "tc_sector_dim", "tc_sector_states", "tc_sector_spectral_bounds",
    "tc_build_sector_hamiltonian", "tc_evolve_sector_workspace_size", "tc_evolve_sector",
    "tc_observables_noalloc_max_dim", "tc_observables_noalloc", "tc_mfma_probe",
]

TC_KERNEL_GEMM_F64 = 0
TC_KERNEL_GEMM_F32 = 1
TC_KERNEL_SPLIT_BF16 = 2
TC_PROBE_BF16_16X16X32 = 0
TC_PROBE_BF16_32X32X16 = 1
TC_PROBE_F64_16X16X4 = 2


class TcmUnavailable(RuntimeError):
    pass


class TcmError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} failed with code {code}: {msg}")
        self.code = code


class tc_c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class tc_model(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("photon_cutoff", ctypes.c_int32),
                ("omega_c", ctypes.c_double), ("omega_a", ctypes.POINTER(ctypes.c_double)),
                ("g", ctypes.POINTER(ctypes.c_double)), ("kappa", ctypes.c_double),
                ("gamma", ctypes.c_double)]


class tc_instance(ctypes.Structure):
    _fields_ = [("model", ctypes.POINTER(tc_model)), ("N", ctypes.c_int64),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64),
                ("rho", ctypes.c_void_p), ("ldr", ctypes.c_int64),
                ("pop_out", ctypes.c_void_p), ("photon_dist_out", ctypes.c_void_p),
                ("checkpoints", ctypes.c_void_p), ("photon_state_out", ctypes.c_void_p)]


class tc_evolve_opts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("dt", ctypes.c_double),
                ("gemm_mode", ctypes.c_int32), ("rho_dtype", ctypes.c_int32),
                ("frame", ctypes.c_int32), ("renorm_every", ctypes.c_int32),
                ("record_every", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("full_product", ctypes.c_int32),
                ("no_resident", ctypes.c_int32), ("sectors", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libtcm (ctypes.CDLL); raises TcmUnavailable if not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TcmUnavailable(f"{LIB_PATH} is missing: build it with "
                                 "`python -m paper_2403_06937_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sz = ctypes.c_size_t
        P = ctypes.POINTER
        L.tc_version.restype = ctypes.c_int
        L.tc_last_error.restype = ctypes.c_char_p
        sig = {
            "tc_dim": [i32, i32, P(i64)],
            "tc_spectral_bounds": [P(tc_model), P(f64), P(f64)],
            "tc_build_hamiltonian": [P(tc_model), vp, i64, vp],
            "tc_expm_workspace_size": [i64, i32, P(sz)],
            "tc_expm": [vp, i64, i64, f64, f64, f64, i32, vp, i64, vp, sz, vp],
            "tc_evolve_workspace_size": [P(tc_instance), i32, P(tc_evolve_opts), P(sz)],
            "tc_evolve": [P(tc_instance), i32, P(tc_evolve_opts), vp, sz, vp],
            "tc_observables_workspace_size": [i64, P(sz)],
            "tc_observables": [P(tc_model), vp, i32, i64, i64, vp, vp, vp, vp, vp, vp, vp, sz,
                               vp],
            "tc_evolve_backward_workspace_size": [P(tc_model), i64, P(tc_evolve_opts), P(sz)],
            "tc_evolve_backward": [P(tc_model), vp, i64, vp, i64, i64, P(tc_evolve_opts), vp,
                                   i32, vp, vp, vp, vp, sz, vp],
            "tc_gemm_workspace_size": [i64, i64, i64, i32, P(sz)],
            "tc_zgemm": [i64, i64, i64, tc_c128, vp, i64, i32, vp, i64, i32, tc_c128, vp, i64,
                         i32, vp, sz, vp],
            "tc_split_bf16": [vp, i64, vp, vp, vp],
            "tc_profile_enable": [i32],
            "tc_profile_read": [i32, P(f64), P(i64)],
            "tc_autotune_workspace_size": [i32, i64, P(sz)],
            "tc_autotune": [i32, i64, vp, sz, vp],
            "tc_autotune_query": [i32, i64, P(i32)],
            "tc_sector_dim": [P(tc_model), i32, P(i64)],
            "tc_sector_states": [P(tc_model), i32, vp],
            "tc_sector_spectral_bounds": [P(tc_model), i32, P(f64), P(f64)],
            "tc_build_sector_hamiltonian": [P(tc_model), i32, vp, i64, vp],
            "tc_evolve_sector_workspace_size": [P(tc_instance), i32, P(tc_evolve_opts), P(sz)],
            "tc_evolve_sector": [P(tc_instance), i32, P(tc_evolve_opts), vp, sz, vp],
            "tc_observables_noalloc_max_dim": [P(i64)],
            "tc_observables_noalloc": [P(tc_model), vp, i32, i64, i64, vp, vp, vp, vp, vp, vp,
                                       vp],
            "tc_mfma_probe": [i32, i32, i32, vp, i64, P(f64), P(f64), vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code: int, func: str):
    if code != TC_OK:
        raise TcmError(code, func, lib().tc_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream=None):
    if stream is not None:
        return int(stream)
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes: int, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class Model:
    """Host description of one instance of Eq. (4)."""
    n: int
    c: int
    g: Sequence[float]
    omega_a: Sequence[float]
    omega_c: float = 1.0
    kappa: float = 0.0            # cavity leakage rate of the Lindblad term
    gamma: float = 0.0            # atomic emission rate of the Lindblad term

    def __post_init__(self):
        self._g = np.ascontiguousarray(self.g, dtype=np.float64)
        self._wa = np.ascontiguousarray(self.omega_a, dtype=np.float64)
        self._s = tc_model(self.n, self.c, float(self.omega_c),
                           self._wa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           self._g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           float(self.kappa), float(self.gamma))

    @property
    def N(self) -> int:
        return tc_dim(self.n, self.c)

    @property
    def struct(self):
        return self._s


# ---------------------------------------------------------------- C entry points

def tc_version() -> int:
    return lib().tc_version()


def tc_dim(n: int, c: int) -> int:
    N = ctypes.c_int64()
    _check(lib().tc_dim(n, c, ctypes.byref(N)), "tc_dim")
    return N.value


def tc_spectral_bounds(model: Model):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().tc_spectral_bounds(ctypes.byref(model.struct), ctypes.byref(lo),
                                    ctypes.byref(hi)), "tc_spectral_bounds")
    return lo.value, hi.value


def tc_build_hamiltonian(model: Model, H, stream=None):
    """H: torch.float64 device tensor (N x ldh, row-major)."""
    _check(lib().tc_build_hamiltonian(ctypes.byref(model.struct), _ptr(H), H.stride(0),
                                      _stream(stream)), "tc_build_hamiltonian")


def tc_expm_workspace_size(N: int, method: int = TC_EXPM_SS_TAYLOR) -> int:
    b = ctypes.c_size_t()
    _check(lib().tc_expm_workspace_size(N, method, ctypes.byref(b)), "tc_expm_workspace_size")
    return b.value


def tc_expm(H, dt: float, lam_lo: float, lam_hi: float, U, method: int = TC_EXPM_SS_TAYLOR,
            ws=None, stream=None):
    """U = exp(-i H dt): H float64 (N x N), U complex128 (N x N), device tensors."""
    N = H.shape[0]
    need = tc_expm_workspace_size(N, method)
    if ws is None:
        ws = _workspace(need, H.device)
    _check(lib().tc_expm(_ptr(H), N, H.stride(0), dt, lam_lo, lam_hi, method, _ptr(U),
                         U.stride(0), _ptr(ws), ws.numel(), _stream(stream)), "tc_expm")


def make_opts(steps, dt, gemm_mode=TC_GEMM_F64, rho_dtype=TC_C128, frame=TC_FRAME_LAB,
              renorm_every=0, record_every=1, checkpoint_every=0, use_graph=0, full_product=0,
              sectors=0, no_resident=0):
    return tc_evolve_opts(int(steps), float(dt), gemm_mode, rho_dtype, frame, renorm_every,
                          record_every, checkpoint_every, use_graph, int(full_product),
                          int(no_resident), int(sectors))


def make_instance(model: Model, U, rho, pop_out=None, photon_dist_out=None, checkpoints=None,
                  photon_state_out=None):
    return tc_instance(ctypes.pointer(model.struct), model.N, _ptr(U), U.stride(0), _ptr(rho),
                       rho.stride(0), _ptr(pop_out), _ptr(photon_dist_out), _ptr(checkpoints),
                       _ptr(photon_state_out))


def tc_evolve_workspace_size(instances, opts) -> int:
    arr = (tc_instance * len(instances))(*instances)
    b = ctypes.c_size_t()
    _check(lib().tc_evolve_workspace_size(arr, len(instances), ctypes.byref(opts),
                                          ctypes.byref(b)), "tc_evolve_workspace_size")
    return b.value


def tc_evolve(instances, opts, ws=None, device=None, stream=None):
    """Steps each tc_instance (see make_instance) opts.steps times."""
    arr = (tc_instance * len(instances))(*instances)
    if ws is None:
        need = tc_evolve_workspace_size(instances, opts)
        ws = _workspace(need, device if device is not None else "cuda")
    _check(lib().tc_evolve(arr, len(instances), ctypes.byref(opts), _ptr(ws), ws.numel(),
                           _stream(stream)), "tc_evolve")


def tc_sector_dim(model: Model, k: int) -> int:
    d = ctypes.c_int64()
    _check(lib().tc_sector_dim(ctypes.byref(model.struct), int(k), ctypes.byref(d)),
           "tc_sector_dim")
    return d.value


def tc_sector_states(model: Model, k: int):
    """Basis indices of excitation sector k, increasing (numpy int64)."""
    import numpy as np
    out = np.zeros(tc_sector_dim(model, k), dtype=np.int64)
    _check(lib().tc_sector_states(ctypes.byref(model.struct), int(k),
                                  out.ctypes.data_as(ctypes.c_void_p)), "tc_sector_states")
    return out


def tc_sector_spectral_bounds(model: Model, k: int):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().tc_sector_spectral_bounds(ctypes.byref(model.struct), int(k), ctypes.byref(lo),
                                           ctypes.byref(hi)), "tc_sector_spectral_bounds")
    return lo.value, hi.value


def tc_build_sector_hamiltonian(model: Model, k: int, H, stream=None):
    """H: torch.float64 device tensor (d_k x ldh, row-major)."""
    _check(lib().tc_build_sector_hamiltonian(ctypes.byref(model.struct), int(k), _ptr(H),
                                             H.stride(0), _stream(stream)),
           "tc_build_sector_hamiltonian")


def tc_evolve_sector_workspace_size(instance, k: int, opts) -> int:
    b = ctypes.c_size_t()
    _check(lib().tc_evolve_sector_workspace_size(ctypes.byref(instance), int(k),
                                                 ctypes.byref(opts), ctypes.byref(b)),
           "tc_evolve_sector_workspace_size")
    return b.value


def tc_evolve_sector(instance, k: int, opts, ws=None, device=None, stream=None):
    """Steps one tc_instance whose matrices are the d_k x d_k blocks of sector k."""
    if ws is None:
        need = tc_evolve_sector_workspace_size(instance, k, opts)
        ws = _workspace(need, device if device is not None else "cuda")
    _check(lib().tc_evolve_sector(ctypes.byref(instance), int(k), ctypes.byref(opts), _ptr(ws),
                                  ws.numel(), _stream(stream)), "tc_evolve_sector")


def tc_observables_workspace_size(N: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().tc_observables_workspace_size(N, ctypes.byref(b)), "tc_observables_workspace_size")
    return b.value


def tc_observables(model: Model, rho, scalars, atom_pop=None, photon_dist=None, exc_dist=None,
                   photon_state=None, dicke=None, ws=None, stream=None):
    import torch
    dtype = TC_C128 if rho.dtype == torch.complex128 else TC_C64
    N = rho.shape[0]
    if ws is None:
        ws = _workspace(tc_observables_workspace_size(N), rho.device)
    _check(lib().tc_observables(ctypes.byref(model.struct), _ptr(rho), dtype, N, rho.stride(0),
                                _ptr(scalars), _ptr(atom_pop), _ptr(photon_dist),
                                _ptr(exc_dist), _ptr(photon_state), _ptr(dicke), _ptr(ws),
                                ws.numel(), _stream(stream)),
           "tc_observables")


def tc_observables_noalloc_max_dim() -> int:
    N = ctypes.c_int64()
    _check(lib().tc_observables_noalloc_max_dim(ctypes.byref(N)), "tc_observables_noalloc_max_dim")
    return N.value


def tc_observables_noalloc(model: Model, rho, scalars, atom_pop=None, photon_dist=None,
                           exc_dist=None, photon_state=None, dicke=None, stream=None):
    """tc_observables without a workspace (the library's own device array)."""
    import torch
    dtype = TC_C128 if rho.dtype == torch.complex128 else TC_C64
    _check(lib().tc_observables_noalloc(ctypes.byref(model.struct), _ptr(rho), dtype,
                                        rho.shape[0], rho.stride(0), _ptr(scalars),
                                        _ptr(atom_pop), _ptr(photon_dist), _ptr(exc_dist),
                                        _ptr(photon_state), _ptr(dicke), _stream(stream)),
           "tc_observables_noalloc")


def tc_evolve_backward_workspace_size(model: Model, opts) -> int:
    b = ctypes.c_size_t()
    _check(lib().tc_evolve_backward_workspace_size(ctypes.byref(model.struct), model.N,
                                                   ctypes.byref(opts), ctypes.byref(b)),
           "tc_evolve_backward_workspace_size")
    return b.value


def tc_evolve_backward(model: Model, H, U, opts, checkpoints, loss_out, grad_g, grad_delta,
                       ws=None, stream=None, observable=TC_OBS_EXCITED_TOTAL):
    if ws is None:
        ws = _workspace(tc_evolve_backward_workspace_size(model, opts), U.device)
    _check(lib().tc_evolve_backward(ctypes.byref(model.struct), _ptr(H), H.stride(0), _ptr(U),
                                    U.stride(0), model.N, ctypes.byref(opts), _ptr(checkpoints),
                                    observable, _ptr(loss_out), _ptr(grad_g), _ptr(grad_delta),
                                    _ptr(ws), ws.numel(), _stream(stream)), "tc_evolve_backward")


def tc_gemm_workspace_size(M, N, K, mode) -> int:
    b = ctypes.c_size_t()
    _check(lib().tc_gemm_workspace_size(M, N, K, mode, ctypes.byref(b)), "tc_gemm_workspace_size")
    return b.value


def tc_zgemm(A, B, C, op_a=0, op_b=0, alpha=1.0, beta=0.0, mode=TC_GEMM_F64, ws=None,
             stream=None):
    """C = alpha op(A) op(B) + beta C on complex128 device tensors (op: 0 N, 1 conj,
    2 transpose, 3 conjugate transpose)."""
    M, N = C.shape
    K = A.shape[1] if op_a < 2 else A.shape[0]
    need = tc_gemm_workspace_size(M, N, K, mode)
    if ws is None and need:
        ws = _workspace(need, C.device)
    al, be = complex(alpha), complex(beta)
    _check(lib().tc_zgemm(M, N, K, tc_c128(al.real, al.imag), _ptr(A), A.stride(0), op_a,
                          _ptr(B), B.stride(0), op_b, tc_c128(be.real, be.imag), _ptr(C),
                          C.stride(0), mode, _ptr(ws) if ws is not None else None,
                          ws.numel() if ws is not None else 0, _stream(stream)), "tc_zgemm")


def tc_split_bf16(x, hi, lo, stream=None):
    """hi, lo: torch.int16 (bit patterns) device tensors of x.numel() elements."""
    _check(lib().tc_split_bf16(_ptr(x), x.numel(), _ptr(hi), _ptr(lo), _stream(stream)),
           "tc_split_bf16")


def tc_profile_enable(enable: bool = True):
    _check(lib().tc_profile_enable(1 if enable else 0), "tc_profile_enable")


def tc_profile_read(kernel: int):
    """(total milliseconds, launches) of one kernel class since tc_profile_enable(True)."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().tc_profile_read(kernel, ctypes.byref(ms), ctypes.byref(n)), "tc_profile_read")
    return ms.value, n.value


def tc_mfma_probe(kind: int, random_operands: bool, iters: int, device="cuda", stream=None):
    """(milliseconds, flops) of one MFMA rate probe launch (kind TC_PROBE_*)."""
    import torch
    props = torch.cuda.get_device_properties(torch.device(device))
    out = torch.empty(512 * props.multi_processor_count, dtype=torch.float32, device=device)
    ms, fl = ctypes.c_double(), ctypes.c_double()
    _check(lib().tc_mfma_probe(kind, 1 if random_operands else 0, iters, _ptr(out), out.numel(),
                               ctypes.byref(ms), ctypes.byref(fl), _stream(stream)),
           "tc_mfma_probe")
    return ms.value, fl.value


def tc_autotune_workspace_size(gemm_mode: int, max_N: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().tc_autotune_workspace_size(gemm_mode, max_N, ctypes.byref(b)),
           "tc_autotune_workspace_size")
    return b.value


def tc_autotune(gemm_mode: int, max_N: int, device="cuda", stream=None):
    """Times the grouped tile shapes per dimension bucket and fills the table."""
    ws = _workspace(tc_autotune_workspace_size(gemm_mode, max_N), device)
    _check(lib().tc_autotune(gemm_mode, max_N, _ptr(ws), ws.numel(), _stream(stream)),
           "tc_autotune")


def tc_autotune_query(gemm_mode: int, N: int) -> int:
    v = ctypes.c_int32()
    _check(lib().tc_autotune_query(gemm_mode, N, ctypes.byref(v)), "tc_autotune_query")
    return v.value
