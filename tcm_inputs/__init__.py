"""Seeded synthetic inputs for the Tavis-Cummings density-matrix stepper.

This module is shared by the CPU oracle and the GPU library's tests and
benchmark.  It holds no arithmetic of the method itself: it only draws the
model parameters (couplings g_i, detunings delta_i, sizes) and the initial
pure state psi0 from seeded generators, and lays psi0 out in the basis order
both sides agree on.

Basis order (the paper leaves it open; Sec. II, Eq. (1)-(2) and (4)):
photon-major Kronecker order |m> (x) |l_1> (x) ... (x) |l_n>, atom 1 the most
significant bit, l_i = 1 meaning atom i is excited, so the basis index of
(m, l) is  s = m * 2**n + sum_i l_i * 2**(n - i).  The photon number runs
0..c (cutoff c), so the Hilbert dimension is N = (c + 1) * 2**n.

Random draws (the paper fixes none): numpy's PCG64 seeded with
[240306937, k] for workload k; draw order is sizes (batched workload only),
then all couplings, then all detunings, then the state.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_ROOT = 240306937


def hilbert_dim(n: int, c: int) -> int:
    """N = (c + 1) * 2**n for n two-level atoms and photon cutoff c."""
    if n < 1 or c < 0:
        raise ValueError("need n >= 1 and c >= 0")
    return (c + 1) << n


def basis_index(n: int, m: int, bits) -> int:
    """Index of |m>|l_1..l_n> in photon-major order, atom 1 most significant."""
    s = m << n
    for i, b in enumerate(bits):
        if b:
            s |= 1 << (n - 1 - i)
    return s


@dataclass
class Instance:
    """One Tavis-Cummings model instance plus its initial pure state."""
    n: int
    c: int
    g: np.ndarray                 # [n] couplings g_i (real)
    omega_a: np.ndarray           # [n] atomic frequencies 1 + delta_i
    omega_c: float = 1.0          # cavity frequency
    psi0: Optional[np.ndarray] = None   # [N] complex128, unit norm
    kappa: float = 0.0            # cavity leakage rate (Lindblad term)
    gamma: float = 0.0            # atomic emission rate (Lindblad term)

    @property
    def N(self) -> int:
        return hilbert_dim(self.n, self.c)

    def rho0(self) -> np.ndarray:
        """Initial density matrix |psi0><psi0| (complex128, N x N)."""
        return np.outer(self.psi0, self.psi0.conj())


@dataclass
class Workload:
    name: str
    instances: List[Instance]
    dt: float
    steps: int
    renorm_every: int = 0
    record_every: int = 1
    checkpoint_every: int = 0
    description: str = ""
    extra: dict = field(default_factory=dict)


def _rng(k: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, k])


def basis_state(n: int, c: int, m: int, bits) -> np.ndarray:
    psi = np.zeros(hilbert_dim(n, c), dtype=np.complex128)
    psi[basis_index(n, m, bits)] = 1.0
    return psi


def haar_qubit(rng: np.random.Generator) -> np.ndarray:
    """Haar-random qubit: z ~ N(0,1) + i N(0,1) in C^2, normalised.
    Component 0 is the ground state |0>, component 1 the excited state."""
    z = rng.standard_normal(2) + 1j * rng.standard_normal(2)
    return z / np.linalg.norm(z)


def product_state(n: int, c: int, m: int, qubits) -> np.ndarray:
    """|m> (x) q_1 (x) ... (x) q_n in photon-major order."""
    photon = np.zeros(c + 1, dtype=np.complex128)
    photon[m] = 1.0
    psi = photon
    for q in qubits:
        psi = np.kron(psi, np.asarray(q, dtype=np.complex128))
    return psi


def gaussian_state(N: int, rng: np.random.Generator) -> np.ndarray:
    z = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return z / np.linalg.norm(z)


# ---------------------------------------------------------------------------
# The five workloads.  Sizes follow the paper's own TCM runs (all atoms
# excited, zero photons, Sec. IV.A) extended with an explicit cavity mode.
# ---------------------------------------------------------------------------

def workload_jc3() -> Workload:
    """n=3, c=3 (N=32), equal g=0.01, resonant, |0>|111>, dt=0.01 x 1000."""
    n, c = 3, 3
    inst = Instance(n=n, c=c, g=np.full(n, 0.01), omega_a=np.ones(n),
                    psi0=basis_state(n, c, 0, [1] * n))
    return Workload("tcm_n3_c3_N32_c128", [inst], dt=0.01, steps=1000,
                    record_every=1,
                    description="n=3 atoms, cutoff 3, N=32, complex128, "
                                "per-step excited-atom population")


def workload_n9() -> Workload:
    """n=9, c=9 (N=5120), g~U(0.005,0.02), delta~N(0,0.005), |0>|1^9>."""
    n, c = 9, 9
    rng = _rng(2)
    g = rng.uniform(0.005, 0.02, n)
    delta = rng.normal(0.0, 0.005, n)
    inst = Instance(n=n, c=c, g=g, omega_a=1.0 + delta,
                    psi0=basis_state(n, c, 0, [1] * n))
    return Workload("tcm_n9_c9_N5120_f64", [inst], dt=0.05, steps=100,
                    record_every=1,
                    description="n=9 atoms, cutoff 9, N=5120, FP64")


def workload_n11() -> Workload:
    """n=11, c=5 (N=12288), |2> (x) Haar product over the atoms."""
    n, c = 11, 5
    rng = _rng(3)
    g = rng.uniform(0.005, 0.02, n)
    delta = rng.normal(0.0, 0.005, n)
    qubits = [haar_qubit(rng) for _ in range(n)]
    inst = Instance(n=n, c=c, g=g, omega_a=1.0 + delta,
                    psi0=product_state(n, c, 2, qubits))
    return Workload("tcm_n11_c5_N12288", [inst], dt=0.05, steps=200,
                    renorm_every=20, record_every=1,
                    description="n=11 atoms, cutoff 5, N=12288, "
                                "2 photons x Haar product state")


def workload_batch64(count: int = 64) -> Workload:
    """64 instances, n in {4..10}, c in {1..6}, delta~N(0,0.01), Gaussian
    pure states, dt=0.02 x 500, complex64."""
    rng = _rng(4)
    ns = rng.integers(4, 11, size=count)
    cs = rng.integers(1, 7, size=count)
    gs = [rng.uniform(0.005, 0.02, int(n)) for n in ns]
    ds = [rng.normal(0.0, 0.01, int(n)) for n in ns]
    insts = []
    for b in range(count):
        n, c = int(ns[b]), int(cs[b])
        insts.append(Instance(n=n, c=c, g=gs[b], omega_a=1.0 + ds[b]))
    for inst in insts:
        inst.psi0 = gaussian_state(inst.N, rng)
    return Workload("tcm_batch64_c64", insts, dt=0.02, steps=500,
                    record_every=1,
                    description="64 uneven instances, N=(c+1)2^n in [32,7168]")


def workload_grad8() -> Workload:
    """n=8, c=8 (N=2304), trainable g_i and delta_i, |0>|1^8>, 500 steps."""
    n, c = 8, 8
    rng = _rng(5)
    g = rng.uniform(0.005, 0.02, n)
    delta = rng.normal(0.0, 0.01, n)
    inst = Instance(n=n, c=c, g=g, omega_a=1.0 + delta,
                    psi0=basis_state(n, c, 0, [1] * n))
    return Workload("tcm_n8_c8_N2304_grad", [inst], dt=0.05, steps=500,
                    checkpoint_every=50, record_every=1,
                    description="n=8 atoms, cutoff 8, N=2304, adjoint gradient")


def workload_paper(n: int) -> Workload:
    """The paper's own runs (Sec. IV): n atoms, all excited, no photons, on the
    2^n states of its atom-only model, which is the excitation-n sector of
    the cavity model with cutoff c = n.  The paper states neither couplings,
    detunings nor dt; the seeded draws follow the N = 5120 workload
    (g_i ~ U(0.005, 0.02), delta_i ~ N(0, 0.005), dt = 0.05)."""
    rng = _rng(600 + n)
    g = rng.uniform(0.005, 0.02, n)
    delta = rng.normal(0.0, 0.005, n)
    inst = Instance(n=n, c=n, g=g, omega_a=1.0 + delta,
                    psi0=basis_state(n, n, 0, [1] * n))
    return Workload(f"tcm_paper_n{n}_N{1 << n}", [inst], dt=0.05, steps=0,
                    description=f"paper's 2^n model, n={n} atoms all excited",
                    extra={"sector": n})


WORKLOADS = {
    "jc3": workload_jc3,
    "n9": workload_n9,
    "n11": workload_n11,
    "batch64": workload_batch64,
    "grad8": workload_grad8,
}


def get(name: str) -> Workload:
    return WORKLOADS[name]()


def random_model(n: int, c: int, seed: int, g_lo=0.005, g_hi=0.02,
                 delta_sigma=0.005, state="gaussian") -> Instance:
    """Small random instance for parity tests (seeded; same draw order)."""
    rng = np.random.default_rng([SEED_ROOT, 1000 + seed])
    g = rng.uniform(g_lo, g_hi, n)
    delta = rng.normal(0.0, delta_sigma, n)
    inst = Instance(n=n, c=c, g=g, omega_a=1.0 + delta)
    N = inst.N
    if state == "gaussian":
        inst.psi0 = gaussian_state(N, rng)
    elif state == "excited":
        inst.psi0 = basis_state(n, c, 0, [1] * n)
    elif state == "haar2":
        m = min(2, c)
        inst.psi0 = product_state(n, c, m, [haar_qubit(rng) for _ in range(n)])
    else:
        raise ValueError(state)
    return inst


def random_matrix(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Seeded Gaussian matrix (complex or real) for kernel-level tests."""
    rng = np.random.default_rng([SEED_ROOT, 5000 + seed])
    if np.issubdtype(dtype, np.complexfloating):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)
    return rng.standard_normal(shape).astype(dtype)


def dense_control(N: int, dt: float, norm: float = 0.8, seed: int = 0):
    """Dense stand-in with no zero structure, for timing only: a real symmetric
    Gaussian matrix H (off-diagonal variance sigma^2, diagonal 2 sigma^2) scaled
    so that its spectral radius, about 2 sigma sqrt(N), times dt is `norm`, and
    a normalised complex Gaussian state psi of length N.  Returns (H, psi)."""
    rng = np.random.default_rng([SEED_ROOT, 9000 + seed])
    sigma = norm / (2.0 * np.sqrt(N) * dt)
    H = rng.standard_normal((N, N))
    H += H.T
    H *= sigma / np.sqrt(2.0)
    psi = gaussian_state(N, rng)
    return H, psi


def random_density(N: int, seed: int, rank: int = 1) -> np.ndarray:
    """Seeded random density matrix (Hermitian, PSD, unit trace)."""
    rng = np.random.default_rng([SEED_ROOT, 7000 + seed])
    Z = rng.standard_normal((N, rank)) + 1j * rng.standard_normal((N, rank))
    rho = Z @ Z.conj().T
    return rho / np.trace(rho).real
