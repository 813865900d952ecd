"""GPU parity of the kernel-level entry points against the oracle:
Hamiltonian, matrix products in the three precisions, the bfloat16 split,
the matrix exponential, observables."""
import math

import numpy as np
import pytest
import torch

import tcm_inputs as ti
from oracle import bf16 as obf16
from oracle import evolve as oev
from oracle import linalg as olin
from oracle import model as omodel
from oracle import observables as oobs

pytestmark = pytest.mark.gpu

tcm = pytest.importorskip("paper_2403_06937_amd")
from paper_2403_06937_amd import pipeline  # noqa: E402

DEV = "cuda"


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tcm.lib()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("n,c,seed", [(1, 0, 0), (1, 5, 1), (3, 3, 2), (5, 4, 3), (7, 2, 4), (9, 1, 5)])
def test_hamiltonian_matches_oracle(n, c, seed):
    inst = ti.random_model(n, c, seed)
    m = pipeline.model_of(inst)
    H = pipeline.hamiltonian(m).cpu().numpy()
    Ho = omodel.hamiltonian(n, c, inst.g, inst.omega_a)
    # identical summation order on the diagonal: equal to the last bit
    assert np.array_equal(H != 0, Ho != 0)
    assert np.max(np.abs(H - Ho)) <= 2 * np.finfo(float).eps * np.max(np.abs(Ho))


def test_hamiltonian_leading_dimension_untouched():
    inst = ti.random_model(3, 2, 9)
    m = pipeline.model_of(inst)
    N = m.N
    buf = torch.full((N, N + 5), 7.0, dtype=torch.float64, device=DEV)
    tcm.tc_build_hamiltonian(m, buf)
    b = buf.cpu().numpy()
    assert np.all(b[:, N:] == 7.0)
    assert np.max(np.abs(b[:, :N] - omodel.hamiltonian(3, 2, inst.g, inst.omega_a))) < 1e-15


SIZES = [(1, 1, 1), (31, 33, 17), (33, 31, 64), (128, 64, 8), (127, 129, 257), (256, 128, 64),
         (300, 200, 1000)]
OPS = [(0, 0), (2, 0), (0, 1), (3, 2), (1, 3)]


def _op(X, o):
    return {0: "n", 1: "c", 2: "t", 3: "h"}[o]


@pytest.mark.parametrize("M,N,K", SIZES)
@pytest.mark.parametrize("op_a,op_b", OPS)
def test_zgemm_f64(M, N, K, op_a, op_b):
    A = ti.random_matrix((K, M) if op_a >= 2 else (M, K), 1)
    B = ti.random_matrix((N, K) if op_b >= 2 else (K, N), 2)
    C0 = ti.random_matrix((M, N), 3)
    alpha, beta = 0.7 - 0.2j, 0.3 + 0.1j
    ref = olin.gemm(A, B, _op(A, op_a), _op(B, op_b), alpha, beta, C0)
    C = _dev(C0)
    tcm.tc_zgemm(_dev(A), _dev(B), C, op_a, op_b, alpha, beta, tcm.TC_GEMM_F64)
    err = np.max(np.abs(C.cpu().numpy() - ref))
    assert err <= 1e-13 * max(1.0, math.sqrt(K)) * np.max(np.abs(ref)) + 1e-15


@pytest.mark.parametrize("M,N,K", SIZES)
def test_zgemm_f32(M, N, K):
    A = ti.random_matrix((M, K), 4)
    B = ti.random_matrix((K, N), 5)
    ref = olin.gemm(A.astype(np.complex64), B.astype(np.complex64))
    C = torch.zeros((M, N), dtype=torch.complex128, device=DEV)
    tcm.tc_zgemm(_dev(A), _dev(B), C, 0, 0, 1.0, 0.0, tcm.TC_GEMM_F32)
    err = np.max(np.abs(C.cpu().numpy() - ref))
    assert err <= 2e-6 * math.sqrt(K) * max(1.0, np.max(np.abs(ref)) / math.sqrt(K))


def split_product_reference(A, B):
    """Exact value of the split-BF16 product of complex64-rounded operands:
    each real operand x -> hi + lo from the oracle's RNE split, products
    hi*hi + hi*lo + lo*hi, summed in FP64."""
    def parts(X):
        out = []
        for comp in (X.real, X.imag):
            h, l = obf16.split(comp.astype(np.float32))
            out.append((obf16.bits_to_float(h).astype(np.float64),
                        obf16.bits_to_float(l).astype(np.float64)))
        return out
    (arh, arl), (aih, ail) = parts(A)
    (brh, brl), (bih, bil) = parts(B)

    def p3(xh, xl, yh, yl):
        return xh @ yh + xh @ yl + xl @ yh
    re = p3(arh, arl, brh, brl) - p3(aih, ail, bih, bil)
    im = p3(arh, arl, bih, bil) + p3(aih, ail, brh, brl)
    return re + 1j * im


@pytest.mark.parametrize("M,N,K", SIZES)
@pytest.mark.parametrize("op_a,op_b", [(0, 0), (2, 1)])
def test_zgemm_split_bf16(M, N, K, op_a, op_b):
    A = ti.random_matrix((K, M) if op_a >= 2 else (M, K), 6)
    B = ti.random_matrix((N, K) if op_b >= 2 else (K, N), 7)
    Aop = olin._op(A, _op(A, op_a)).astype(np.complex64)
    Bop = olin._op(B, _op(B, op_b)).astype(np.complex64)
    emu = split_product_reference(Aop, Bop)
    exact = Aop.astype(np.complex128) @ Bop.astype(np.complex128)
    C = torch.zeros((M, N), dtype=torch.complex128, device=DEV)
    tcm.tc_zgemm(_dev(A), _dev(B), C, op_a, op_b, 1.0, 0.0, tcm.TC_GEMM_SPLIT_BF16)
    got = C.cpu().numpy()
    scale = np.max(np.abs(exact))
    # equals the emulated split product up to FP32 accumulation ...
    assert np.max(np.abs(got - emu)) <= 4e-7 * math.sqrt(K) * max(scale, 1.0)
    # ... and the exact product to the split's own 2^-16-level error
    assert np.max(np.abs(got - exact)) <= 3e-5 * math.sqrt(K) * max(scale / math.sqrt(K), 1.0)


@pytest.mark.parametrize("M,N,K", [(2048, 2048, 256), (2048, 4096, 96)])
def test_zgemm_split_bf16_band_order(M, N, K):
    """Tile grids that are multiples of 16 x 16 tiles take the band order (all
    XCDs in one 16-row band, each walking its quarter of the columns): every
    tile is computed exactly once and equals the emulated split product."""
    A = ti.random_matrix((M, K), 8)
    B = ti.random_matrix((K, N), 9)
    Aop, Bop = A.astype(np.complex64), B.astype(np.complex64)
    emu = split_product_reference(Aop, Bop)
    C = torch.full((M, N), complex(np.nan, np.nan), dtype=torch.complex128, device=DEV)
    tcm.tc_zgemm(_dev(A), _dev(B), C, 0, 0, 1.0, 0.0, tcm.TC_GEMM_SPLIT_BF16)
    got = C.cpu().numpy()
    assert np.all(np.isfinite(got))
    scale = np.max(np.abs(emu))
    assert np.max(np.abs(got - emu)) <= 4e-7 * math.sqrt(K) * max(scale, 1.0)


def test_split_bf16_bit_exact():
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(1 << 16) * np.exp(rng.uniform(-30, 30, 1 << 16))).astype(np.float32)
    x[:8] = np.array([0.0, -0.0, 1.0, 3.0, 1e-30, -7.5e20, 0x3F808000, 1.00390625], np.float32)
    xt = torch.from_numpy(x).to(DEV)
    hi = torch.empty(x.size, dtype=torch.int16, device=DEV)
    lo = torch.empty(x.size, dtype=torch.int16, device=DEV)
    tcm.tc_split_bf16(xt, hi, lo)
    h, l = obf16.split(x)
    assert np.array_equal(hi.cpu().numpy().view(np.uint16), h)
    assert np.array_equal(lo.cpu().numpy().view(np.uint16), l)


EXPM_CASES = [(3, 3, 0.01, 0), (5, 4, 0.05, 1), (2, 6, 0.9, 2), (7, 1, 0.05, 3), (4, 2, 3.0, 4)]


@pytest.mark.parametrize("n,c,dt,seed", EXPM_CASES)
def test_expm_matches_eigendecomposition(n, c, dt, seed):
    inst = ti.random_model(n, c, seed)
    m = pipeline.model_of(inst)
    _, U = pipeline.propagator(m, dt)
    Ug = U.cpu().numpy()
    Ho = omodel.hamiltonian(n, c, inst.g, inst.omega_a)
    Uo = oev.propagator(Ho, dt)
    assert np.max(np.abs(Ug - Uo)) <= 1e-13 * max(1.0, abs(dt) * np.max(np.abs(np.linalg.eigvalsh(Ho))))
    assert np.array_equal(Ug, Ug.T)                                   # symmetrised
    assert np.max(np.abs(Ug.conj().T @ Ug - np.eye(m.N))) < 1e-13    # unitary
    k = omodel.total_excitation_diag(n, c)
    assert np.all(Ug[k[:, None] != k[None, :]] == 0)                 # exact zeros across sectors


@pytest.mark.parametrize("n,c,dt", [(3, 3, 0.01), (5, 4, 0.05), (6, 3, 0.05)])
def test_expm_taylor10_matches_oracle(n, c, dt):
    inst = ti.random_model(n, c, 11)
    m = pipeline.model_of(inst)
    _, L = pipeline.propagator(m, dt, method=tcm.TC_EXPM_TAYLOR10)
    Ho = omodel.hamiltonian(n, c, inst.g, inst.omega_a)
    Lo, _ = oev.taylor_factors(Ho, dt)
    assert np.max(np.abs(L.cpu().numpy() - Lo)) < 1e-12


def test_observables_match_oracle():
    n, c = 4, 3
    inst = ti.random_model(n, c, 13)
    m = pipeline.model_of(inst)
    rho = ti.random_density(m.N, 1, rank=3)
    rho[3, 5] += 1e-3            # a non-Hermitian perturbation to measure
    got = pipeline.observables(m, _dev(rho))
    inv = oobs.invariants(rho)
    assert abs(got["trace_re"] - inv["trace_re"]) < 1e-14
    assert abs(got["trace_im"] - inv["trace_im"]) < 1e-14
    assert abs(got["purity"] - inv["purity"]) < 1e-14
    assert abs(got["herm_err"] - inv["herm_err"]) < 1e-15
    assert abs(got["excitation_total"] - oobs.excitation_total(rho, n, c)) < 1e-14
    assert abs(got["photon_mean"] - oobs.photon_mean(rho, n, c)) < 1e-14
    assert abs(got["excitation_mean"] - oobs.excitation_mean(rho, n, c)) < 1e-14
    assert np.max(np.abs(got["atom_pop"] - oobs.atom_populations(rho, n, c))) < 1e-14
    assert np.max(np.abs(got["photon_dist"] - oobs.photon_distribution(rho, n, c))) < 1e-14
    assert np.max(np.abs(got["exc_dist"] - oobs.excitation_distribution(rho, n, c))) < 1e-14
    # both readings of Eq. (13); rho has coherences inside each {m> set, so the
    # symmetric reading differs from the sector reading
    ps, dk = oobs.photon_state_probability(rho, n, c), oobs.dicke_probability(rho, n, c)
    assert np.max(np.abs(ps - dk)) > 1e-3
    assert np.max(np.abs(got["photon_state"] - ps)) < 1e-14
    assert np.max(np.abs(got["dicke"] - dk)) < 1e-14
    assert got["nonfinite"] == 0.0
    rho[2, 2] = np.nan
    assert pipeline.observables(m, _dev(rho))["nonfinite"] == 1.0


def test_observables_complex64_and_ragged():
    n, c = 3, 2     # N = 24, not a multiple of the 32-wide tiles
    inst = ti.random_model(n, c, 14)
    m = pipeline.model_of(inst)
    rho = ti.random_density(m.N, 2).astype(np.complex64)
    got = pipeline.observables(m, _dev(rho))
    r64 = rho.astype(np.complex128)
    assert abs(got["purity"] - oobs.invariants(r64)["purity"]) < 1e-6
    assert np.max(np.abs(got["photon_dist"] - oobs.photon_distribution(r64, n, c))) < 1e-7
    assert np.max(np.abs(got["photon_state"] - oobs.photon_state_probability(r64, n, c))) < 1e-7
    assert np.max(np.abs(got["dicke"] - oobs.dicke_probability(r64, n, c))) < 1e-7


@pytest.mark.parametrize("n,c", [(1, 3), (5, 2), (6, 6), (11, 5)])
def test_eq13_readings_shapes(n, c):
    """Both Eq. (13) readings for c < n, c = n, c > n and the N = 12288 shape
    (one row of the Dicke pass per atom pattern, 462 states in its largest
    set) on a random mixed state."""
    inst = ti.random_model(n, c, 15 + n)
    m = pipeline.model_of(inst)
    rho = ti.random_density(m.N, 5, rank=2)
    got = pipeline.observables(m, _dev(rho))
    assert got["photon_state"].shape == (min(n, c) + 1,)
    assert np.max(np.abs(got["photon_state"] - oobs.photon_state_probability(rho, n, c))) < 1e-14
    assert np.max(np.abs(got["dicke"] - oobs.dicke_probability(rho, n, c))) < 1e-14


@pytest.mark.parametrize("kind,peak", [(tcm.TC_PROBE_BF16_16X16X32, 2.5e15),
                                       (tcm.TC_PROBE_BF16_32X32X16, 2.5e15),
                                       (tcm.TC_PROBE_F64_16X16X4, 78.6e12)])
def test_mfma_probe_rates(kind, peak):
    """The MFMA rate probe issues what it reports (2 flops per multiply-add,
    16 / 8 / 8 MFMAs per wave and round on 8 waves of every compute unit)
    and runs within the datasheet peak: zero operands near it, random ones
    not faster than zeros by more than timing noise."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    per = {tcm.TC_PROBE_BF16_16X16X32: 16 * 16 * 16 * 32 * 2,
           tcm.TC_PROBE_BF16_32X32X16: 8 * 32 * 32 * 16 * 2,
           tcm.TC_PROBE_F64_16X16X4: 8 * 16 * 16 * 4 * 2}[kind]
    iters = 20000 if kind != tcm.TC_PROBE_F64_16X16X4 else 4000
    tcm.tc_mfma_probe(kind, True, 1000)
    ms_z, fl_z = tcm.tc_mfma_probe(kind, False, iters)
    ms_r, fl_r = tcm.tc_mfma_probe(kind, True, iters)
    assert fl_z == fl_r == float(per) * iters * cus * 8
    fz, fr = fl_z / (ms_z * 1e-3) / peak, fl_r / (ms_r * 1e-3) / peak
    print(f"probe kind {kind}: zero operands {fz:.3f} of peak, random {fr:.3f}", flush=True)
    assert 0.5 < fz < 1.05 and 0.3 < fr < 1.05
    assert fr < fz * 1.05
