"""Pin of the oracle's matrix-product definition (oracle.linalg.gemm), which
checks every kernel-level product test, against the entry-by-entry sum

    C[i][j] = alpha * sum_k op_a(A)[i][k] * op_b(B)[k][j] + beta * C0[i][j] + gamma * [i == j]

written out in pure-Python loops, with op(X)[i][k] read from X directly:
'n' X[i][k], 'c' conj(X[i][k]), 't' X[k][i], 'h' conj(X[k][i]).  The shapes
are rectangular and pairwise distinct, and the values complex with nonzero
real and imaginary parts, so a transposed operand fails on its shape and a
missing or extra conjugation, a swapped 't' / 'h' branch, a dropped alpha,
beta or gamma term, or a sign error each change the result."""
import itertools

import numpy as np
import pytest

from oracle import linalg as olin


def _entry(X, op, i, k):
    if op == "n":
        return X[i][k]
    if op == "c":
        return X[i][k].conjugate()
    if op == "t":
        return X[k][i]
    if op == "h":
        return X[k][i].conjugate()
    raise ValueError(op)


def _loops(A, B, op_a, op_b, alpha, beta, C0, gamma, M, N, K):
    A, B, C0 = A.tolist(), B.tolist(), C0.tolist()
    out = [[0j] * N for _ in range(M)]
    for i in range(M):
        for j in range(N):
            s = 0j
            for k in range(K):
                s += _entry(A, op_a, i, k) * _entry(B, op_b, k, j)
            out[i][j] = alpha * s + beta * C0[i][j] + (gamma if i == j else 0)
    return np.array(out, dtype=np.complex128)


def _cplx(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("op_a,op_b", list(itertools.product("ncth", repeat=2)))
def test_gemm_matches_entrywise_definition(op_a, op_b):
    rng = np.random.default_rng(7 + 4 * "ncth".index(op_a) + "ncth".index(op_b))
    M, N, K = 3, 4, 5
    A = _cplx(rng, (K, M) if op_a in "th" else (M, K))
    B = _cplx(rng, (N, K) if op_b in "th" else (K, N))
    C0 = _cplx(rng, (M, N))
    alpha, beta, gamma = 0.7 - 1.3j, -0.4 + 0.9j, 1.1 + 0.25j
    got = olin.gemm(A, B, op_a, op_b, alpha, beta, C0, gamma)
    ref = _loops(A, B, op_a, op_b, alpha, beta, C0, gamma, M, N, K)
    assert got.shape == (M, N)
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_gemm_defaults_and_real_inputs():
    """Defaults are alpha = 1, beta = 0, gamma = 0 (C0 ignored); real inputs
    stay real."""
    rng = np.random.default_rng(3)
    A, B = rng.standard_normal((3, 5)), rng.standard_normal((5, 2))
    got = olin.gemm(A, B)
    ref = _loops(A.astype(complex), B.astype(complex), "n", "n", 1.0, 0.0,
                 np.zeros((3, 2), complex), 0.0, 3, 2, 5)
    assert got.dtype == np.float64
    assert np.max(np.abs(got - ref.real)) <= 1e-13 and np.all(ref.imag == 0)
    C0 = _cplx(rng, (3, 2))
    assert np.array_equal(olin.gemm(A, B, C0=C0), got)


def test_gemm_rejects_unknown_op():
    with pytest.raises(ValueError):
        olin.gemm(np.eye(2), np.eye(2), op_a="x")
