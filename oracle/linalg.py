"""Plain matrix-product definitions for kernel-level checks (FP64).

C = alpha * op_a(A) @ op_b(B) + beta * C0 + gamma * I, where op is identity,
complex conjugate or conjugate transpose.  numpy's matmul is the product.
"""
from __future__ import annotations

import numpy as np


def _op(X, op):
    if op == "n":
        return X
    if op == "c":
        return X.conj()
    if op == "t":
        return X.T
    if op == "h":
        return X.conj().T
    raise ValueError(op)


def gemm(A, B, op_a="n", op_b="n", alpha=1.0, beta=0.0, C0=None, gamma=0.0):
    A = np.asarray(A, dtype=np.complex128 if np.iscomplexobj(A) else np.float64)
    B = np.asarray(B, dtype=np.complex128 if np.iscomplexobj(B) else np.float64)
    C = alpha * (_op(A, op_a) @ _op(B, op_b))
    if C0 is not None and beta != 0:
        C = C + beta * C0
    if gamma != 0:
        C = C + gamma * np.eye(C.shape[0], C.shape[1])
    return C
