"""Independent checks used to pin the oracle: the dense op(A) written out with
numpy, exact rational arithmetic with Python fractions, and Gaussian
elimination on the full dense matrix.  None of this touches the oracle's
triangle-walking code."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

VARIANTS = [(s, u, t) for s in "LR" for u in "LU" for t in "NTC"]
VARIANTS_NT = [(s, u, t) for s in "LR" for u in "LU" for t in "NT"]


def dense_op(A: np.ndarray, uplo: str, trans: str, diag: str) -> np.ndarray:
    """Explicit op(A): the named triangle of A (zeros elsewhere), unit diagonal
    substituted when diag='U', transposed when trans is 'T' or 'C'."""
    A = np.nan_to_num(np.asarray(A, dtype=np.float64), nan=0.0)
    T = np.tril(A) if uplo.upper() == "L" else np.triu(A)
    if diag.upper() == "U":
        T = T.copy()
        np.fill_diagonal(T, 1.0)
    return T.T.copy() if trans.upper() in "TC" else T


def to_frac(M: np.ndarray):
    return [[Fraction(float(v)) for v in row] for row in np.asarray(M)]


def frac_matmul(P, Q):
    n, k, p = len(P), len(Q), len(Q[0])
    return [[sum((P[i][t] * Q[t][j] for t in range(k)), Fraction(0)) for j in range(p)] for i in range(n)]


def frac_solve(M, Bm):
    """Solve M X = Bm exactly by Gaussian elimination with row pivoting on the
    first non-zero entry (M dense, any non-singular square matrix)."""
    n = len(M)
    p = len(Bm[0])
    aug = [list(M[i]) + list(Bm[i]) for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if aug[r][c] != 0)
        aug[c], aug[piv] = aug[piv], aug[c]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                f = aug[r][c] / aug[c][c]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[c])]
    return [[aug[i][n + j] / aug[i][i] for j in range(p)] for i in range(n)]


def transpose(M):
    return [list(r) for r in zip(*M)]


def exact_trmm(side, uplo, trans, diag, alpha, A, B):
    T = to_frac(dense_op(A, uplo, trans, diag))
    Bf = to_frac(B)
    a = Fraction(float(alpha))
    P = frac_matmul(T, Bf) if side.upper() == "L" else frac_matmul(Bf, T)
    return [[a * v for v in row] for row in P]


def exact_trsm(side, uplo, trans, diag, alpha, A, B):
    T = to_frac(dense_op(A, uplo, trans, diag))
    a = Fraction(float(alpha))
    Bf = [[a * v for v in row] for row in to_frac(B)]
    if side.upper() == "L":
        return frac_solve(T, Bf)
    # X T = B  <=>  T^T X^T = B^T
    return transpose(frac_solve(transpose(T), transpose(Bf)))


def frac_to_f64_exact(M) -> np.ndarray:
    """Convert a rational matrix to float64, asserting that every entry is exact."""
    out = np.empty((len(M), len(M[0])), order="F")
    for i, row in enumerate(M):
        for j, v in enumerate(row):
            f = float(v)
            assert Fraction(f) == v, f"entry ({i},{j}) = {v} is not exactly representable"
            out[i, j] = f
    return out
