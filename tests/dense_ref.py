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


class GRat:
    """Exact Gaussian rational re + im*i with Fraction parts, enough arithmetic
    for frac_matmul / frac_solve on complex inputs."""
    __slots__ = ("re", "im")

    def __init__(self, re, im=0):
        self.re = Fraction(re)
        self.im = Fraction(im)

    @staticmethod
    def of(x):
        if isinstance(x, GRat):
            return x
        if isinstance(x, complex):
            return GRat(Fraction(x.real), Fraction(x.imag))
        return GRat(x)

    def __add__(self, o):
        o = GRat.of(o)
        return GRat(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = GRat.of(o)
        return GRat(self.re - o.re, self.im - o.im)

    def __rsub__(self, o):
        return GRat.of(o) - self

    def __mul__(self, o):
        o = GRat.of(o)
        return GRat(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = GRat.of(o)
        d = o.re * o.re + o.im * o.im
        return GRat((self.re * o.re + self.im * o.im) / d, (self.im * o.re - self.re * o.im) / d)

    def __neg__(self):
        return GRat(-self.re, -self.im)

    def __eq__(self, o):
        o = GRat.of(o)
        return self.re == o.re and self.im == o.im

    def __ne__(self, o):
        return not self == o

    __hash__ = None


def zdense_op(A: np.ndarray, uplo: str, trans: str, diag: str) -> np.ndarray:
    """Explicit complex op(A): the named triangle (zeros elsewhere), unit
    diagonal when diag='U', transposed for 'T', conjugate-transposed for 'C'."""
    A = np.nan_to_num(np.asarray(A, dtype=np.complex128), nan=0.0)
    T = np.tril(A) if uplo.upper() == "L" else np.triu(A)
    if diag.upper() == "U":
        T = T.copy()
        np.fill_diagonal(T, 1.0)
    if trans.upper() == "T":
        return T.T.copy()
    if trans.upper() == "C":
        return T.conj().T.copy()
    return T


def to_grat(M: np.ndarray):
    return [[GRat(Fraction(float(v.real)), Fraction(float(v.imag))) for v in row] for row in np.asarray(M)]


def grat_to_c128_exact(M) -> np.ndarray:
    out = np.empty((len(M), len(M[0])), dtype=np.complex128, order="F")
    for i, row in enumerate(M):
        for j, v in enumerate(row):
            re, im = float(v.re), float(v.im)
            assert Fraction(re) == v.re and Fraction(im) == v.im, f"entry ({i},{j}) is not exactly representable"
            out[i, j] = complex(re, im)
    return out


def exact_ztrsm(side, uplo, trans, diag, alpha, A, B):
    T = to_grat(zdense_op(A, uplo, trans, diag))
    a = GRat.of(complex(alpha))
    Bf = [[a * v for v in row] for row in to_grat(B)]
    if side.upper() == "L":
        return frac_solve(T, Bf)
    return transpose(frac_solve(transpose(T), transpose(Bf)))


def exact_ztrmm(side, uplo, trans, diag, alpha, A, B):
    T = to_grat(zdense_op(A, uplo, trans, diag))
    Bf = to_grat(B)
    a = GRat.of(complex(alpha))
    P = frac_matmul(T, Bf) if side.upper() == "L" else frac_matmul(Bf, T)
    return [[a * v for v in row] for row in P]
