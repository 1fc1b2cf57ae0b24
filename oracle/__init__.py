"""Python front end of the plain FP64 CPU reference (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library's product path.  It shares
no code with the GPU library.

All matrices are numpy float64 arrays in column-major (Fortran) order.  The
functions copy nothing they do not need to and never modify their inputs,
except ``trmm``/``trsm`` which return a new array holding the result.

Codes: side 'L'/'R', uplo 'L'/'U', trans 'N'/'T'/'C', diag 'N'/'U' (the
equations of the paper's Sec. 2.1, eqs. (1)-(4)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_i64 = ctypes.c_int64
_c_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        sig_op = [ctypes.c_int] * 4 + [_c_i64, _c_i64, ctypes.c_double, _c_dp, _c_i64, _c_dp, _c_i64]
        for name in ("oracle_trmm", "oracle_trsm"):
            f = getattr(L, name)
            f.argtypes = sig_op
            f.restype = None
        L.oracle_trmm_dot2.argtypes = sig_op + [_c_dp, _c_i64]
        L.oracle_trmm_dot2.restype = None
        L.oracle_trsm_residual.argtypes = sig_op + [_c_dp, _c_i64, _c_dp, _c_i64]
        L.oracle_trsm_residual.restype = None
        L.oracle_trsm_eta.argtypes = sig_op + [_c_dp, _c_i64]
        L.oracle_trsm_eta.restype = ctypes.c_double
        L.oracle_trmm_eta.argtypes = sig_op + [_c_dp, _c_i64]
        L.oracle_trmm_eta.restype = ctypes.c_double
        for name in ("oracle_opnorm_inf", "oracle_opnorm_one"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_int] * 3 + [_c_i64, _c_dp, _c_i64]
            f.restype = ctypes.c_double
        zsig = [ctypes.c_int] * 4 + [_c_i64, _c_i64, ctypes.c_double, ctypes.c_double, _c_dp, _c_i64, _c_dp, _c_i64]
        for name in ("oracle_ztrmm", "oracle_ztrsm"):
            f = getattr(L, name)
            f.argtypes = zsig
            f.restype = None
        L.oracle_ztrsm_residual.argtypes = zsig + [_c_dp, _c_i64, _c_dp]
        L.oracle_ztrsm_residual.restype = None
        L.oracle_ztrmm_dot2.argtypes = zsig + [_c_dp]
        L.oracle_ztrmm_dot2.restype = None
        for name in ("oracle_ztrsm_eta", "oracle_ztrmm_eta"):
            f = getattr(L, name)
            f.argtypes = zsig + [_c_dp, _c_i64]
            f.restype = ctypes.c_double
        L.oracle_zopnorm.argtypes = [ctypes.c_int] * 3 + [_c_i64, _c_dp, _c_i64, ctypes.c_int]
        L.oracle_zopnorm.restype = ctypes.c_double
        L.oracle_trtri.argtypes = [ctypes.c_int, ctypes.c_int, _c_i64, _c_dp, _c_i64]
        L.oracle_trtri.restype = None
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


_SIDE = {"L": 0, "R": 1}
_UPLO = {"L": 0, "U": 1}
_TRANS = {"N": 0, "T": 1, "C": 2}
_DIAG = {"N": 0, "U": 1}


def _codes(side, uplo, trans, diag):
    return _SIDE[side.upper()], _UPLO[uplo.upper()], _TRANS[trans.upper()], _DIAG[diag.upper()]


def _f64(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    if a.ndim != 2:
        raise ValueError("expected a 2-D matrix")
    return np.asfortranarray(a)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_c_dp)


def _ld(a: np.ndarray) -> int:
    return max(1, a.shape[0])


def _check(side, A, B):
    m, n = B.shape
    ka = m if side.upper() == "L" else n
    if A.shape[0] < ka or A.shape[1] < ka:
        raise ValueError(f"A is {A.shape}, needs at least {ka}x{ka}")
    return m, n


def trmm(side, uplo, trans, diag, alpha, A, B) -> np.ndarray:
    """Return alpha*op(A)*B (side L) or alpha*B*op(A) (side R); eqs. (1), (2)."""
    A = _f64(A)
    X = _f64(B).copy(order="F")
    m, n = _check(side, A, X)
    lib().oracle_trmm(*_codes(side, uplo, trans, diag), m, n, float(alpha), _p(A), _ld(A), _p(X), _ld(X))
    return X


def trsm(side, uplo, trans, diag, alpha, A, B) -> np.ndarray:
    """Return X with op(A)*X = alpha*B (side L) or X*op(A) = alpha*B (side R); eqs. (3), (4)."""
    A = _f64(A)
    X = _f64(B).copy(order="F")
    m, n = _check(side, A, X)
    lib().oracle_trsm(*_codes(side, uplo, trans, diag), m, n, float(alpha), _p(A), _ld(A), _p(X), _ld(X))
    return X


def trmm_dot2(side, uplo, trans, diag, alpha, A, B) -> np.ndarray:
    """Compensated (Dot2) product, the accurate reference for TRMM errors."""
    A = _f64(A)
    B = _f64(B)
    m, n = _check(side, A, B)
    C = np.zeros((m, n), order="F")
    lib().oracle_trmm_dot2(*_codes(side, uplo, trans, diag), m, n, float(alpha), _p(A), _ld(A), _p(B), _ld(B),
                           _p(C), _ld(C))
    return C


def trsm_residual(side, uplo, trans, diag, alpha, A, B, X) -> np.ndarray:
    """Compensated residual alpha*B - op(A)*X (side L) or alpha*B - X*op(A) (side R)."""
    A = _f64(A)
    B = _f64(B)
    X = _f64(X)
    m, n = _check(side, A, B)
    R = np.zeros((m, n), order="F")
    lib().oracle_trsm_residual(*_codes(side, uplo, trans, diag), m, n, float(alpha), _p(A), _ld(A), _p(B),
                               _ld(B), _p(X), _ld(X), _p(R), _ld(R))
    return R


def trsm_eta(side, uplo, trans, diag, alpha, A, B, X) -> float:
    """Normwise backward error of a computed TRSM solution X (max over columns / rows)."""
    A = _f64(A)
    B = _f64(B)
    X = _f64(X)
    m, n = _check(side, A, B)
    if X.shape != (m, n):
        raise ValueError("X shape")
    return float(lib().oracle_trsm_eta(*_codes(side, uplo, trans, diag), m, n, float(alpha), _p(A), _ld(A),
                                       _p(B), _ld(B), _p(X), _ld(X)))


def trmm_eta(side, uplo, trans, diag, alpha, A, B, C) -> float:
    """Normwise error of a computed TRMM product C against the compensated reference."""
    A = _f64(A)
    B = _f64(B)
    C = _f64(C)
    m, n = _check(side, A, B)
    if C.shape != (m, n):
        raise ValueError("C shape")
    return float(lib().oracle_trmm_eta(*_codes(side, uplo, trans, diag), m, n, float(alpha), _p(A), _ld(A),
                                       _p(B), _ld(B), _p(C), _ld(C)))


def opnorm_inf(uplo, trans, diag, A) -> float:
    A = _f64(A)
    return float(lib().oracle_opnorm_inf(_UPLO[uplo.upper()], _TRANS[trans.upper()], _DIAG[diag.upper()],
                                         A.shape[0], _p(A), _ld(A)))


def opnorm_one(uplo, trans, diag, A) -> float:
    A = _f64(A)
    return float(lib().oracle_opnorm_one(_UPLO[uplo.upper()], _TRANS[trans.upper()], _DIAG[diag.upper()],
                                         A.shape[0], _p(A), _ld(A)))


def cond_one(uplo, diag, A) -> float:
    """1-norm condition number |A|_1 |A^-1|_1 of the triangular factor, with the
    inverse taken column by column from the substitution above (trsm on I)."""
    m = A.shape[0]
    inv = trsm("L", uplo, "N", diag, 1.0, A, np.eye(m, order="F"))
    return opnorm_one(uplo, "N", diag, A) * float(np.abs(inv).sum(axis=0).max())


# ---- complex (interleaved complex128, column-major) ---------------------------

def _c128(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype != np.complex128 or not a.flags["F_CONTIGUOUS"]:
        a = np.asfortranarray(a, dtype=np.complex128)
    return a


def _zp(a: np.ndarray):
    return a.ctypes.data_as(_c_dp)


def _zld(a: np.ndarray) -> int:
    return max(1, a.shape[0])


def _zargs(side, uplo, trans, diag, alpha, A, B):
    A, B = _c128(A), _c128(B)
    m, n = B.shape
    ka = m if side.upper() == "L" else n
    if A.shape[0] < ka or A.shape[1] < ka:
        raise ValueError(f"A is {A.shape}, side {side} needs order {ka}")
    al = complex(alpha)
    return A, B, m, n, (*_codes(side, uplo, trans, diag), m, n, al.real, al.imag, _zp(A), _zld(A))


def ztrmm(side, uplo, trans, diag, alpha, A, B) -> np.ndarray:
    """Complex TRMM (eqs. (1)/(2), op(A) = A, A^T or conj(A^T)): a new array."""
    A, B, m, n, args = _zargs(side, uplo, trans, diag, alpha, A, B)
    X = B.copy(order="F")
    lib().oracle_ztrmm(*args, _zp(X), _zld(X))
    return X


def ztrsm(side, uplo, trans, diag, alpha, A, B) -> np.ndarray:
    """Complex TRSM (eqs. (3)/(4)) by substitution: a new array."""
    A, B, m, n, args = _zargs(side, uplo, trans, diag, alpha, A, B)
    X = B.copy(order="F")
    lib().oracle_ztrsm(*args, _zp(X), _zld(X))
    return X


def ztrsm_residual(side, uplo, trans, diag, alpha, A, B, X) -> np.ndarray:
    A, B, m, n, args = _zargs(side, uplo, trans, diag, alpha, A, B)
    X = _c128(X)
    R = np.zeros((m, n), dtype=np.complex128, order="F")
    lib().oracle_ztrsm_residual(*args, _zp(B), _zld(B), _zp(X), _zld(X), _zp(R))
    return R


def ztrmm_dot2(side, uplo, trans, diag, alpha, A, B) -> np.ndarray:
    A, B, m, n, args = _zargs(side, uplo, trans, diag, alpha, A, B)
    C = np.zeros((m, n), dtype=np.complex128, order="F")
    lib().oracle_ztrmm_dot2(*args, _zp(B), _zld(B), _zp(C))
    return C


def ztrsm_eta(side, uplo, trans, diag, alpha, A, B, X) -> float:
    A, B, m, n, args = _zargs(side, uplo, trans, diag, alpha, A, B)
    X = _c128(X)
    return float(lib().oracle_ztrsm_eta(*args, _zp(B), _zld(B), _zp(X), _zld(X)))


def ztrmm_eta(side, uplo, trans, diag, alpha, A, B, C) -> float:
    A, B, m, n, args = _zargs(side, uplo, trans, diag, alpha, A, B)
    C = _c128(C)
    return float(lib().oracle_ztrmm_eta(*args, _zp(B), _zld(B), _zp(C), _zld(C)))


def zopnorm(uplo, trans, diag, A, by_rows=True) -> float:
    """|op(A)|_inf (by_rows) or |op(A)|_1, entries measured by their modulus."""
    A = _c128(A)
    return float(lib().oracle_zopnorm(_UPLO[uplo.upper()], _TRANS[trans.upper()], _DIAG[diag.upper()], A.shape[0],
                                      _zp(A), _zld(A), int(bool(by_rows))))


def trtri(uplo, diag, A) -> np.ndarray:
    """A copy of A whose triangle named by uplo (and diagonal unless diag='U')
    holds that triangle of inv(A); the other triangle is copied unchanged."""
    X = _f64(A).copy(order="F")
    n = X.shape[0]
    if X.shape[1] != n:
        raise ValueError("A must be square")
    lib().oracle_trtri(_UPLO[uplo.upper()], _DIAG[diag.upper()], n, _p(X), _ld(X))
    return X


def potrs(uplo, A, B) -> np.ndarray:
    """X with S X = B for S = L L^T (uplo 'L', L the lower triangle of A) or
    S = U^T U (uplo 'U'): the two triangular solves of the factored system,
    in order (L then L^T; U^T then U)."""
    if uplo.upper() == "L":
        return trsm("L", "L", "T", "N", 1.0, A, trsm("L", "L", "N", "N", 1.0, A, B))
    return trsm("L", "U", "N", "N", 1.0, A, trsm("L", "U", "T", "N", 1.0, A, B))


def laswp(B, ipiv, forward=True) -> np.ndarray:
    """Row interchanges of LAPACK's pivot sequence (1-based ipiv): for i in
    order, swap rows i and ipiv[i]-1 of a copy of B (in reverse order when
    forward is False, which applies the inverse permutation)."""
    X = _f64(B).copy(order="F")
    order = range(len(ipiv)) if forward else range(len(ipiv) - 1, -1, -1)
    for i in order:
        p = int(ipiv[i]) - 1
        if p != i:
            X[[i, p], :] = X[[p, i], :]
    return X


def getrs(trans, LU, ipiv, B) -> np.ndarray:
    """X with S X = B (trans 'N') or S^T X = B (trans 'T') for P S = L U, the
    unit lower L and upper U packed in LU with LAPACK's pivot sequence ipiv:
    trans N: rows of B interchanged by ipiv, then L, then U;
    trans T: U^T, then L^T, then the interchanges undone in reverse order."""
    if trans.upper() == "N":
        Y = trsm("L", "L", "N", "U", 1.0, LU, laswp(B, ipiv, True))
        return trsm("L", "U", "N", "N", 1.0, LU, Y)
    Y = trsm("L", "U", "T", "N", 1.0, LU, B)
    return laswp(trsm("L", "L", "T", "U", 1.0, LU, Y), ipiv, False)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """Thread count of later oracle calls (timing only: results do not depend on it)."""
    lib().oracle_set_threads(int(n))
