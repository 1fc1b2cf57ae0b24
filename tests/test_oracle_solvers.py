"""Pins of the oracle's neighbouring operations (no GPU): the triangular
inverse (TRTRI) and the two-solve systems of a Cholesky factor (POTRS) and of
an LU factorisation with row interchanges (GETRS), each against what the
mathematics fixes:
  exact integers vs rational Gaussian elimination  -> every index, sign, order
  diagonal closed form (bitwise)                    -> division, unit diagonal
  host LAPACK (scipy dtrtri / dpotrs / dgetrs)      -> whole-operation agreement
  the explicitly formed system (numpy solve)        -> which triangle, which order
  untouched other triangle, inverse of the inverse  -> invariants"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.linalg.lapack as slapack

import synth
from dense_ref import dense_op, frac_matmul, frac_solve, frac_to_f64_exact, to_frac, transpose

RNG = lambda *k: synth.rng(synth.W_TEST, 7000, *k)  # noqa: E731


def _tri_dense(A, uplo, diag):
    return dense_op(A, uplo, "N", diag)


# ---- TRTRI ---------------------------------------------------------------------

@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("diag", "NU")
def test_trtri_exact_integers(orc, uplo, diag):
    """Small-integer triangles whose inverses are exact dyadic rationals: the
    oracle's inverse equals the rational one bit for bit."""
    g = RNG(1, uplo == "U", diag == "U")
    for n in (1, 2, 5, 9, 14):
        dset = (1.0, -1.0) if diag == "U" else (1.0, -1.0, 2.0, -2.0, 4.0)
        A = synth.exact_tri(n, uplo, g, offdiag=(-1, 0, 1), diag=dset)
        if diag == "U":
            np.fill_diagonal(A, np.nan)
        T = _tri_dense(A, uplo, diag)
        want = frac_to_f64_exact(frac_solve(to_frac(T), to_frac(np.eye(n))))
        got = orc.trtri(uplo, diag, A)
        tri = np.tril if uplo == "L" else np.triu
        mask = tri(np.ones((n, n), bool), -1 if uplo == "L" else 1) | (np.eye(n, dtype=bool) & (diag == "N"))
        assert np.array_equal(got[mask], want[mask]), (n, uplo, diag)
        # the other triangle (NaN here) and a unit diagonal are not written
        assert np.all(np.isnan(got[~mask & ~np.eye(n, dtype=bool)]))
        if diag == "U":
            assert np.all(np.isnan(np.diag(got)))


def test_trtri_diagonal(orc):
    d = np.array([3.0, -0.5, 7.0, 1.25, -9.0])
    A = np.diag(d).copy(order="F")
    for uplo in "LU":
        assert np.array_equal(np.diag(orc.trtri(uplo, "N", A)), 1.0 / d)


@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("diag", "NU")
def test_trtri_against_lapack(orc, uplo, diag):
    g = RNG(2)
    for n in (1, 7, 40, 129):
        A = synth.tri(n, uplo, g, "unit" if diag == "U" else "stress", fill=0.0)
        want, info = slapack.dtrtri(A, lower=int(uplo == "L"), unitdiag=int(diag == "U"))
        assert info == 0
        got = orc.trtri(uplo, diag, A)
        T = _tri_dense(want, uplo, diag)
        Gt = _tri_dense(got, uplo, diag)
        assert np.max(np.abs(Gt - T)) <= 1e-13 * np.max(np.abs(T))


@pytest.mark.parametrize("uplo", "LU")
def test_trtri_inverse_of_inverse(orc, uplo):
    g = RNG(3)
    A = synth.tri(60, uplo, g, "stress")
    X = orc.trtri(uplo, "N", orc.trtri(uplo, "N", A))
    T, Tx = _tri_dense(A, uplo, "N"), _tri_dense(X, uplo, "N")
    assert np.max(np.abs(Tx - T)) <= 1e-13 * np.max(np.abs(T))


# ---- POTRS ---------------------------------------------------------------------

@pytest.mark.parametrize("uplo", "LU")
def test_potrs_exact(orc, uplo):
    """Cholesky-type factor with power-of-two diagonal and small-integer
    off-diagonal entries: S = L L^T (or U^T U) and its solution are exact
    rationals, and the two substitutions reproduce them bit for bit."""
    g = RNG(4, uplo == "U")
    for n in (1, 3, 6, 10):
        A = synth.exact_tri(n, uplo, g, offdiag=(-1, 0, 1), diag=(1.0, 2.0))
        B = synth.exact_dense(n, 3, g)
        T = to_frac(_tri_dense(A, uplo, "N"))
        S = frac_matmul(T, transpose(T)) if uplo == "L" else frac_matmul(transpose(T), T)
        want = frac_to_f64_exact(frac_solve(S, to_frac(B)))
        assert np.array_equal(orc.potrs(uplo, A, B), want), (uplo, n)


@pytest.mark.parametrize("uplo", "LU")
def test_potrs_against_formed_system_and_lapack(orc, uplo):
    g = RNG(5)
    n, k = 50, 7
    A = synth.tri(n, uplo, g, "stress", fill=0.0)
    B = synth.dense(n, k, g)
    T = _tri_dense(A, uplo, "N")
    S = T @ T.T if uplo == "L" else T.T @ T
    X = orc.potrs(uplo, A, B)
    assert np.allclose(X, np.linalg.solve(S, B), rtol=1e-12, atol=1e-13)
    Xl, info = slapack.dpotrs(A, B, lower=int(uplo == "L"))
    assert info == 0
    assert np.max(np.abs(X - Xl)) <= 1e-13 * np.max(np.abs(Xl))


# ---- GETRS (and the row interchanges) ----------------------------------------------

def test_laswp_is_the_pivot_permutation(orc):
    g = RNG(6)
    n = 9
    ipiv = np.array([int(g.integers(i, n)) + 1 for i in range(n)], dtype=np.int32)   # 1-based, ipiv[i] >= i+1
    P = np.eye(n)
    for i in range(n):
        p = ipiv[i] - 1
        P[[i, p], :] = P[[p, i], :]
    B = synth.dense(n, 4, g)
    assert np.array_equal(orc.laswp(B, ipiv, True), P @ B)
    assert np.array_equal(orc.laswp(P @ B, ipiv, False), B)


@pytest.mark.parametrize("trans", "NT")
def test_getrs_exact(orc, trans):
    """P S = L U with unit lower L and upper U of small integers (diagonal
    +-1, +-2): S, its solution and every intermediate are exact rationals."""
    g = RNG(7, trans == "T")
    for n in (1, 4, 8):
        L = synth.exact_tri(n, "L", g, offdiag=(-1, 0, 1), diag=(1.0,))
        U = synth.exact_tri(n, "U", g, offdiag=(-1, 0, 1), diag=(1.0, -1.0, 2.0, -2.0))
        LU = np.where(np.tril(np.ones((n, n), bool), -1), L, U).copy(order="F")
        ipiv = np.array([int(g.integers(i, n)) + 1 for i in range(n)], dtype=np.int32)
        P = np.eye(n)
        for i in range(n):
            p = ipiv[i] - 1
            P[[i, p], :] = P[[p, i], :]
        Lf = to_frac(_tri_dense(L, "L", "U"))
        Uf = to_frac(_tri_dense(U, "U", "N"))
        S = frac_matmul(to_frac(P.T), frac_matmul(Lf, Uf))   # P S = L U
        B = synth.exact_dense(n, 3, g)
        Sx = S if trans == "N" else transpose(S)
        want = frac_to_f64_exact(frac_solve(Sx, to_frac(B)))
        assert np.array_equal(orc.getrs(trans, LU, ipiv, B), want), (trans, n)


@pytest.mark.parametrize("trans", "NT")
def test_getrs_against_lapack(orc, trans):
    g = RNG(8)
    n, k = 60, 5
    S = synth.dense(n, n, g) + 0.1 * np.eye(n)
    lu, piv = sla.lu_factor(S)
    ipiv = (piv + 1).astype(np.int32)
    B = synth.dense(n, k, g)
    X = orc.getrs(trans, np.asfortranarray(lu), ipiv, B)
    Xl, info = slapack.dgetrs(lu, piv, B, trans=0 if trans == "N" else 1)
    assert info == 0
    assert np.max(np.abs(X - Xl)) <= 1e-12 * np.max(np.abs(Xl))
    Sx = S if trans == "N" else S.T
    assert np.allclose(Sx @ X, B, rtol=1e-10, atol=1e-10)
