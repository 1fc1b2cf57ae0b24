"""Pins of the complex oracle (eqs. (1)-(4) with op(A) = A, A^T or conj(A^T);
no GPU).  Each pin targets a different way it could be wrong:
  real inputs reduce to the real oracle (bitwise)      -> the complex formulas' real parts
  conj(A^T) equals A^T of the conjugate (bitwise)      -> the conjugation
  exact Gaussian integers vs Gaussian-rational GE      -> every index, sign, order, transpose
  host BLAS (scipy ztrsm / ztrmm)                      -> whole-operation agreement
  round trip, backward-error closed form, Dot2 bound   -> invariants and the metrics"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg.blas as sblas

import synth
from dense_ref import VARIANTS, VARIANTS_NT, exact_ztrmm, exact_ztrsm, grat_to_c128_exact, to_grat, zdense_op

RNG = lambda *k: synth.rng(synth.W_TEST, 9000, *k)  # noqa: E731


def ztri(n, uplo, g, kind="stress", fill=np.nan):
    """Complex triangle: the real generator for both parts (imaginary part of
    the diagonal 0.5 * U(0,1))."""
    re = synth.tri(n, uplo, g, kind, fill=fill)
    im = synth.tri(n, uplo, g, kind, fill=fill)
    if kind != "unit":
        im[np.diag_indices(n)] = 0.5 * g.random(n)
    return np.asfortranarray(re + 1j * im)


def zdense(m, n, g):
    return np.asfortranarray(synth.dense(m, n, g) + 1j * synth.dense(m, n, g))


def _ka(side, m, n):
    return m if side == "L" else n


@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
@pytest.mark.parametrize("diag", "NU")
def test_real_inputs_reduce_to_real_oracle(orc, side, uplo, trans, diag):
    g = RNG(1)
    m, n = 13, 9
    ka = _ka(side, m, n)
    A = synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress")
    B = synth.dense(m, n, g)
    for zf, rf in ((orc.ztrsm, orc.trsm), (orc.ztrmm, orc.trmm)):
        z = zf(side, uplo, trans, diag, -1.25, A.astype(np.complex128), B.astype(np.complex128))
        r = rf(side, uplo, trans, diag, -1.25, A, B)
        assert np.array_equal(z.real, r) and np.all(z.imag == 0)


@pytest.mark.parametrize("side", "LR")
@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("diag", "NU")
def test_conj_transpose_is_transpose_of_conjugate(orc, side, uplo, diag):
    g = RNG(2)
    m, n = 11, 8
    ka = _ka(side, m, n)
    A = ztri(ka, uplo, g, "unit" if diag == "U" else "stress")
    B = zdense(m, n, g)
    Ac = np.asfortranarray(np.conj(A))
    for fn in (orc.ztrsm, orc.ztrmm):
        assert np.array_equal(fn(side, uplo, "C", diag, 0.5 - 1j, A, B), fn(side, uplo, "T", diag, 0.5 - 1j, Ac, B))


@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
@pytest.mark.parametrize("diag", "NU")
def test_exact_gaussian_integers(orc, side, uplo, trans, diag):
    """Gaussian-integer entries with unit-modulus diagonals (+-1, +-i), so every
    quotient is exact: the substitution and the product equal the exact
    Gaussian-rational results bit for bit."""
    g = RNG(3, ord(side), ord(uplo), ord(trans), ord(diag))
    for trial in range(2):
        m = int(g.integers(1, 12))
        n = int(g.integers(1, 5))
        if side == "R":
            m, n = n, m
        ka = _ka(side, m, n)
        re = g.integers(-1, 2, size=(ka, ka)).astype(np.float64)
        im = g.integers(-1, 2, size=(ka, ka)).astype(np.float64)
        A = np.asfortranarray(re + 1j * im)
        units = np.array([1, -1, 1j, -1j])
        A[np.diag_indices(ka)] = units[g.integers(0, 4, size=ka)]
        mask = np.triu(np.ones((ka, ka), bool), 1) if uplo == "L" else np.tril(np.ones((ka, ka), bool), -1)
        A[mask] = np.nan
        if diag == "U":
            A[np.diag_indices(ka)] = np.nan
        B = np.asfortranarray(g.integers(-4, 5, size=(m, n)) + 1j * g.integers(-4, 5, size=(m, n)))
        alpha = (1 + 1j) if trial else 1.0
        want = grat_to_c128_exact(exact_ztrsm(side, uplo, trans, diag, alpha, A, B))
        assert np.array_equal(orc.ztrsm(side, uplo, trans, diag, alpha, A, B), want), (m, n)
        want = grat_to_c128_exact(exact_ztrmm(side, uplo, trans, diag, alpha, A, B))
        assert np.array_equal(orc.ztrmm(side, uplo, trans, diag, alpha, A, B), want), (m, n)


@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
@pytest.mark.parametrize("diag", "NU")
def test_against_host_blas(orc, side, uplo, trans, diag):
    g = RNG(4)
    for (m, n) in [(1, 1), (7, 3), (33, 17)]:
        ka = _ka(side, m, n)
        A = ztri(ka, uplo, g, "unit" if diag == "U" else "stress")
        B = zdense(m, n, g)
        kw = dict(side=int(side == "R"), lower=int(uplo == "L"), trans_a={"N": 0, "T": 1, "C": 2}[trans],
                  diag=int(diag == "U"))
        alpha = 0.75 - 0.5j
        Az = np.nan_to_num(A, nan=0.0)
        ref = sblas.ztrsm(alpha, Az, B, **kw)
        got = orc.ztrsm(side, uplo, trans, diag, alpha, A, B)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
        ref = sblas.ztrmm(alpha, Az, B, **kw)
        got = orc.ztrmm(side, uplo, trans, diag, alpha, A, B)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
def test_round_trip(orc, side, uplo, trans):
    g = RNG(5)
    m, n = 30, 17
    ka = _ka(side, m, n)
    A = ztri(ka, uplo, g, "base")
    X = zdense(m, n, g)
    Y = orc.ztrmm(side, uplo, trans, "N", 1.0, A, X)
    assert np.max(np.abs(orc.ztrsm(side, uplo, trans, "N", 1.0, A, Y) - X)) <= 1e-13


@pytest.mark.parametrize("side", "LR")
@pytest.mark.parametrize("trans", "NTC")
def test_eta_closed_form_and_residual_bound(orc, side, trans):
    """eta of an exact solution is 0; one planted perturbation gives the closed
    form; the compensated residual of a near solution is within the Dot2 bound
    of the exact Gaussian-rational residual."""
    g = RNG(6)
    m, n = (8, 3) if side == "L" else (3, 8)
    ka = _ka(side, m, n)
    re = g.integers(-1, 2, size=(ka, ka)).astype(np.float64)
    im = g.integers(-1, 2, size=(ka, ka)).astype(np.float64)
    A = np.asfortranarray(np.tril(re + 1j * im))
    A[np.diag_indices(ka)] = np.array([1, -1j, 1j, -1, 1, 1j, -1, 1])[:ka]
    B = np.asfortranarray(g.integers(-4, 5, size=(m, n)) + 1j * g.integers(-4, 5, size=(m, n)))
    X = grat_to_c128_exact(exact_ztrsm(side, "L", trans, "N", 2.0, A, B))
    assert orc.ztrsm_eta(side, "L", trans, "N", 2.0, A, B, X) == 0.0
    T = zdense_op(A, "L", trans, "N")
    d = 2.0 ** -20 * (1 + 1j)
    Xp = X.copy(order="F")
    if side == "L":
        Xp[2, 1] += d
        r = np.abs(T[:, 2] * d).max()
        den = np.abs(T).sum(axis=1).max() * np.abs(Xp[:, 1]).max() + 2.0 * np.abs(B[:, 1]).max()
    else:
        Xp[1, 2] += d
        r = np.abs(T[2, :] * d).max()
        den = np.abs(T).sum(axis=0).max() * np.abs(Xp[1, :]).max() + 2.0 * np.abs(B[1, :]).max()
    assert orc.ztrsm_eta(side, "L", trans, "N", 2.0, A, B, Xp) == pytest.approx(r / den, rel=1e-12)
    # compensated residual of a non-exact near solution against exact rationals
    Ar = ztri(ka, "L", g, "stress", fill=0.0)
    Br = zdense(m, n, g)
    Tr = zdense_op(Ar, "L", trans, "N")
    Xn = np.linalg.solve(Tr, Br) if side == "L" else np.linalg.solve(Tr.T, Br.T).T
    Xn = np.asfortranarray(Xn)
    R = orc.ztrsm_residual(side, "L", trans, "N", 1.0, Ar, Br, Xn)
    Tf, Bf, Xf = to_grat(Tr), to_grat(Br), to_grat(Xn)
    u = 2.0 ** -53
    nt = 4 * (ka + 1)
    gam = nt * u / (1 - nt * u)
    for i in range(m):
        for j in range(n):
            terms = [Tf[i][k] * Xf[k][j] for k in range(ka)] if side == "L" else [Xf[i][k] * Tf[k][j] for k in range(ka)]
            ex = Bf[i][j] - sum(terms, Fraction(0))
            mag = abs(complex(float(Bf[i][j].re), float(Bf[i][j].im))) + sum(
                abs(complex(float(t.re), float(t.im))) for t in terms)
            for part, got in ((ex.re, R[i, j].real), (ex.im, R[i, j].imag)):
                assert abs(got - float(part)) <= u * abs(float(part)) + 2 * gam * gam * mag
