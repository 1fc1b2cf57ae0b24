"""Pins of the CPU oracle against facts the mathematics fixes (no GPU).

Each pin targets a different way the oracle could be wrong:
  identity / diagonal closed forms    -> diagonal handling, alpha, division
  exact integers vs rational GE        -> every index, sign, order and transpose
  host LAPACK/BLAS (scipy dtrsm/dtrmm) -> whole-operation agreement on random data
  round trip, transpose identity,
  storage duality, NaN sentinels,
  power-of-two linearity               -> invariants of eqs. (1)-(4)
  Dot2 residual / eta vs exact         -> the error metrics themselves
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg.blas as sblas

import synth
from dense_ref import (VARIANTS, VARIANTS_NT, dense_op, exact_trmm, exact_trsm, frac_solve, frac_to_f64_exact,
                       to_frac)

RNG = lambda *k: synth.rng(synth.W_TEST, *k)  # noqa: E731


def _ka(side, m, n):
    return m if side == "L" else n


# ---- P1: identity factor ----------------------------------------------------

@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
@pytest.mark.parametrize("diag", "NU")
def test_identity(orc, side, uplo, trans, diag):
    m, n = 9, 7
    ka = _ka(side, m, n)
    g = RNG(1)
    A = np.full((ka, ka), np.nan, order="F")
    tri = np.tril if uplo == "L" else np.triu
    mask = tri(np.ones((ka, ka), bool), -1 if uplo == "L" else 1)
    A[mask] = 0.0
    np.fill_diagonal(A, 1.0 if diag == "N" else np.nan)
    B = synth.dense(m, n, g)
    alpha = 1.5
    want = alpha * B
    assert np.array_equal(orc.trmm(side, uplo, trans, diag, alpha, A, B), want)
    assert np.array_equal(orc.trsm(side, uplo, trans, diag, alpha, A, B), want)


# ---- P2: diagonal factor ----------------------------------------------------

@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
def test_diagonal(orc, side, uplo, trans):
    m, n = 11, 6
    ka = _ka(side, m, n)
    g = RNG(2)
    d = 0.5 + g.random(ka) * 3.0
    A = np.zeros((ka, ka), order="F")
    np.fill_diagonal(A, d)
    B = synth.dense(m, n, g)
    if side == "L":
        mm, dd = d[:, None] * B, B / d[:, None]
    else:
        mm, dd = B * d[None, :], B / d[None, :]
    assert np.array_equal(orc.trmm(side, uplo, trans, "N", 1.0, A, B), mm)
    assert np.array_equal(orc.trsm(side, uplo, trans, "N", 1.0, A, B), dd)


# ---- P3: exact integers against rational Gaussian elimination ----------------

EXACT_CASES = [
    # (op, diag, m-range bound, off-diagonal set, diagonal set)
    ("trsm", "U", 24, (-1, 0, 1), (1.0,)),
    ("trsm", "N", 12, (-1, 0, 1), (1.0, -1.0, 2.0, -2.0, 4.0, -4.0)),
    ("trmm", "N", 40, (-2, -1, 0, 1, 2), (1.0, -1.0, 2.0, -2.0)),
    ("trmm", "U", 40, (-2, -1, 0, 1, 2), (1.0,)),
]


@pytest.mark.parametrize("side,uplo,trans", VARIANTS_NT)
@pytest.mark.parametrize("case", range(len(EXACT_CASES)))
def test_exact_integers(orc, side, uplo, trans, case):
    op, diag, mmax, offd, dset = EXACT_CASES[case]
    g = RNG(3, case)
    for trial in range(2):
        m = int(g.integers(1, mmax + 1))
        n = int(g.integers(1, 6))
        if side == "R":
            m, n = n, m
        ka = _ka(side, m, n)
        A = synth.exact_tri(ka, uplo, g, offdiag=offd, diag=dset)
        if diag == "U":
            np.fill_diagonal(A, np.nan)
        B = synth.exact_dense(m, n, g)
        alpha = 2.0 if trial else 1.0
        if op == "trsm":
            want = frac_to_f64_exact(exact_trsm(side, uplo, trans, diag, alpha, A, B))
            got = orc.trsm(side, uplo, trans, diag, alpha, A, B)
        else:
            want = frac_to_f64_exact(exact_trmm(side, uplo, trans, diag, alpha, A, B))
            got = orc.trmm(side, uplo, trans, diag, alpha, A, B)
        assert np.array_equal(got, want), (op, side, uplo, trans, diag, m, n)


# ---- P4: dense Gaussian elimination (LAPACK gesv) at tiny sizes ---------------

@pytest.mark.parametrize("side,uplo,trans", VARIANTS_NT)
def test_dense_solve_small(orc, side, uplo, trans):
    g = RNG(4)
    for m in range(1, 9):
        n = 3
        ka = _ka(side, m, n)
        A = synth.tri(ka, uplo, g, "stress")
        B = synth.dense(m, n, g)
        T = dense_op(A, uplo, trans, "N")
        want = np.linalg.solve(T, 0.75 * B) if side == "L" else np.linalg.solve(T.T, 0.75 * B.T).T
        got = orc.trsm(side, uplo, trans, "N", 0.75, A, B)
        assert np.allclose(got, want, rtol=1e-13, atol=1e-14)


# ---- host BLAS: scipy's dtrsm / dtrmm on random data -------------------------

def _blas_ref(fn, side, uplo, trans, diag, alpha, A, B):
    Az = np.nan_to_num(A, nan=0.0)
    return fn(alpha, Az, B, side=int(side == "R"), lower=int(uplo == "L"),
              trans_a={"N": 0, "T": 1, "C": 2}[trans], diag=int(diag == "U"))


@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
@pytest.mark.parametrize("diag", "NU")
def test_against_host_blas(orc, side, uplo, trans, diag):
    g = RNG(5)
    for (m, n) in [(1, 1), (7, 3), (33, 17), (64, 40)]:
        ka = _ka(side, m, n)
        A = synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress")
        B = synth.dense(m, n, g)
        alpha = -1.25
        got = orc.trsm(side, uplo, trans, diag, alpha, A, B)
        ref = _blas_ref(sblas.dtrsm, side, uplo, trans, diag, alpha, A, B)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
        got = orc.trmm(side, uplo, trans, diag, alpha, A, B)
        ref = _blas_ref(sblas.dtrmm, side, uplo, trans, diag, alpha, A, B)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


# ---- P5: round trip TRSM(A, TRMM(A, X)) = X ------------------------------------

@pytest.mark.parametrize("side,uplo,trans", VARIANTS_NT)
@pytest.mark.parametrize("diag", "NU")
def test_round_trip(orc, side, uplo, trans, diag):
    g = RNG(6)
    m, n = 50, 23
    ka = _ka(side, m, n)
    A = synth.tri(ka, uplo, g, "unit" if diag == "U" else "base")
    X = synth.dense(m, n, g)
    Y = orc.trmm(side, uplo, trans, diag, 1.0, A, X)
    Z = orc.trsm(side, uplo, trans, diag, 1.0, A, Y)
    assert np.max(np.abs(Z - X)) <= 1e-13


# ---- P6: side R equals side L on the transpose (bitwise) ------------------------

@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("trans", "NT")
@pytest.mark.parametrize("diag", "NU")
def test_transpose_identity(orc, uplo, trans, diag):
    g = RNG(7)
    m, n = 13, 29
    A = synth.tri(n, uplo, g, "unit" if diag == "U" else "stress")
    B = synth.dense(m, n, g)
    flip = "T" if trans == "N" else "N"
    for fn in (orc.trsm, orc.trmm):
        r = fn("R", uplo, trans, diag, 0.5, A, B)
        l = fn("L", uplo, flip, diag, 0.5, A, np.asfortranarray(B.T))
        assert np.array_equal(r, l.T)


# ---- P7: storage duality: (U, N) on A equals (L, T) on A^T ---------------------

@pytest.mark.parametrize("side", "LR")
@pytest.mark.parametrize("diag", "NU")
def test_storage_duality(orc, side, diag):
    g = RNG(8)
    m, n = 21, 17
    ka = _ka(side, m, n)
    A = synth.tri(ka, "U", g, "unit" if diag == "U" else "stress")
    At = np.asfortranarray(A.T)
    B = synth.dense(m, n, g)
    for fn in (orc.trsm, orc.trmm):
        assert np.array_equal(fn(side, "U", "N", diag, 1.0, A, B), fn(side, "L", "T", diag, 1.0, At, B))
        assert np.array_equal(fn(side, "U", "T", diag, 1.0, A, B), fn(side, "L", "N", diag, 1.0, At, B))


# ---- P8: the unreferenced triangle (and unit diagonal) are never read ----------

@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
@pytest.mark.parametrize("diag", "NU")
def test_nan_sentinels(orc, side, uplo, trans, diag):
    g = RNG(9)
    m, n = 19, 12
    ka = _ka(side, m, n)
    A = synth.tri(ka, uplo, g, "unit" if diag == "U" else "base", fill=np.nan)
    A0 = np.nan_to_num(A, nan=0.0)
    if diag == "U":
        np.fill_diagonal(A0, 7.0)   # must be ignored
    B = synth.dense(m, n, g)
    for fn in (orc.trsm, orc.trmm):
        x = fn(side, uplo, trans, diag, 1.0, A, B)
        assert np.all(np.isfinite(x))
        assert np.array_equal(x, fn(side, uplo, trans, diag, 1.0, A0, B))


# ---- P10: power-of-two linearity (bitwise) -------------------------------------

@pytest.mark.parametrize("side,uplo,trans", VARIANTS_NT)
def test_pow2_linearity(orc, side, uplo, trans):
    g = RNG(10)
    m, n = 17, 9
    ka = _ka(side, m, n)
    A = synth.tri(ka, uplo, g, "stress")
    B = synth.dense(m, n, g)
    for fn in (orc.trsm, orc.trmm):
        base = fn(side, uplo, trans, "N", 1.0, A, B)
        assert np.array_equal(fn(side, uplo, trans, "N", 1.0, A, 8.0 * B), 8.0 * base)
        assert np.array_equal(fn(side, uplo, trans, "N", 0.25, A, B), 0.25 * base)


# ---- quick returns -------------------------------------------------------------

def test_empty(orc):
    A = np.eye(3, order="F")
    for shape in [(0, 3), (3, 0)]:
        B = np.zeros(shape, order="F")
        assert orc.trsm("L", "L", "N", "N", 1.0, A, B).shape == shape
        assert orc.trmm("R", "U", "T", "N", 1.0, A, B).shape == shape


# ---- metrics: Dot2 residual and eta against exact rationals --------------------

@pytest.mark.parametrize("side", "LR")
def test_dot2_residual_exact(orc, side):
    """The compensated residual meets the Dot2 error bound of Ogita, Rump and
    Oishi (2005, Prop. 5.5 / Thm. 5.3):  |res - s| <= u|s| + gamma_n^2 sum|terms|
    against the exact rational residual s, even under heavy cancellation."""
    g = RNG(11)
    m, n = 12, 5
    ka = _ka(side, m, n)
    A = synth.tri(ka, "L", g, "stress")
    B = synth.dense(m, n, g)
    X = orc.trsm(side, "L", "N", "N", 1.0, A, B)   # near-exact solution: residual cancels
    R = orc.trsm_residual(side, "L", "N", "N", 1.0, A, B, X)
    T = to_frac(dense_op(A, "L", "N", "N"))
    Bf, Xf = to_frac(B), to_frac(X)
    for i in range(m):
        for j in range(n):
            if side == "L":
                terms = [T[i][k] * Xf[k][j] for k in range(ka)]
            else:
                terms = [Xf[i][k] * T[k][j] for k in range(ka)]
            ex = Bf[i][j] - sum(terms, Fraction(0))
            fe = float(ex)
            u = 2.0 ** -53
            nt = ka + 1
            gam = nt * u / (1 - nt * u)
            bound = u * abs(fe) + gam * gam * (abs(float(Bf[i][j])) + sum(abs(float(t)) for t in terms))
            assert abs(R[i, j] - fe) <= bound


def test_eta_definition(orc):
    """eta is 0 for the exact solution and equals the closed form for a
    single planted perturbation."""
    g = RNG(12)
    m, n = 10, 3
    A = synth.exact_tri(m, "L", g, offdiag=(-1, 0, 1), diag=(1.0, 2.0))
    B = synth.exact_dense(m, n, g)
    X = frac_to_f64_exact(exact_trsm("L", "L", "N", "N", 1.0, A, B))
    assert orc.trsm_eta("L", "L", "N", "N", 1.0, A, B, X) == 0.0
    Xp = X.copy(order="F")
    Xp[4, 1] += 2.0 ** -20
    T = dense_op(A, "L", "N", "N")
    r = np.abs(T[:, 4]).max() * 2.0 ** -20           # residual column 1 = -T[:,4]*delta
    den = np.abs(T).sum(axis=1).max() * np.abs(Xp[:, 1]).max() + np.abs(B[:, 1]).max()
    assert orc.trsm_eta("L", "L", "N", "N", 1.0, A, B, Xp) == pytest.approx(r / den, rel=1e-12)


def test_trmm_eta_definition(orc):
    g = RNG(13)
    m, n = 8, 4
    A = synth.exact_tri(m, "U", g, offdiag=(-2, 0, 2), diag=(1.0, 3.0))
    B = synth.exact_dense(m, n, g)
    C = frac_to_f64_exact(exact_trmm("L", "U", "N", "N", 1.0, A, B))
    assert orc.trmm_eta("L", "U", "N", "N", 1.0, A, B, C) == 0.0
    C2 = C.copy(order="F")
    C2[0, 2] += 1.0
    den = np.abs(dense_op(A, "U", "N", "N")).sum(axis=1).max() * np.abs(B[:, 2]).max()
    assert orc.trmm_eta("L", "U", "N", "N", 1.0, A, B, C2) == pytest.approx(1.0 / den, rel=1e-12)


def test_eta_side_right_uses_row_systems(orc):
    """For side R the backward error of row i is that of the transposed system
    op(A)^T x_i^T = alpha b_i^T: the eta of X for (R, A) equals the eta of X^T
    for (L, A, flipped trans)."""
    g = RNG(14)
    m, n = 7, 11
    A = synth.tri(n, "U", g, "stress")
    B = synth.dense(m, n, g)
    X = orc.trsm("R", "U", "N", "N", 1.0, A, B)
    X[2, 5] += 1e-6
    e_r = orc.trsm_eta("R", "U", "N", "N", 1.0, A, B, X)
    e_l = orc.trsm_eta("L", "U", "T", "N", 1.0, A, np.asfortranarray(B.T), np.asfortranarray(X.T))
    assert e_r == pytest.approx(e_l, rel=1e-14)
    C = orc.trmm("R", "U", "N", "N", 1.0, A, B)
    C[3, 1] += 1e-6
    c_r = orc.trmm_eta("R", "U", "N", "N", 1.0, A, B, C)
    c_l = orc.trmm_eta("L", "U", "T", "N", 1.0, A, np.asfortranarray(B.T), np.asfortranarray(C.T))
    assert c_r == pytest.approx(c_l, rel=1e-14)


def test_cond_one_diagonal(orc):
    d = np.array([1.0, 4.0, 0.5, 2.0])
    A = np.diag(d).copy(order="F")
    assert orc.cond_one("L", "N", A) == pytest.approx(d.max() / d.min(), rel=1e-15)


@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("diag", "NU")
def test_cond_one_exact_nondiagonal(orc, uplo, diag):
    """kappa_1 = |A|_1 |A^-1|_1 of a small integer triangle, the inverse taken
    exactly by rational Gaussian elimination.  The case is chosen so that the
    1-norm and the inf-norm differ for both A and its inverse: a slip that
    takes row sums for column sums (of either factor) cannot pass."""
    g = RNG(15, uplo == "U", diag == "U")
    for _ in range(50):
        A = synth.exact_tri(7, uplo, g, offdiag=(-3, -1, 0, 1, 2), diag=(1.0, 2.0, -4.0, 0.5))
        if diag == "U":
            np.fill_diagonal(A, np.nan)
        T = dense_op(A, uplo, "N", diag)
        inv = frac_solve(to_frac(T), to_frac(np.eye(7)))
        absinv = [[abs(v) for v in row] for row in inv]
        inv_one = max(sum(absinv[i][j] for i in range(7)) for j in range(7))
        inv_inf = max(sum(absinv[i][j] for j in range(7)) for i in range(7))
        a_one, a_inf = np.abs(T).sum(axis=0).max(), np.abs(T).sum(axis=1).max()
        if inv_one != inv_inf and a_one != a_inf:
            break
    else:
        pytest.fail("no discriminating case drawn")
    want = float(Fraction(float(a_one)) * inv_one)
    assert orc.cond_one(uplo, diag, A) == pytest.approx(want, rel=1e-14)
    assert abs(want - float(a_inf) * float(inv_inf)) > 1e-6 * want


# ---- the counter-based input generator against its published answers ----------

def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 published with the Random123
    library (Salmon et al., SC'11): zero, all-ones and pi-digit inputs."""
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
        ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
        ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
         (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
    ]
    for c, k, want in cases:
        got = tuple(int(v) for v in synth.philox4x32_10(*c, *k))
        assert got == want, [hex(v) for v in got]
