"""The operations built on the recursive TRSM, on the GPU, against the oracle:

* TRTRI: the inverse against the oracle's column-by-column substitution
  (elementwise, relative to the inverse's size), its residual X op(A) - I and
  op(A) X - I measured by the oracle's compensated product (the TRMM error
  metric with C = I, within the TRMM tolerance), the untouched other
  triangle, and bit for bit on exact small integers.
* POTRS / GETRS: the solution against the oracle's two substitutions (and row
  interchanges), and the backward error of the factored system
  |B - F1 F2 X| / (|F1| |F2| |X| + |B|), the product formed by the oracle's
  compensated multiply.  Every test prints its case first."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from dense_ref import dense_op, frac_solve, frac_to_f64_exact, to_frac
from gpu_util import TOL, rounded, say, torch_dtype

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_13821_amd as rt
    return rt


@pytest.fixture()
def h(rt):
    hd = rt.Handle()
    yield hd
    hd.close()


def G(*k):
    return synth.rng(synth.W_TEST, 8000, *k)


def _inverse_eta(orc, uplo, diag, A, X):
    """max of the two normwise residuals of a computed inverse X of op(A) = A:
    rows of X A - I (side R metric) and columns of A X - I (side L metric)."""
    n = A.shape[0]
    Xd = np.asfortranarray(dense_op(X, uplo, "N", diag))
    eye = np.eye(n, order="F")
    return max(orc.trmm_eta("R", uplo, "N", diag, 1.0, A, Xd, eye), orc.trmm_eta("L", uplo, "N", diag, 1.0, A, Xd, eye))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("n", [1, 63, 64, 65, 300, 1000])
def test_trtri(rt, h, orc, dt, diag, uplo, n):
    say("trtri", dt, uplo, diag, n)
    g = G(1, n, dt == "f64", uplo == "U", diag == "U")
    A = rounded(synth.tri(n, uplo, g, "unit" if diag == "U" else "stress"), dt)   # NaN off the triangle
    Ad = rt.to_device(A, torch_dtype(dt))
    rt.trtri(h, uplo, diag, Ad)
    torch.cuda.synchronize()
    X = rt.to_host(Ad).astype(np.float64)
    tri = np.tril if uplo == "L" else np.triu
    inner = tri(np.ones((n, n), bool), -1 if uplo == "L" else 1)
    # the other triangle keeps its NaN, a unit diagonal is not written
    assert np.all(np.isnan(X[~inner & ~np.eye(n, dtype=bool)]))
    if diag == "U":
        assert np.all(np.isnan(np.diag(X)))
    e = _inverse_eta(orc, uplo, diag, A, X)
    Xo = orc.trtri(uplo, diag, A)
    Td, Tod = dense_op(X, uplo, "N", diag), dense_op(Xo, uplo, "N", diag)
    fwd = float(np.max(np.abs(Td - Tod)) / np.max(np.abs(Tod)))
    say("  eta", e, "fwd", fwd)
    assert e <= TOL[dt], (dt, uplo, diag, n, e)
    assert fwd <= 100 * TOL[dt], fwd


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("uplo", "LU")
def test_trtri_exact(rt, h, orc, dt, uplo):
    """Unit-diagonal and power-of-two-diagonal integer triangles across several
    base blocks: every entry of the inverse is an exact dyadic rational, so the
    result equals the rational inverse bit for bit."""
    n = 24 if dt == "f32" else 150
    say("trtri exact", dt, uplo, n)
    g = G(2, dt == "f64", uplo == "U")
    A = synth.exact_tri(n, uplo, g, offdiag=(0.0, 0.0, 0.0, 1.0, -1.0), diag=(1.0, -1.0))
    if dt == "f64":   # bidiagonal keeps the inverse's entries small
        A[np.tril_indices(n, -2) if uplo == "L" else np.triu_indices(n, 2)] = 0.0
    Ad = rt.to_device(A, torch_dtype(dt))
    rt.trtri(h, uplo, "N", Ad)
    torch.cuda.synchronize()
    X = rt.to_host(Ad).astype(np.float64)
    want = frac_to_f64_exact(frac_solve(to_frac(dense_op(A, uplo, "N", "N")), to_frac(np.eye(n))))
    mask = (np.tril if uplo == "L" else np.triu)(np.ones((n, n), bool))
    assert np.array_equal(X[mask], want[mask])
    assert np.array_equal(X[mask], orc.trtri(uplo, "N", A)[mask])


def _two_eta(orc, F1, F2, X, B):
    """|B - F1 (F2 X)| / (|F1| |F2| |X| + |B|), per column, max; F1, F2 dense
    triangular (explicit) matrices, the products compensated by the oracle."""
    n = F1.shape[0]
    lo1 = bool(np.all(np.triu(F1, 1) == 0))
    lo2 = bool(np.all(np.triu(F2, 1) == 0))
    W = orc.trmm_dot2("L", "L" if lo2 else "U", "N", "N", 1.0, np.asfortranarray(F2), X)
    P = orc.trmm_dot2("L", "L" if lo1 else "U", "N", "N", 1.0, np.asfortranarray(F1), W)
    n1, n2 = np.abs(F1).sum(axis=1).max(), np.abs(F2).sum(axis=1).max()
    r = np.abs(B - P).max(axis=0)
    den = n1 * n2 * np.abs(X).max(axis=0) + np.abs(B).max(axis=0)
    assert n == X.shape[0]
    return float(np.max(r / den))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("n,nrhs", [(300, 7), (2048, 96)])
def test_potrs(rt, h, orc, dt, uplo, n, nrhs):
    say("potrs", dt, uplo, n, nrhs)
    g = G(3, n, dt == "f64", uplo == "U")
    A = rounded(synth.tri(n, uplo, g, "stress"), dt)
    B = rounded(synth.dense(n, nrhs, g), dt)
    td = torch_dtype(dt)
    Ad, Bd = rt.to_device(A, td), rt.to_device(B, td)
    rt.potrs(h, uplo, Ad, Bd)
    torch.cuda.synchronize()
    X = rt.to_host(Bd).astype(np.float64)
    T = dense_op(A, uplo, "N", "N")
    F1, F2 = (T, T.T) if uplo == "L" else (T.T, T)
    e = _two_eta(orc, F1, F2, X, B)
    Xo = orc.potrs(uplo, A, B)
    fwd = float(np.max(np.abs(X - Xo)) / np.max(np.abs(Xo)))
    say("  eta", e, "fwd", fwd)
    assert e <= 2 * TOL[dt], e
    assert fwd <= 100 * TOL[dt], fwd


def _lu_system(n, g):
    """A random system with a pivoted LU from the host LAPACK (a factorisation
    given to the solver, not part of what is tested)."""
    S = synth.dense(n, n, g)
    lu, piv = sla.lu_factor(S)
    return S, np.asfortranarray(lu), (piv + 1).astype(np.int32)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("trans", "NT")
@pytest.mark.parametrize("n,nrhs", [(300, 5), (1500, 130)])
def test_getrs(rt, h, orc, dt, trans, n, nrhs):
    say("getrs", dt, trans, n, nrhs)
    g = G(4, n, dt == "f64", trans == "T")
    S, lu, ipiv = _lu_system(n, g)
    LU = rounded(lu, dt)
    B = rounded(synth.dense(n, nrhs, g), dt)
    td = torch_dtype(dt)
    LUd, Bd = rt.to_device(LU, td), rt.to_device(B, td)
    rt.getrs(h, trans, LUd, ipiv, Bd)
    torch.cuda.synchronize()
    X = rt.to_host(Bd).astype(np.float64)
    Xo = orc.getrs(trans, LU, ipiv, B)
    fwd = float(np.max(np.abs(X - Xo)) / np.max(np.abs(Xo)))
    Lm = dense_op(LU, "L", "N", "U")
    Um = dense_op(LU, "U", "N", "N")
    if trans == "N":   # L U X = P B
        e = _two_eta(orc, Lm, Um, X, orc.laswp(B, ipiv, True))
    else:              # U^T L^T (P X) = B
        e = _two_eta(orc, Um.T, Lm.T, orc.laswp(X, ipiv, True), B)
    say("  eta", e, "fwd", fwd)
    assert e <= 2 * TOL[dt], e
    # the system's own condition enters the forward error: compare at its scale
    kappa = np.linalg.cond(S, 1)
    assert fwd <= max(100.0, kappa) * TOL[dt], (fwd, kappa)


def test_getrs_identity_pivots_and_bad_ipiv(rt, h, orc):
    n, nrhs = 200, 9
    g = G(5)
    L = synth.tri(n, "L", g, "unit", fill=0.0)
    U = synth.tri(n, "U", g, "stress", fill=0.0)
    LU = np.where(np.tril(np.ones((n, n), bool), -1), L, U).copy(order="F")
    ipiv = np.arange(1, n + 1, dtype=np.int32)    # no interchanges
    B = synth.dense(n, nrhs, g)
    LUd, Bd = rt.to_device(LU, torch.float64), rt.to_device(B, torch.float64)
    rt.getrs(h, "N", LUd, ipiv, Bd)
    torch.cuda.synchronize()
    want = orc.trsm("L", "U", "N", "N", 1.0, LU, orc.trsm("L", "L", "N", "U", 1.0, LU, B))
    assert np.max(np.abs(rt.to_host(Bd) - want)) <= 1e-12 * np.max(np.abs(want))
    bad = ipiv.copy()
    bad[3] = n + 1
    with pytest.raises(rt.RtriError):
        rt.getrs(h, "N", LUd, bad, Bd)
