"""The INT8-product TRMM (rtri_dtrmm_ozaki: the modular Ozaki scheme, FP64
accuracy from exact INT8 matrix-core products) against the oracle.

Bound (stated in the header): with row exponents e_i of op(A) (max_k
|op(A)_ik| < 2^e_i), column exponents f_j of B, and beta = min(55,
floor((log2 P - 2 - log2 K) / 2)) kept bits (P the product of the 16 moduli),
    |W_ij - (alpha op(A) B)_ij| <= |alpha| (2^(e_i-beta-1) ||B_:j||_1
        + 2^(f_j-beta-1) ||op(A)_i:||_1 + K 2^(e_i+f_j-2 beta-2))
        + 2 u (|W_exact| + that)
(side R: the same with the roles of rows and columns exchanged).  The exact
product comes from the oracle's compensated TRMM.  Small-integer inputs are
scaled exactly, so the result must equal the oracle's bit for bit."""
import numpy as np
import pytest

import synth
from dense_ref import dense_op
from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = 2.0 ** -53
MODULI = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191]


def beta_for(K):
    lp = float(np.sum(np.log2(np.array(MODULI, dtype=np.float64))))
    return min(55, int(np.floor((lp - 2.0 - np.log2(max(K, 1))) / 2.0)))


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


def _exp_of_max(x, axis):
    mx = np.max(np.abs(x), axis=axis)
    _, e = np.frexp(mx)
    return np.where(mx > 0, e, -1100).astype(np.int64)


def _bound(side, uplo, trans, diag, alpha, A, B, W_exact):
    opA = dense_op(A, uplo, trans, diag)
    if side == "L":
        P, Q = opA, B
    else:
        P, Q = B, opA
    K = P.shape[1]
    BETA = beta_for(K)
    e = _exp_of_max(P, 1)[:, None].astype(np.float64)
    f = _exp_of_max(Q, 0)[None, :].astype(np.float64)
    q1 = np.sum(np.abs(Q), axis=0)[None, :]
    p1 = np.sum(np.abs(P), axis=1)[:, None]
    b = abs(alpha) * (np.exp2(e - BETA - 1) * q1 + np.exp2(f - BETA - 1) * p1 + K * np.exp2(e + f - 2 * BETA - 2))
    return b + 2 * U * (np.abs(W_exact) + b)


CASES = [("L", "L", "N", "N", 300, 200), ("L", "U", "T", "U", 517, 129), ("L", "U", "N", "N", 256, 256),
         ("L", "L", "T", "N", 1100, 70), ("R", "L", "N", "N", 150, 333), ("R", "U", "T", "U", 90, 700),
         ("R", "U", "N", "N", 257, 256), ("R", "L", "T", "N", 64, 1030)]


@pytest.mark.parametrize("case", CASES)
def test_ozaki_trmm_bound(rt, h, orc, case):
    side, uplo, trans, diag, m, n = case
    say("ozaki", case)
    g = synth.rng(synth.W_TEST, 7400, m, n)
    ka = m if side == "L" else n
    A = synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress")
    B = synth.dense(m, n, g)
    alpha = -1.25
    Ad = rt.to_device(A, torch.float64)
    Bd = rt.to_device(B, torch.float64)
    rt.trmm_ozaki(h, side, uplo, trans, diag, alpha, Ad, Bd)
    torch.cuda.synchronize()
    W = rt.to_host(Bd)
    W_exact = orc.trmm_dot2(side, uplo, trans, diag, alpha, A, B)
    bound = _bound(side, uplo, trans, diag, alpha, A, B, W_exact)
    err = np.abs(W - W_exact)
    assert np.all(err <= bound), (case, float(np.max(err / bound)))
    # the normwise error the refined solve's residual sees
    eta = orc.trmm_eta(side, uplo, trans, diag, alpha, A, B, W)
    say("ozaki eta", eta)
    assert eta <= 1e-14, (case, eta)


@pytest.mark.parametrize("case", CASES[:4])
def test_ozaki_trmm_exact_integers(rt, h, orc, case):
    """Integer inputs scale exactly (powers of two): the product is exact."""
    side, uplo, trans, diag, m, n = case
    say("ozaki exact", case)
    g = synth.rng(synth.W_TEST, 7401, m, n)
    ka = m if side == "L" else n
    A = g.integers(-2, 3, size=(ka, ka)).astype(np.float64)
    np.fill_diagonal(A, g.choice([-2.0, -1.0, 1.0, 2.0], size=ka))
    B = g.integers(-8, 9, size=(m, n)).astype(np.float64)
    Ad = rt.to_device(np.asfortranarray(A), torch.float64)
    Bd = rt.to_device(np.asfortranarray(B), torch.float64)
    rt.trmm_ozaki(h, side, uplo, trans, diag, 2.0, Ad, Bd)
    torch.cuda.synchronize()
    assert np.array_equal(rt.to_host(Bd), orc.trmm(side, uplo, trans, diag, 2.0, A, B))


def test_ozaki_trmm_alpha_zero_and_empty(rt, h):
    say("ozaki alpha=0 / empty")
    A = torch.full((40, 40), float("nan"), dtype=torch.float64, device="cuda").t()
    B = torch.ones((30, 40), dtype=torch.float64, device="cuda").t()
    rt.trmm_ozaki(h, "L", "L", "N", "N", 0.0, A, B)
    torch.cuda.synchronize()
    assert torch.count_nonzero(B).item() == 0
    E = torch.zeros((40, 0), dtype=torch.float64, device="cuda")
    rt.trmm_ozaki(h, "L", "L", "N", "N", 1.0, A, E)


# ---- the refined solve with the INT8 residual product -------------------------------

from dense_ref import VARIANTS_NT  # noqa: E402


def _mixed(rt, h, orc, side, uplo, trans, diag, alpha, A, B, gemm, **kw):
    Ad = rt.to_device(A, torch.float64)
    Bd = rt.to_device(B, torch.float64)
    info = rt.trsm_mixed(h, side, uplo, trans, diag, alpha, Ad, Bd, gemm=gemm, **kw)
    torch.cuda.synchronize()
    X = rt.to_host(Bd)
    return X, info, orc.trsm_eta(side, uplo, trans, diag, alpha, A, B, X)


@pytest.mark.parametrize("gemm", ["bf16", "f32"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("side,uplo,trans", VARIANTS_NT)
def test_mixed_int8_residual_variants(rt, h, orc, gemm, diag, side, uplo, trans):
    m, n = (300, 70) if side == "L" else (70, 300)
    say("mixed int8 residual", gemm, side, uplo, trans, diag)
    g = synth.rng(synth.W_TEST, 7402, m, 1 if diag == "U" else 0)
    ka = m if side == "L" else n
    A = synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress")
    B = synth.dense(m, n, g)
    h.set_option(rt.OPT_RESIDUAL, 1)
    X, info, e = _mixed(rt, h, orc, side, uplo, trans, diag, -0.75, A, B, gemm)
    assert info["converged"] and e <= 1e-12, (info, e)
    assert e <= 4 * max(info["eta"], 1e-16)


@pytest.mark.parametrize("gemm", ["bf16", "f32"])
@pytest.mark.parametrize("c", [40.0, 4.5])
def test_mixed_int8_residual_conditioned(rt, h, orc, gemm, c):
    """cond_1 ~1e2 and ~1e6 at m = 1024."""
    m, n = 1024, 64
    g = synth.rng(synth.W_TEST, 7403, int(c * 10))
    A = synth.tri(m, "L", g, "cond", c=c)
    B = synth.dense(m, n, g)
    say("mixed int8 residual cond", gemm, c)
    h.set_option(rt.OPT_RESIDUAL, 1)
    X, info, e = _mixed(rt, h, orc, "L", "L", "N", "N", 1.0, A, B, gemm, max_iter=30)
    assert info["converged"] and e <= 1e-12, (info, e)


def test_factor_int8_residual_matches_plain(rt, h, orc):
    """A factor keeps op(A)'s residue planes; its refined solve equals the plain
    entry point's bit for bit, on the second call too."""
    m, n = 700, 90
    g = synth.rng(synth.W_TEST, 7404)
    A = synth.tri(m, "U", g, "stress")
    B = synth.dense(m, n, g)
    say("factor int8 residual")
    h.set_option(rt.OPT_RESIDUAL, 1)
    Ad = rt.to_device(A, torch.float64)
    f = rt.Factor(h, "U", "N", Ad)
    try:
        outs = []
        for _ in range(2):
            Bd = rt.to_device(B, torch.float64)
            f.trsm(h, "L", "T", 1.5, Bd, precision="mixed_bf16")
            torch.cuda.synchronize()
            outs.append(rt.to_host(Bd))
        X, info, e = _mixed(rt, h, orc, "L", "U", "T", "N", 1.5, A, B, "bf16")
        assert np.array_equal(outs[0], X) and np.array_equal(outs[1], X)
        assert e <= 1e-12
    finally:
        f.close()
