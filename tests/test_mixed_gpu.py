"""Low-precision paths against the CPU oracle.

* TRMM with BF16 / FP16 inputs and FP32 accumulation: against the oracle run
  on the same (exactly widened) 16-bit values, the error is at the FP32 level;
  small-integer inputs agree bit for bit.
* Mixed-precision TRSM with FP64 refinement: the returned X must have normwise
  backward error <= 1e-12 by the oracle's own (compensated) residual, for GEMM
  updates in BF16 and in FP32, over conditioned factors up to cond_1 ~ 1e6."""
import numpy as np
import pytest

import synth
from dense_ref import VARIANTS_NT
from gpu_util import rounded, say

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
    return synth.rng(synth.W_TEST, 2000, *k)


T16 = {"bf16": "bfloat16", "f16": "float16"}


def _run_trmm_ex(rt, h, side, uplo, trans, diag, alpha, A, B, dt):
    td = getattr(torch, T16[dt])
    Ad = rt.to_device(A, td)
    Bd = rt.to_device(B, td)
    m, n = B.shape
    Cd = torch.full((n, m), float("nan"), dtype=torch.float32, device="cuda").t()
    rt.trmm_ex(h, side, uplo, trans, diag, alpha, Ad, Bd, Cd)
    torch.cuda.synchronize()
    return rt.to_host(Cd).astype(np.float64)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("side,uplo,trans", [("L", "L", "N"), ("R", "U", "T")])
def test_trmm_ex_leaf_schedules_agree(rt, h, orc, dt, side, uplo, trans):
    """The 16-bit TRMM with one launch per leaf and with every leaf in one
    launch (its updates run concurrently): bit-identical results."""
    m, n = (700, 150) if side == "L" else (150, 700)
    say("trmm_ex schedules", dt, side, uplo, trans)
    g = G(3, m)
    ka = m if side == "L" else n
    A = rounded(synth.tri(ka, uplo, g, "stress"), dt)
    B = rounded(synth.dense(m, n, g), dt)
    h.set_option(rt.OPT_LEAF_F32, 64)
    out = []
    for mode in (1, 2):
        h.set_option(rt.OPT_TRMM_LEAVES, mode)
        out.append(_run_trmm_ex(rt, h, side, uplo, trans, "N", 0.5, A, B, dt))
    h.set_option(rt.OPT_TRMM_LEAVES, 0)
    assert np.array_equal(out[0], out[1])
    assert orc.trmm_eta(side, uplo, trans, "N", 0.5, A, B, out[1]) <= 7 * np.sqrt(ka) * 2.0 ** -24


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("side,uplo,trans", VARIANTS_NT)
def test_trmm_ex_parity(rt, h, orc, dt, diag, side, uplo, trans):
    m, n = (300, 90) if side == "L" else (90, 300)
    say("trmm_ex", dt, side, uplo, trans, diag)
    g = G(1, m)
    ka = m if side == "L" else n
    A = rounded(synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress"), dt)
    B = rounded(synth.dense(m, n, g), dt)
    C = _run_trmm_ex(rt, h, side, uplo, trans, diag, 0.5, A, B, dt)
    e = orc.trmm_eta(side, uplo, trans, diag, 0.5, A, B, C)
    # FP32 accumulation over at most ka terms: 7 sqrt(ka) u32 (same margin as the FP32 path)
    assert e <= 7 * np.sqrt(ka) * 2.0 ** -24, e


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("side,uplo,trans", VARIANTS_NT)
def test_trmm_ex_exact(rt, h, orc, dt, side, uplo, trans):
    ka, other = 70, 11
    m, n = (ka, other) if side == "L" else (other, ka)
    say("trmm_ex exact", dt, side, uplo, trans)
    g = G(2, ka)
    A = synth.exact_tri(ka, uplo, g, offdiag=(-1, 0, 1), diag=(1.0, -1.0, 2.0))
    B = synth.exact_dense(m, n, g)
    C = _run_trmm_ex(rt, h, side, uplo, trans, "N", 2.0, A, B, dt)
    assert np.array_equal(C, orc.trmm(side, uplo, trans, "N", 2.0, A, B))


def test_trmm_ex_rejects_types(rt, h):
    A = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    B = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    C = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    rc = rt.rtri_trmm_ex(h.ptr, 0, 0, 0, 0, 4, 4, 1.0, A.data_ptr(), rt.F32, 4, B.data_ptr(), rt.F32, 4,
                         C.data_ptr(), rt.F32, 4)
    assert rc == rt.ERR_UNSUPPORTED


# ---- mixed-precision refined TRSM ------------------------------------------------

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
def test_mixed_variants(rt, h, orc, gemm, diag, side, uplo, trans):
    m, n = (260, 70) if side == "L" else (70, 260)
    say("mixed", gemm, side, uplo, trans, diag)
    g = G(3, m)
    ka = m if side == "L" else n
    A = synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress")
    B = synth.dense(m, n, g)
    X, info, e = _mixed(rt, h, orc, side, uplo, trans, diag, -0.75, A, B, gemm)
    assert info["converged"] and e <= 1e-12, (info, e)
    assert info["eta"] <= 1e-12
    # the library's own eta and the oracle's compensated eta describe the same residual
    assert e <= 4 * max(info["eta"], 1e-16)
    # the norm in that eta: |op(A)|_inf for side L, |op(A)|_1 for side R (each row of X solves with op(A)^T)
    norm = orc.opnorm_inf if side == "L" else orc.opnorm_one
    ref = norm(uplo, trans, diag, A)
    assert abs(info["anorm"] - ref) <= 1e-14 * ref, (info["anorm"], ref)


@pytest.mark.parametrize("gemm", ["bf16", "f32"])
@pytest.mark.parametrize("c", [40.0, 8.0, 4.5])
def test_mixed_conditioned(rt, h, orc, gemm, c):
    """Diagonal c + U(0,1) at m = 1024 spans cond_1 from ~1e2 to ~1e6."""
    m, n = 1024, 64
    g = G(4, int(c * 10))
    A = synth.tri(m, "L", g, "cond", c=c)
    kappa = orc.cond_one("L", "N", A)
    say("mixed cond", gemm, c, f"{kappa:.2e}")
    B = synth.dense(m, n, g)
    X, info, e = _mixed(rt, h, orc, "L", "L", "N", "N", 1.0, A, B, gemm, max_iter=30)
    assert info["converged"] and e <= 1e-12, (kappa, info, e)


def test_mixed_not_converged_status(rt, h, orc):
    m, n = 200, 20
    g = G(5)
    A = synth.tri(m, "U", g, "stress")
    B = synth.dense(m, n, g)
    X, info, e = _mixed(rt, h, orc, "L", "U", "N", "N", 1.0, A, B, "bf16", tol=0.0, max_iter=1,
                        allow_not_converged=True)
    assert info["status"] == rt.NOT_CONVERGED and info["iters"] == 1 and not info["converged"]
    # the iterate after one low-precision solve is returned and is a BF16-level solution
    assert e <= 1e-2


def test_mixed_alpha_zero(rt, h):
    A = torch.full((8, 8), float("nan"), dtype=torch.float64, device="cuda").t()
    B = torch.ones((8, 3), dtype=torch.float64, device="cuda").t().contiguous().t()
    info = rt.trsm_mixed(h, "L", "L", "N", "N", 0.0, A, B)
    torch.cuda.synchronize()
    assert info["converged"] and torch.count_nonzero(B).item() == 0


def test_mixed_zero_rhs(rt, h):
    """alpha B = 0 with alpha != 0: no correction is made and X = 0 is returned."""
    A = torch.full((40, 40), float("nan"), dtype=torch.float64, device="cuda").t()
    B = torch.zeros((40, 5), dtype=torch.float64, device="cuda").t().contiguous().t()
    B.fill_(-0.0)
    info = rt.trsm_mixed(h, "L", "L", "N", "N", 2.0, A, B)
    torch.cuda.synchronize()
    assert info["converged"] and info["iters"] == 0
    assert torch.all(B == 0) and not torch.any(torch.signbit(B))


def test_mixed_8192_sampled(rt, h, orc):
    """The mixed-precision workload size, m = n = 8192, BF16 GEMM updates, checked on sampled columns."""
    m = n = 8192
    g = synth.rng(synth.W_MIXED, 0, 45)
    A = synth.tri(m, "L", g, "cond", c=45.0)
    B = synth.dense(m, n, g)
    say("mixed 8192")
    Ad = rt.to_device(A, torch.float64)
    Bd = rt.to_device(B, torch.float64)
    info = rt.trsm_mixed(h, "L", "L", "N", "N", 1.0, Ad, Bd, gemm="bf16")
    torch.cuda.synchronize()
    idx = np.sort(synth.rng(synth.W_MIXED, 1).choice(n, 8, replace=False))
    Xs = np.asfortranarray(Bd[:, torch.as_tensor(idx, device="cuda")].cpu().numpy())
    e = orc.trsm_eta("L", "L", "N", "N", 1.0, A, np.asfortranarray(B[:, idx]), Xs)
    assert info["converged"] and e <= 1e-12, (info, e)


# ---- the mixed-precision workload: m = n = 8192, three condition classes ---------

C3_OFFSETS = (450.0, 45.0, 17.0)   # diagonal c + U(0,1): cond_1 ~ 1e2, 1e4, 1e6 (tests/golden/c3_cond.json)


@pytest.mark.parametrize("gemm", ["bf16", "f32"])
@pytest.mark.parametrize("c", C3_OFFSETS)
def test_mixed_8192_classes(rt, h, orc, gemm, c):
    """The benchmark's refined solves, on its device-drawn inputs (Philox fill,
    the host twin of which is pinned bit for bit elsewhere): every condition
    class with BF16 and with FP32 GEMM updates, checked on sampled columns
    against the oracle's compensated backward error (<= 1e-12) and against the
    oracle's own solution (forward error within cond_1 * 1e-12)."""
    import json
    import os
    m = n = 8192
    say("mixed 8192", gemm, c)
    Ad = torch.empty((m, m), dtype=torch.float64, device="cuda").t()
    Bd = torch.empty((m, m), dtype=torch.float64, device="cuda").t()
    rt.synth_fill(h, 1, synth.SEED, synth.W_MIXED, 1, Ad, param=c)
    rt.synth_fill(h, 0, synth.SEED, synth.W_MIXED, 2, Bd)
    idx = np.sort(synth.rng(synth.W_MIXED, 2, int(c)).choice(n, 8, replace=False))
    tidx = torch.as_tensor(idx, device="cuda")
    Bs = np.asfortranarray(Bd[:, tidx].cpu().numpy())
    info = rt.trsm_mixed(h, "L", "L", "N", "N", 1.0, Ad, Bd, gemm=gemm, tol=1e-12, max_iter=30)
    torch.cuda.synchronize()
    Xs = np.asfortranarray(Bd[:, tidx].cpu().numpy())
    A = rt.to_host(Ad)
    del Ad, Bd
    e = orc.trsm_eta("L", "L", "N", "N", 1.0, A, Bs, Xs)
    Xo = orc.trsm("L", "L", "N", "N", 1.0, A, Bs)
    fwd = float(np.max(np.abs(Xs - Xo)) / np.max(np.abs(Xo)))
    with open(os.path.join(os.path.dirname(__file__), "golden", "c3_cond.json")) as f:
        kappa = {case["c"]: case["cond1"] for case in json.load(f)["cases"]}[c]
    say("  iters", info["iters"], "lib eta", info["eta"], "oracle eta", e, "fwd", fwd, "cond1", kappa)
    assert info["converged"] and e <= 1e-12, (info, e)
    assert e <= 4 * max(info["eta"], 1e-16)
    assert fwd <= kappa * 1e-12, (fwd, kappa)


# ---- the 16-bit TRMM on its full-tile path ---------------------------------------

@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("side,uplo,trans", [("L", "L", "N"), ("L", "U", "T"), ("R", "U", "N"), ("R", "L", "T")])
def test_trmm_ex_full_tiles(rt, h, orc, dt, side, uplo, trans):
    """Orders and leading dimensions that are multiples of 8 with updates of at
    least 128 x 128 (the 16-bit GEMM's 16-byte full-tile loads with both
    operands 16-bit, the path of the benchmark's TRMM at 8192), with 64- and
    256-row leaves: one launch per leaf (each update its own launch) and every
    leaf in one launch (side L with 256-row leaves: all updates in one grouped
    launch of 256x256 tiles, another MFMA shape, so the two agree to within
    the bound rather than bit for bit); against the oracle on the rounded
    inputs, and bit for bit on small integers (every partial sum an integer
    below 2^24)."""
    for leaf, ka in ((64, 1024), (256, 2048)):
        m, n = (ka, 512) if side == "L" else (512, ka)
        say("trmm_ex full tiles", dt, side, uplo, trans, leaf, ka)
        h.set_option(rt.OPT_LEAF_F32, leaf)
        g = G(6, ka)
        A = rounded(synth.tri(ka, uplo, g, "stress"), dt)
        B = rounded(synth.dense(m, n, g), dt)
        out = []
        for mode in (1, 2):
            h.set_option(rt.OPT_TRMM_LEAVES, mode)
            out.append(_run_trmm_ex(rt, h, side, uplo, trans, "N", 0.5, A, B, dt))
        h.set_option(rt.OPT_TRMM_LEAVES, 0)
        bound = 7 * np.sqrt(ka) * 2.0 ** -24
        for X in out:
            e = orc.trmm_eta(side, uplo, trans, "N", 0.5, A, B, X)
            assert e <= bound, (leaf, e)
        if leaf == 64:
            assert np.array_equal(out[0], out[1])
        Ai = synth.exact_tri(ka, uplo, g, offdiag=(-1, 0, 1), diag=(1.0, -1.0, 2.0, -2.0))
        Bi = synth.exact_dense(m, n, g)
        want = orc.trmm(side, uplo, trans, "N", 1.0, Ai, Bi)
        for mode in (1, 2):
            h.set_option(rt.OPT_TRMM_LEAVES, mode)
            Ci = _run_trmm_ex(rt, h, side, uplo, trans, "N", 1.0, Ai, Bi, dt)
            assert np.array_equal(Ci, want), (leaf, mode)
        h.set_option(rt.OPT_TRMM_LEAVES, 0)
    h.set_option(rt.OPT_LEAF_F32, 0)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("uplo,trans,diag", [("L", "N", "N"), ("L", "T", "U"), ("U", "N", "U"), ("U", "T", "N")])
def test_trmm_ex_grouped_ragged(rt, h, orc, dt, uplo, trans, diag):
    """Side L with 256-row leaves and every leaf in one launch: the updates of
    an output tile go into one FP32 accumulator when their origins fall on
    256-row boundaries (else the updates run depth by depth).  Orders and
    panel widths that are not multiples of 256 (ragged last tiles, ragged K
    segments for the upper / transposed factors), against the oracle on the
    rounded inputs (both schedules) within the FP32-accumulation bound, and
    bit for bit on small integers."""
    ka, n = 1500, 700
    say("trmm_ex grouped ragged", dt, uplo, trans, diag)
    h.set_option(rt.OPT_LEAF_F32, 256)
    g = G(7, ka, ord(uplo), ord(trans), ord(diag))
    A = rounded(synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress"), dt)
    B = rounded(synth.dense(ka, n, g), dt)
    out = []
    for mode in (1, 2):
        h.set_option(rt.OPT_TRMM_LEAVES, mode)
        out.append(_run_trmm_ex(rt, h, "L", uplo, trans, diag, -0.75, A, B, dt))
    h.set_option(rt.OPT_TRMM_LEAVES, 0)
    bound = 7 * np.sqrt(ka) * 2.0 ** -24
    for X in out:
        e = orc.trmm_eta("L", uplo, trans, diag, -0.75, A, B, X)
        assert e <= bound, e
    Ai = synth.exact_tri(ka, uplo, g, offdiag=(-1, 0, 1), diag=(1.0, -1.0, 2.0, -2.0))
    Bi = synth.exact_dense(ka, n, g)
    want = orc.trmm("L", uplo, trans, diag, 1.0, Ai, Bi)
    h.set_option(rt.OPT_TRMM_LEAVES, 2)
    Ci = _run_trmm_ex(rt, h, "L", uplo, trans, diag, 1.0, Ai, Bi, dt)
    h.set_option(rt.OPT_TRMM_LEAVES, 0)
    h.set_option(rt.OPT_LEAF_F32, 0)
    assert np.array_equal(Ci, want)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_trmm_ex_grouped_direct_lds(rt, h, orc, dt):
    """The grouped launch of a 16-bit TRMM whose tiles are all full (order and
    width multiples of 256): the direct-to-LDS kernel (OPT_GEMM16_TILE 0)
    against the register-staged grouped kernel (3), bit for bit (same
    segments in the same order, same MFMA sequence), and against the oracle."""
    ka, n = 2048, 768
    say("trmm_ex grouped direct-to-LDS", dt)
    h.set_option(rt.OPT_LEAF_F32, 256)
    h.set_option(rt.OPT_TRMM_LEAVES, 2)
    g = G(8, ka)
    A = rounded(synth.tri(ka, "L", g, "stress"), dt)
    B = rounded(synth.dense(ka, n, g), dt)
    out = []
    for tile in (0, 3):
        h.set_option(rt.OPT_GEMM16_TILE, tile)
        out.append(_run_trmm_ex(rt, h, "L", "L", "N", "N", 1.5, A, B, dt))
    h.set_option(rt.OPT_GEMM16_TILE, 0)
    h.set_option(rt.OPT_TRMM_LEAVES, 0)
    h.set_option(rt.OPT_LEAF_F32, 0)
    assert np.array_equal(out[0], out[1])
    assert orc.trmm_eta("L", "L", "N", "N", 1.5, A, B, out[0]) <= 7 * np.sqrt(ka) * 2.0 ** -24

