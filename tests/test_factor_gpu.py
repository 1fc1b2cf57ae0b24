"""Factor objects (rtri_factor_*) on the GPU: one triangular factor against
many right-hand sides.  The factor keeps the packed diagonal blocks, the
GEMM-type copy of A and |op(A)| between calls, so every call after the first
skips those passes; the results must be bit for bit those of the plain entry
points (rtri_dtrsm / rtri_dtrmm / rtri_strsm / rtri_strmm / rtri_dtrsm_mixed)
with the same handle, and meet the oracle's bounds."""
import numpy as np
import pytest

import synth
from gpu_util import TOL, eta, rounded, say, torch_dtype

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
    return synth.rng(synth.W_TEST, 4000, *k)


def _plain(rt, h, op, side, uplo, trans, diag, alpha, Ad, B, td):
    Bd = rt.to_device(B, td)
    (rt.trsm if op == "trsm" else rt.trmm)(h, side, uplo, trans, diag, alpha, Ad, Bd)
    torch.cuda.synchronize()
    return rt.to_host(Bd).astype(np.float64)


def _fac(rt, h, f, op, side, trans, alpha, B, td, **kw):
    Bd = rt.to_device(B, td)
    info = f.trsm(h, side, trans, alpha, Bd, **kw) if op == "trsm" else f.trmm(h, side, trans, alpha, Bd)
    torch.cuda.synchronize()
    return rt.to_host(Bd).astype(np.float64), info


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("uplo", "LU")
def test_factor_plain_bitwise(rt, h, orc, dt, diag, uplo):
    """All side / trans combinations, three leaf sizes and right-hand-side
    widths (both TRMM leaf schedules) on one factor, each call twice: bitwise
    equal to the plain call, within the oracle's bound."""
    ka = 700
    td = torch_dtype(dt)
    g = G(1, dt == "f64", uplo == "U", diag == "U")
    A = rounded(synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress"), dt)
    Ad = rt.to_device(A, td)
    f = rt.Factor(h, uplo, diag, Ad)
    opt = rt.OPT_LEAF_F64 if dt == "f64" else rt.OPT_LEAF_F32
    for side in "LR":
        for trans in "NTC":
            for nv, leaf in ((33, 32), (300, 128), (9000, 0)):
                h.set_option(opt, leaf)   # a kept pack per leaf size
                m, n = (ka, nv) if side == "L" else (nv, ka)
                B = rounded(synth.dense(m, n, g), dt)
                for op in ("trsm", "trmm"):
                    say("factor", dt, uplo, diag, side, trans, nv, op)
                    want = _plain(rt, h, op, side, uplo, trans, diag, -0.5, Ad, B, td)
                    for _ in range(2):
                        got, _ = _fac(rt, h, f, op, side, trans, -0.5, B, td)
                        assert np.array_equal(got, want), (dt, uplo, diag, side, trans, nv, op)
                    if nv == 33:
                        assert eta(orc, op, side, uplo, trans, diag, -0.5, A, B, got) <= TOL[dt]
    say("  factor bytes", f.bytes())
    assert f.bytes() > 0
    f.close()


@pytest.mark.parametrize("gemm", ["bf16", "f32"])
@pytest.mark.parametrize("side,uplo,trans", [("L", "L", "N"), ("L", "U", "T"), ("R", "U", "N"), ("R", "L", "T")])
def test_factor_mixed_bitwise(rt, h, orc, gemm, side, uplo, trans):
    """Refined solves through a factor: bitwise equal to rtri_dtrsm_mixed, the
    same iteration count and backward error, and the oracle's eta <= 1e-12.
    The second and third calls reuse the kept copy, blocks and norm: the
    factor's memory does not grow after the first."""
    m, n = (640, 96) if side == "L" else (96, 640)
    ka = 640
    say("factor mixed", gemm, side, uplo, trans)
    g = G(2, gemm == "bf16", side == "L")
    A = synth.tri(ka, uplo, g, "cond", c=8.0)
    B = synth.dense(m, n, g)
    Ad = rt.to_device(A, torch.float64)
    Bd = rt.to_device(B, torch.float64)
    ref = rt.trsm_mixed(h, side, uplo, trans, "N", 1.25, Ad, Bd, gemm=gemm, tol=1e-12, max_iter=30)
    torch.cuda.synchronize()
    want = rt.to_host(Bd)
    f = rt.Factor(h, uplo, "N", Ad)
    sizes = []
    for _ in range(3):
        got, info = _fac(rt, h, f, "trsm", side, trans, 1.25, B, torch.float64, precision=f"mixed_{gemm}", tol=1e-12,
                         max_iter=30)
        sizes.append(f.bytes())
        assert np.array_equal(got, want)
        assert info["iters"] == ref["iters"] and info["eta"] == ref["eta"] and info["anorm"] == ref["anorm"]
    e = orc.trsm_eta(side, uplo, trans, "N", 1.25, A, B, got)
    say("  iters", info["iters"], "eta", info["eta"], "oracle", e, "bytes", sizes)
    assert info["converged"] and e <= 1e-12
    assert sizes[0] > 0 and sizes[0] == sizes[1] == sizes[2]
    f.close()


def test_factor_copy_outlives_input(rt, h, orc):
    """With copy=True the factor keeps its own A: overwriting the caller's
    tensor afterwards changes nothing."""
    ka, n = 500, 40
    g = G(3)
    A = synth.tri(ka, "L", g, "stress")
    B = synth.dense(ka, n, g)
    Ad = rt.to_device(A, torch.float64)
    f = rt.Factor(h, "L", "N", Ad, copy=True)
    want = _plain(rt, h, "trsm", "L", "L", "N", "N", 1.0, Ad, B, torch.float64)
    Ad.fill_(float("nan"))
    got, _ = _fac(rt, h, f, "trsm", "L", "N", 1.0, B, torch.float64)
    assert np.array_equal(got, want)
    got, info = _fac(rt, h, f, "trsm", "L", "N", 1.0, B, torch.float64, precision="mixed_f32")
    assert info["converged"] and orc.trsm_eta("L", "L", "N", "N", 1.0, A, B, got) <= 1e-12
    f.close()


def test_factor_across_streams(rt, orc):
    """Parts made on one handle's stream and used from another handle on a
    second stream (the second waits for them on the device): same bits."""
    ka, n = 900, 300
    g = G(4)
    A = synth.tri(ka, "U", g, "stress")
    B = synth.dense(ka, n, g)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    h1, h2 = rt.Handle(s1), rt.Handle(s2)
    Ad = rt.to_device(A, torch.float64)
    torch.cuda.synchronize()
    f = rt.Factor(h1, "U", "N", Ad)
    outs = []
    for hh, st in ((h1, s1), (h2, s2), (h2, s2)):
        Bd = rt.to_device(B, torch.float64)
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            f.trsm(hh, "L", "T", 1.0, Bd, precision="mixed_bf16")
        st.synchronize()
        outs.append(rt.to_host(Bd))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
    assert orc.trsm_eta("L", "U", "T", "N", 1.0, A, B, outs[0]) <= 1e-12
    f.close()
    h1.close()
    h2.close()


def test_factor_alpha_zero_and_empty(rt, h):
    ka = 64
    Ad = torch.full((ka, ka), float("nan"), dtype=torch.float64, device="cuda").t()
    f = rt.Factor(h, "L", "N", Ad)
    B = torch.ones((ka, 5), dtype=torch.float64, device="cuda").t().contiguous().t()
    f.trsm(h, "L", "N", 0.0, B, precision="mixed_f32")
    f.trmm(h, "L", "N", 0.0, B)
    torch.cuda.synchronize()
    assert torch.count_nonzero(B).item() == 0
    E = torch.zeros((0, ka), dtype=torch.float64, device="cuda").t()
    info = f.trsm(h, "L", "N", 1.0, E, precision="mixed_bf16")
    assert info["converged"]
    f.close()
