"""The 16-bit GEMM update on its own (BF16 / FP16 P and Q, FP32 C, FP32
accumulation), through rtri_gemm_update, in both tile families: 128x128 tiles
of 16x16x32 MFMA blocks and 256x256 tiles of 32x32x16 blocks (taken where both
operands are k-contiguous, op(P) = P^T and op(Q) = Q).

Bound: the inputs are exact 16-bit values, each product is exact in FP32, and
the K-term sums round in FP32, so |got - exact| <= 2 (K + 2) u32 (|beta C| +
|s| |op(P)| |op(Q)|) elementwise.  Small-integer inputs keep every partial sum
exact, so both tile families must then agree bit for bit with the exact
result."""
import numpy as np
import pytest

import synth
from gpu_util import say

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


def _dev(rt, x, dt):
    return rt.to_device(x, dt)


def _operands(M, N, K, tp, tq, g, kind, t16):
    if kind == "int":
        P = g.integers(-3, 4, size=(K, M) if tp == "T" else (M, K)).astype(np.float64)
        Q = g.integers(-3, 4, size=(N, K) if tq == "T" else (K, N)).astype(np.float64)
        C = g.integers(-8, 9, size=(M, N)).astype(np.float64)
    else:
        P = synth.round_to(synth.dense(K, M, g) if tp == "T" else synth.dense(M, K, g), t16)
        Q = synth.round_to(synth.dense(N, K, g) if tq == "T" else synth.dense(K, N, g), t16)
        C = synth.round_to(synth.dense(M, N, g), "f32")
    return np.asfortranarray(P), np.asfortranarray(Q), np.asfortranarray(C)


# (M, N, K): one tile, ragged edges in every dimension, several wide tiles with
# K not a multiple of the 64-deep k step, and shapes large enough for the
# automatic choice to take the wide tiles
SHAPES = [(1, 1, 1), (37, 50, 19), (256, 256, 64), (300, 520, 77), (777, 515, 131), (1024, 768, 512),
          (2048, 1536, 1024)]


@pytest.mark.parametrize("t16", ["bf16", "f16"])
@pytest.mark.parametrize("tp,tq", [("T", "N"), ("N", "N"), ("T", "T"), ("N", "T")])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tile", [0, 1, 2, 3])
def test_gemm16_random(rt, h, t16, tp, tq, shape, tile):
    M, N, K = shape
    if max(shape) > 1024 and (tp, tq) != ("T", "N"):
        pytest.skip("large shapes only in the layout the library's 16-bit copies use")
    say("gemm16", t16, tp, tq, shape, tile)
    g = synth.rng(synth.W_TEST, 7300, M, N, K)
    P, Q, C = _operands(M, N, K, tp, tq, g, "rand", t16)
    td = torch.bfloat16 if t16 == "bf16" else torch.float16
    h.set_option(rt.OPT_GEMM16_TILE, tile)
    opP = P.T if tp == "T" else P
    opQ = Q.T if tq == "T" else Q
    for beta, s in ((0.0, -0.75), (1.5, 2.0)):
        Pd, Qd, Cd = _dev(rt, P, td), _dev(rt, Q, td), _dev(rt, C, torch.float32)
        rt.gemm_update(h, tp, tq, s, Pd, Qd, beta, Cd)
        torch.cuda.synchronize()
        got = rt.to_host(Cd).astype(np.float64)
        want = beta * C + s * (opP @ opQ)
        bound = np.abs(beta * C) + abs(s) * (np.abs(opP) @ np.abs(opQ))
        err = np.abs(got - want)
        lim = 2 * (K + 2) * 2.0 ** -24 * bound + 1e-30
        assert np.all(err <= lim), (t16, tp, tq, shape, tile, beta, float(np.max(err / lim)))


@pytest.mark.parametrize("t16", ["bf16", "f16"])
@pytest.mark.parametrize("shape", [(256, 256, 64), (777, 515, 131), (1024, 768, 512)])
def test_gemm16_tiles_exact_integers(rt, h, t16, shape):
    """Exact inputs: both tile families give the exact result, bit for bit."""
    M, N, K = shape
    say("gemm16 exact", t16, shape)
    g = synth.rng(synth.W_TEST, 7301, M, N, K)
    P, Q, C = _operands(M, N, K, "T", "N", g, "int", t16)
    td = torch.bfloat16 if t16 == "bf16" else torch.float16
    want = 1.0 * C - 2.0 * (P.T @ Q)
    outs = []
    for tile in (1, 2):
        h.set_option(rt.OPT_GEMM16_TILE, tile)
        Cd = _dev(rt, C, torch.float32)
        rt.gemm_update(h, "T", "N", -2.0, _dev(rt, P, td), _dev(rt, Q, td), 1.0, Cd)
        torch.cuda.synchronize()
        outs.append(rt.to_host(Cd).astype(np.float64))
    assert np.array_equal(outs[0], want)
    assert np.array_equal(outs[1], want)


@pytest.mark.parametrize("t16", ["bf16", "f16"])
@pytest.mark.parametrize("shape", [(256, 256, 32), (512, 768, 96), (1024, 1024, 1024), (768, 512, 4000)])
def test_gemm16_direct_lds_matches_register_staged(rt, h, t16, shape):
    """Full 256x256 tiles with both operands 16-bit and K a multiple of 32 go
    through the direct-to-LDS pipeline (OPT_GEMM16_TILE 2); 3 keeps the
    register-staged loads.  Same MFMA sequence per accumulator, so the results
    agree bit for bit (and meet the bound)."""
    M, N, K = shape
    say("gemm16 direct-to-LDS vs register-staged", t16, shape)
    g = synth.rng(synth.W_TEST, 7301, M, N, K)
    P, Q, C = _operands(M, N, K, "T", "N", g, "rand", t16)
    td = torch.bfloat16 if t16 == "bf16" else torch.float16
    out = []
    for tile in (2, 3):
        h.set_option(rt.OPT_GEMM16_TILE, tile)
        Pd, Qd, Cd = _dev(rt, P, td), _dev(rt, Q, td), _dev(rt, C, torch.float32)
        rt.gemm_update(h, "T", "N", 0.5, Pd, Qd, 1.25, Cd)
        torch.cuda.synchronize()
        out.append(rt.to_host(Cd).astype(np.float64))
    h.set_option(rt.OPT_GEMM16_TILE, 0)
    assert np.array_equal(out[0], out[1])
    want = 1.25 * C + 0.5 * (P.T @ Q)
    bound = 2 * (K + 2) * 2.0 ** -24 * (1.25 * np.abs(C) + 0.5 * (np.abs(P.T) @ np.abs(Q)))
    assert np.all(np.abs(out[0] - want) <= bound)

