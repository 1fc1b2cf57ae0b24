"""The FP64 / FP32 GEMM update on its own, across tile shapes and K.

FP32 64x64 tiles stage two k-steps (32 values of K) per LDS buffer; the
128x128 tiles (4 or 8 wavefronts) stage one.  All issue, for every element of
C, the same MFMA sequence over K (k-steps of 16 in order, within a step lane
group g taking k = 4g + t in MFMA number t), so the tile shapes must agree bit
for bit for every K: ragged K included, where the last stage holds one k-step,
or part of one, and the second half of a stage is skipped.  FP64 tiles stage
one k-step in every shape (the same check as a control).

Bound against the exact result (FP64 reference of the rounded inputs):
|got - exact| <= 2 (K + 2) u (|beta C| + |s| |op(P)| |op(Q)|) elementwise,
u the unit roundoff of the type."""
import numpy as np
import pytest

import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}


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


def _operands(M, N, K, tp, tq, g, dt):
    P = synth.dense(K, M, g) if tp == "T" else synth.dense(M, K, g)
    Q = synth.dense(N, K, g) if tq == "T" else synth.dense(K, N, g)
    C = synth.dense(M, N, g)
    if dt == "f32":
        P, Q, C = (x.astype(np.float32).astype(np.float64) for x in (P, Q, C))
    return np.asfortranarray(P), np.asfortranarray(Q), np.asfortranarray(C)


def _run(rt, h, tile, tp, tq, s, P, Q, beta, C, dt):
    tdt = torch.float64 if dt == "f64" else torch.float32
    h.set_option(rt.OPT_GEMM_TILE, tile)
    Cd = rt.to_device(C, tdt)
    rt.gemm_update(h, tp, tq, s, rt.to_device(P, tdt), rt.to_device(Q, tdt), beta, Cd)
    torch.cuda.synchronize()
    return rt.to_host(Cd).astype(np.float64)


# K: below one k-step, exactly one, one and a bit, one stage of two, a stage
# and a part, several stages with a ragged end
KS = [1, 3, 15, 16, 17, 31, 32, 33, 47, 48, 63, 65, 200]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("tp,tq", [("N", "N"), ("T", "N"), ("N", "T")])
@pytest.mark.parametrize("beta", [0.0, 1.25])
def test_tile_shapes_agree_over_k(rt, h, dt, tp, tq, beta):
    M, N = 150, 70   # ragged in both directions for both tile shapes
    s = -0.75
    for K in KS:
        say("gemm stages", dt, tp, tq, beta, "K", K)
        g = synth.rng(synth.W_TEST, 3100, K, ord(tp) * 3 + ord(tq), int(beta * 4))
        P, Q, C = _operands(M, N, K, tp, tq, g, dt)
        c64 = _run(rt, h, 2, tp, tq, s, P, Q, beta, C, dt)    # 64x64 tiles
        c128 = _run(rt, h, 1, tp, tq, s, P, Q, beta, C, dt)   # 128x128 tiles, 4 wavefronts
        c8w = _run(rt, h, 3, tp, tq, s, P, Q, beta, C, dt)    # 128x128 tiles, 8 wavefronts
        assert np.array_equal(c64, c128), (dt, tp, tq, beta, K, float(np.max(np.abs(c64 - c128))))
        assert np.array_equal(c64, c8w), (dt, tp, tq, beta, K, float(np.max(np.abs(c64 - c8w))))
        op_p = P.T if tp == "T" else P
        op_q = Q.T if tq == "T" else Q
        exact = beta * C + s * (op_p @ op_q)
        bound = 2 * (K + 2) * U[dt] * (abs(beta) * np.abs(C) + abs(s) * (np.abs(op_p) @ np.abs(op_q)))
        err = np.abs(c64 - exact)
        assert np.all(err <= bound), (dt, tp, tq, beta, K, float(np.max(err / np.maximum(bound, 1e-300))))
