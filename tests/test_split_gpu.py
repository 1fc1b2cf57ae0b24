"""Updates split along K (narrow panels: fewer 64x64 tiles than CUs and
K >= 1024) against the oracle, and the TRMM whose concurrent updates each use
their own stream's partial-product region: both leaf schedules bit for bit."""
import numpy as np
import pytest

import synth
from gpu_util import TOL, eta, rounded, run_op, say

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
    return synth.rng(synth.W_TEST, 3000, *k)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("side,uplo,trans", [("L", "L", "N"), ("L", "U", "T"), ("R", "L", "N")])
def test_split_narrow_parity(rt, h, orc, dt, op, side, uplo, trans):
    ka, other = 4133, 70   # ragged: the split slices and the tiles both end short
    m, n = (ka, other) if side == "L" else (other, ka)
    say("split", op, dt, side, uplo, trans, m, n)
    g = G(1, ka)
    A = rounded(synth.tri(ka, uplo, g, "stress"), dt)
    B = rounded(synth.dense(m, n, g), dt)
    X = run_op(rt, h, op, side, uplo, trans, "N", -0.5, A, B, dt)
    e = eta(orc, op, side, uplo, trans, "N", -0.5, A, B, X)
    assert e <= TOL[dt], (op, dt, side, uplo, trans, e)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_split_trmm_concurrent_schedules(rt, h, orc, dt):
    """m = 8192, 128 vectors: one launch per leaf, whose long updates split K,
    against every leaf in one launch followed by one grouped launch of all
    updates (no split): the same sums in another order, so both must meet the
    oracle's bound and agree to within it."""
    m, n = 8192, 128
    say("split trmm schedules", dt)
    g = G(2, m)
    A = rounded(synth.tri(m, "L", g, "base"), dt)
    B = rounded(synth.dense(m, n, g), dt)
    h.set_option(rt.OPT_LEAF_F64 if dt == "f64" else rt.OPT_LEAF_F32, 256)
    out = []
    for mode in (1, 2):
        h.set_option(rt.OPT_TRMM_LEAVES, mode)
        out.append(run_op(rt, h, "trmm", "L", "L", "N", "N", 1.0, A, B, dt))
    h.set_option(rt.OPT_TRMM_LEAVES, 0)
    idx = np.sort(G(3).choice(n, 8, replace=False))
    for X in out:
        e = orc.trmm_eta("L", "L", "N", "N", 1.0, A, np.asfortranarray(B[:, idx]), np.asfortranarray(X[:, idx]))
        assert e <= TOL[dt], e
    scale = np.max(np.abs(out[0]))
    assert np.max(np.abs(out[0] - out[1])) <= 64 * TOL[dt] * scale
