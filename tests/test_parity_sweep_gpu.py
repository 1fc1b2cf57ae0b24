"""The square sweep at its large orders against the CPU oracle, in the launch
configuration the benchmark times (the shipped tuning database loaded).

* Order 4096: every side / uplo / trans combination with both diagonal types,
  FP64 and FP32, TRSM and TRMM.
* Order 8192: FP64 and FP32, TRSM and TRMM, on the sweep generator (diagonal
  m + U(0,1)) and on the stress generator (diagonal sqrt(m)(1 + U(0,1)), so the
  GEMM updates are not damped by a nearly diagonal factor).
* Order 16384: FP64 and FP32, TRSM and TRMM, sweep generator.

Columns (side L) or rows (side R) of the result are independent, so each
result is checked on a seeded sample of them: the oracle's compensated
backward error within the tolerance (FP64 1e-13, FP32 5e-5), and the
difference from the oracle's own result.  Every test prints its case first."""
import zlib

import numpy as np
import pytest

import synth
from dense_ref import VARIANTS_NT
from gpu_util import TOL, eta, oracle_op, rounded, run_op, say

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
    hd.load_tuning(rt.TUNING_DB)
    yield hd
    hd.close()


def _sampled(rt, h, orc, op, side, uplo, trans, diag, m, dt, kind, nsamp):
    n = m
    g = synth.rng(synth.W_SWEEP, m, zlib.crc32(f"{side}{uplo}{trans}{diag}{dt}{kind}".encode()) & 0xFFFF)
    A = rounded(synth.tri(m, uplo, g, kind), dt)
    B = rounded(synth.dense(m, n, g), dt)
    X = run_op(rt, h, op, side, uplo, trans, diag, 1.0, A, B, dt)
    idx = np.sort(synth.rng(synth.W_SWEEP, m, 78).choice(m, nsamp, replace=False))
    if side == "L":
        Bs, Xs = np.asfortranarray(B[:, idx]), np.asfortranarray(X[:, idx])
    else:
        Bs, Xs = np.asfortranarray(B[idx, :]), np.asfortranarray(X[idx, :])
    e = eta(orc, op, side, uplo, trans, diag, 1.0, A, Bs, Xs)
    Xo = oracle_op(orc, op, side, uplo, trans, diag, 1.0, A, Bs)
    return e, float(np.max(np.abs(Xs - Xo)) / np.max(np.abs(Xo)))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("side,uplo,trans", VARIANTS_NT)
def test_all_variants_4096(rt, h, orc, dt, op, diag, side, uplo, trans):
    m = 4096
    kind = "unit" if diag == "U" else "stress"
    say("sweep 4096", dt, op, side, uplo, trans, diag, "leaf", h.leaf(dt, op, m, m))
    e, fwd = _sampled(rt, h, orc, op, side, uplo, trans, diag, m, dt, kind, 12)
    say("  eta", e, "fwd", fwd)
    assert e <= TOL[dt], (dt, op, side, uplo, trans, diag, e)
    assert fwd <= 100 * TOL[dt], fwd


@pytest.mark.parametrize("kind", ["base", "stress"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
def test_sweep_8192(rt, h, orc, kind, dt, op):
    m = 8192
    say("sweep 8192", kind, dt, op, "leaf", h.leaf(dt, op, m, m))
    e, fwd = _sampled(rt, h, orc, op, "L", "L", "N", "N", m, dt, kind, 8)
    say("  eta", e, "fwd", fwd)
    assert e <= TOL[dt], (kind, dt, op, e)
    assert fwd <= 100 * TOL[dt], fwd


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
def test_sweep_16384(rt, h, orc, dt, op):
    m = 16384
    say("sweep 16384", dt, op, "leaf", h.leaf(dt, op, m, m))
    e, fwd = _sampled(rt, h, orc, op, "L", "L", "N", "N", m, dt, "base", 6)
    say("  eta", e, "fwd", fwd)
    assert e <= TOL[dt], (dt, op, e)
    assert fwd <= 100 * TOL[dt], fwd
