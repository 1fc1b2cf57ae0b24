"""The tuning step on the GPU: rtri_tune sweeps leaf sizes and GEMM tiles on
synthetic problems, writes its rules as JSON, and a handle that loads them
still computes results the oracle accepts."""
import json

import numpy as np
import pytest

import synth
from gpu_util import TOL, eta, run_op, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_13821_amd as rt
    return rt


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_tune_write_load_solve(rt, orc, dt, tmp_path):
    db = str(tmp_path / f"tune_{dt}.json")
    h = rt.Handle()
    say("tune", dt)
    h.tune(dt, max_order=512, db_path=db)
    rules = json.load(open(db))
    say("  rules", json.dumps(rules)[:400])
    text = json.dumps(rules)
    assert '"leaf"' in text and '"tile"' in text
    h.close()
    h2 = rt.Handle()
    h2.load_tuning(db)
    g = synth.rng(synth.W_TEST, 3000, dt == "f64")
    for (m, n, side, uplo, trans) in [(512, 512, "L", "L", "N"), (300, 70, "L", "U", "T"), (70, 256, "R", "U", "N")]:
        ka = m if side == "L" else n
        assert h2.leaf(dt, "trsm", ka, n if side == "L" else m) in (16, 32, 64, 128, 256)
        A = synth.round_to(synth.tri(ka, uplo, g, "stress"), dt)
        B = synth.round_to(synth.dense(m, n, g), dt)
        for op in ("trsm", "trmm"):
            X = run_op(rt, h2, op, side, uplo, trans, "N", 1.0, A, B, dt)
            e = eta(orc, op, side, uplo, trans, "N", 1.0, A, B, X)
            say("  ", op, m, n, side, uplo, trans, e)
            assert e <= TOL[dt], (op, m, n, e)
    h2.close()
