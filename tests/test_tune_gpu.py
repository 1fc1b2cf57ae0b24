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
    assert [r["leaf"] in (32, 64) for r in rules["batched"] if r["dtype"] == dt] == [True]
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


def test_tune_batched_leaf_used(rt, orc, tmp_path):
    """A batch run under tuned rules (the batched rule set to each leaf in
    turn) gives results the oracle accepts."""
    g = synth.rng(synth.W_TEST, 3001)
    shapes = [(int(m), int(n)) for m, n in zip(synth.loguniform_int(g, 16, 300, 12), g.integers(1, 100, 12))]
    As = [synth.tri(m, "L", g, "stress") for m, n in shapes]
    Bs = [synth.dense(m, n, g) for m, n in shapes]
    for leaf in (32, 64):
        db = tmp_path / f"b{leaf}.json"
        db.write_text(json.dumps({"arch": "gfx950", "version": 1, "leaf": [], "gemm_tile": [],
                                  "batched": [{"dtype": "f64", "leaf": leaf}]}))
        h = rt.Handle()
        h.load_tuning(str(db))
        say("tuned batch leaf", leaf)
        Ad = [rt.to_device(A, torch.float64) for A in As]
        Bd = [rt.to_device(B, torch.float64) for B in Bs]
        plan = rt.BatchPlan(h, [("trsm", "L", "L", "N", "N", 1.0, Ad[i], Bd[i]) for i in range(len(shapes))])
        plan.run()
        torch.cuda.synchronize()
        plan.close()
        for i in range(len(shapes)):
            e = orc.trsm_eta("L", "L", "N", "N", 1.0, As[i], Bs[i], rt.to_host(Bd[i]))
            assert e <= TOL["f64"], (leaf, shapes[i], e)
        h.close()


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_tune16_write_load(rt, orc, dt, tmp_path):
    """The 16-bit tile sweep writes 16-bit GEMM rules next to any others; a
    16-bit TRMM under them meets the FP32-accumulation bound."""
    db = str(tmp_path / f"tune_{dt}.json")
    h = rt.Handle()
    say("tune16", dt)
    h.tune(dt, max_order=1024, db_path=db)
    rules = json.load(open(db))
    tiles = [r for r in rules["gemm_tile"] if r["dtype"] == dt]
    assert tiles and all(r["tile"] in (1, 2) for r in tiles)
    h.close()
    h2 = rt.Handle()
    h2.load_tuning(db)
    g = synth.rng(synth.W_TEST, 3002)
    m, n = 1024, 512
    A = synth.round_to(synth.tri(m, "L", g, "stress"), dt)
    B = synth.round_to(synth.dense(m, n, g), dt)
    td = torch.bfloat16 if dt == "bf16" else torch.float16
    Cd = torch.zeros((n, m), dtype=torch.float32, device="cuda").t()
    rt.trmm_ex(h2, "L", "L", "N", "N", 0.5, rt.to_device(A, td), rt.to_device(B, td), Cd)
    torch.cuda.synchronize()
    e = orc.trmm_eta("L", "L", "N", "N", 0.5, A, B, rt.to_host(Cd).astype(np.float64))
    assert e <= 7 * np.sqrt(m) * 2.0 ** -24, e
    h2.close()
