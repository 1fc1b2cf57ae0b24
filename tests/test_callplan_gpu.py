"""Call plans (rtri_call_plan_*): one TRSM / TRMM captured in a HIP graph and
replayed.  Every replay must equal the plain call on the same inputs bit for
bit (a TRMM: the plain call with one launch per leaf, the schedule a plan
captures), and meet the oracle's bound.  Replays alternate with unrelated
eager work and other library calls on the same handle, and each replay is
checked, not only the first."""
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


CASES = [("trsm", "f64", "L", "L", "N", "N", 600, 130), ("trsm", "f32", "L", "U", "T", "U", 4133, 256),
         ("trsm", "f64", "R", "U", "N", "N", 90, 700), ("trmm", "f64", "L", "L", "T", "N", 1000, 257),
         ("trmm", "f32", "L", "L", "N", "N", 4096, 256), ("trmm", "f64", "R", "L", "N", "U", 77, 300),
         ("trsm", "f64", "L", "L", "N", "N", 16, 5)]


@pytest.mark.parametrize("case", CASES)
def test_call_plan_replays_equal_plain_call(rt, orc, case):
    op, dt, side, uplo, trans, diag, m, n = case
    say("call plan", case)
    g = synth.rng(synth.W_TEST, 7700, m, n)
    ka = m if side == "L" else n
    A = rounded(synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress"), dt)
    B = rounded(synth.dense(m, n, g), dt)
    td = torch_dtype(dt)
    h = rt.Handle()
    try:
        h.set_option(rt.OPT_TRMM_LEAVES, 1)
        Ad = rt.to_device(A, td)
        B0 = rt.to_device(B, td)
        Bp = B0.clone()
        plan = rt.CallPlan(h, op, side, uplo, trans, diag, -0.5, Ad, Bp)
        Be = B0.clone()
        (rt.trsm if op == "trsm" else rt.trmm)(h, side, uplo, trans, diag, -0.5, Ad, Be)
        torch.cuda.synchronize()
        want = rt.to_host(Be)
        other = rt.to_device(synth.dense(64, 64, g), td)
        Ao = rt.to_device(rounded(synth.tri(64, "L", g, "base"), dt), td)
        for rep in range(3):
            Bp.copy_(B0)
            plan.run()
            # unrelated eager work and another library call between replays
            (other * 2.0).sum()
            rt.trsm(h, "L", "L", "N", "N", 1.0, Ao, other)
            torch.cuda.synchronize()
            got = rt.to_host(Bp)
            assert np.array_equal(got, want), (rep, float(np.max(np.abs(got - want))))
        e = eta(orc, op, side, uplo, trans, diag, -0.5, A, B, got.astype(np.float64))
        assert e <= TOL[dt], e
        plan.close()
    finally:
        h.close()


def test_call_plan_alpha_zero_and_empty(rt):
    h = rt.Handle()
    try:
        say("call plan alpha=0 / empty")
        A = torch.full((32, 32), float("nan"), dtype=torch.float64, device="cuda").t()
        B = torch.ones((16, 32), dtype=torch.float64, device="cuda").t()
        p = rt.CallPlan(h, "trsm", "L", "L", "N", "N", 0.0, A, B)
        p.run()
        torch.cuda.synchronize()
        assert torch.count_nonzero(B).item() == 0
        p.close()
        E = torch.zeros((32, 0), dtype=torch.float64, device="cuda")
        p = rt.CallPlan(h, "trmm", "L", "L", "N", "N", 1.0, A, E)
        p.run()
        torch.cuda.synchronize()
        p.close()
    finally:
        h.close()
