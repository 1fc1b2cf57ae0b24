"""Batched persistent launches (many independent problems in one launch).

Every problem of a batch must give bitwise the result of the single-call path
on the same inputs (same recursion, same per-element arithmetic), and that
result must meet the oracle's backward-error bound.  Graph replays must all
agree with the eager launch."""
import ctypes

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


def _problem(shape, kind, g, dt, side="L", trans="N", diag="N"):
    m, n, uplo = shape
    ka = m if side == "L" else n
    A = rounded(synth.tri(ka, uplo, g, "unit" if diag == "U" else kind, fill=np.nan), dt)
    B = rounded(synth.dense(m, n, g), dt)
    return A, B


def _single(rt, h, op, side, uplo, trans, diag, alpha, A, B, dt):
    td = torch_dtype(dt)
    Ad, Bd = rt.to_device(A, td), rt.to_device(B, td)
    (rt.trsm if op == "trsm" else rt.trmm)(h, side, uplo, trans, diag, alpha, Ad, Bd)
    torch.cuda.synchronize()
    return rt.to_host(Bd).astype(np.float64)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_mixed_variant_batch(rt, h, orc, dt):
    g = synth.rng(synth.W_TEST, 3000, 1)
    td = torch_dtype(dt)
    cases = []
    for i, (side, uplo, trans, diag) in enumerate([(s, u, t, d) for s in "LR" for u in "LU" for t in "NT" for d in "NU"]):
        for op in ("trsm", "trmm"):
            m = int(g.integers(1, 300))
            n = int(g.integers(1, 150))
            A, B = _problem((m, n, uplo), "stress", g, dt, side, trans, diag)
            alpha = float(g.choice([1.0, -0.5, 2.0]))
            cases.append((op, side, uplo, trans, diag, alpha, A, B))
    dev = [(op, s, u, t, d, a, rt.to_device(A, td), rt.to_device(B, td)) for (op, s, u, t, d, a, A, B) in cases]
    say("batch variants", dt, len(cases))
    rt.batched(h, dev)
    for (op, s, u, t, d, a, A, B), (_, _, _, _, _, _, Ad, Bd) in zip(cases, dev):
        X = rt.to_host(Bd).astype(np.float64)
        ref = _single(rt, h, op, s, u, t, d, a, A, B, dt)
        assert np.array_equal(X, ref), (op, s, u, t, d, A.shape, B.shape)
        assert eta(orc, op, s, u, t, d, a, A, B, X) <= TOL[dt]


def test_batch_edge_entries(rt, h):
    A = torch.eye(8, dtype=torch.float64, device="cuda").t()
    B = torch.ones((8, 5), dtype=torch.float64, device="cuda").t().contiguous().t()
    E = torch.ones((0, 5), dtype=torch.float64, device="cuda")
    rt.batched(h, [("trsm", "L", "L", "N", "N", 0.0, A, B)])
    torch.cuda.synchronize()
    assert torch.count_nonzero(B).item() == 0
    arr, dt, n = rt.batch_entries([("trsm", "L", "L", "N", "N", 1.0, A, B)])
    arr[0].lda = 3                                     # invalid: lda < m
    bad = ctypes.c_int(-1)
    assert rt.rtri_batched(h.ptr, dt, 1, arr, ctypes.byref(bad)) == -9 and bad.value == 0


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_uneven_batch_4096(rt, h, orc, dt):
    """4096 problems, m log-uniform on [16, 1024], nrhs uniform on [1, 128],
    lower / upper 50/50, TRSM then TRMM on the results; side L, trans N, diag N."""
    td = torch_dtype(dt)
    g = synth.rng(synth.W_BATCH, 0)
    shapes = synth.batch_shapes(4096, g)
    A_host, B_host, A_dev, B_dev = [], [], [], []
    for i, sh in enumerate(shapes):
        A, B = _problem(sh, "base", g, dt)
        A_host.append(A)
        B_host.append(B)
    say("batch 4096", dt, "total A elements", sum(a.size for a in A_host))
    A_dev = [rt.to_device(A, td) for A in A_host]
    B_dev = [rt.to_device(B, td) for B in B_host]
    plan = rt.BatchPlan(h, [("trsm", "L", sh[2], "N", "N", 1.0, A_dev[i], B_dev[i]) for i, sh in enumerate(shapes)])
    assert plan.chunks() == sum((sh[1] + 63) // 64 for sh in shapes)
    plan.run()
    torch.cuda.synchronize()
    X_dev = [rt.to_host(b).astype(np.float64) for b in B_dev]
    sub = synth.rng(synth.W_BATCH, 1).choice(4096, 96, replace=False)
    for i in sub:
        uplo = shapes[i][2]
        e = orc.trsm_eta("L", uplo, "N", "N", 1.0, A_host[i], B_host[i], X_dev[i])
        assert e <= TOL[dt], (i, shapes[i], e)
        ref = _single(rt, h, "trsm", "L", uplo, "N", "N", 1.0, A_host[i], B_host[i], dt)
        assert np.array_equal(X_dev[i], ref), (i, shapes[i])
    # graph replays: restore B, replay, compare with the first (eager-equivalent) result
    for rep in range(2):
        for i in range(4096):
            B_dev[i].copy_(rt.to_device(B_host[i], td))
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        for i in sub:
            assert np.array_equal(rt.to_host(B_dev[i]).astype(np.float64), X_dev[i]), (rep, i)
    plan.close()
    # TRMM batch on the solutions: multiplies back to B (round trip)
    plan2 = rt.BatchPlan(h, [("trmm", "L", sh[2], "N", "N", 1.0, A_dev[i], B_dev[i]) for i, sh in enumerate(shapes)])
    plan2.run()
    torch.cuda.synchronize()
    for i in sub:
        Y = rt.to_host(B_dev[i]).astype(np.float64)
        e = orc.trmm_eta("L", shapes[i][2], "N", "N", 1.0, A_host[i], X_dev[i], Y)
        assert e <= TOL[dt], (i, e)
    plan2.close()
