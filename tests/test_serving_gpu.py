"""Serving loop: continuous batching under an HBM budget.

Every request of a mixed stream (TRSM / TRMM, FP64 / mixed precision, small
ones batched, large ones alone, factors shared between requests) must return
bitwise the result of the same request computed alone through the single-call
API, and sampled results must meet the oracle's backward-error bound."""
import numpy as np
import pytest

import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 250413821


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


@pytest.mark.parametrize("kind,m,n", [(0, 37, 19), (1, 70, 70), (2, 65, 65), (0, 1, 300)])
def test_synth_fill_matches_host_twin(rt, h, kind, m, n):
    X = torch.empty((n, m), dtype=torch.float64, device="cuda").t()
    rt.synth_fill(h, kind, SEED, 7, (1 << 40) + 5, X, param=float(m))
    torch.cuda.synchronize()
    assert np.array_equal(rt.to_host(X), synth.philox_matrix(kind, SEED, 7, (1 << 40) + 5, m, n, float(m)))


def _stream(count, g, m_hi=2048, n_hi=256, mixed_frac=0.15, n_factors=60):
    """Requests with factors shared between several requests."""
    fac = []
    for f in range(n_factors):
        ka = int(synth.loguniform_int(g, 32, m_hi, 1)[0])
        fac.append((1000 + f, ka, "L" if g.random() < 0.5 else "U"))
    reqs = []
    for i in range(count):
        fid, ka, uplo = fac[int(g.integers(0, n_factors))]
        op = "trsm" if g.random() < 0.8 else "trmm"
        n = int(synth.loguniform_int(g, 1, n_hi, 1)[0])
        prec = 0
        if op == "trsm" and g.random() < mixed_frac:
            prec = 1 if g.random() < 0.5 else 2
        trans = "N" if g.random() < 0.5 else "T"
        reqs.append(dict(op=op, side="L", uplo=uplo, trans=trans, diag="N", m=ka, n=n, alpha=1.0, precision=prec,
                         factor_id=fid, rhs_id=50000 + i))
    return reqs


def _alone(rt, h, r):
    ka = r["m"]
    A = torch.empty((ka, ka), dtype=torch.float64, device="cuda").t()
    rt.synth_fill(h, 1 if r["uplo"] == "L" else 2, SEED, 1, r["factor_id"], A, param=float(ka))
    B = torch.empty((r["n"], r["m"]), dtype=torch.float64, device="cuda").t()
    rt.synth_fill(h, 0, SEED, 2, r["rhs_id"], B)
    if r["precision"] == 0:
        (rt.trsm if r["op"] == "trsm" else rt.trmm)(h, "L", r["uplo"], r["trans"], "N", r["alpha"], A, B)
    else:
        rt.trsm_mixed(h, "L", r["uplo"], r["trans"], "N", r["alpha"], A, B, gemm="bf16" if r["precision"] == 1 else "f32",
                      tol=1e-12, max_iter=30)
    torch.cuda.synchronize()
    return rt.to_host(B)


def _run_stream(rt, reqs, rate, **cfg):
    srv = rt.Server(**cfg)
    t0 = srv.now() + 0.05
    g = synth.rng(synth.W_SERVE, 99)
    arrivals = t0 + np.cumsum(g.exponential(1.0 / rate, len(reqs)))
    results = {}
    for r, ta in zip(reqs, arrivals):
        res = np.zeros((r["m"], r["n"]), order="F")
        tk = srv.submit(result=res, t_arrival=float(ta), **r)
        results[tk] = (r, res)
    srv.drain()
    comps = srv.poll(len(reqs) + 10)
    stats = srv.stats()
    srv.close()
    return results, comps, stats


def test_serving_alone_vs_mix(rt, h, orc):
    g = synth.rng(synth.W_SERVE, 1)
    reqs = _stream(400, g)
    say("serving mix", len(reqs))
    results, comps, stats = _run_stream(rt, reqs, rate=4000.0, slots=4, max_batch=64, small_max=1024)
    assert len(comps) == len(reqs)
    assert all(c["status"] == 0 for c in comps), [c for c in comps if c["status"] != 0][:3]
    assert stats["batched_launches"] > 0 and stats["batched_requests"] > stats["batched_launches"]
    assert stats["factor_hits"] > 0
    # without refine_requeue a refined solve runs to the end in one turn
    assert stats["refine_turns"] == sum(1 for r, _ in results.values() if r["precision"])
    for c in comps:
        assert c["t_done"] >= c["t_start"] >= c["t_arrival"] - 1e-6
    for tk, (r, res) in results.items():
        assert np.array_equal(res, _alone(rt, h, r)), r
    # sampled results against the oracle on the host twin of the inputs
    for tk in list(results)[::40]:
        r, res = results[tk]
        ka = r["m"]
        A = synth.philox_matrix(1 if r["uplo"] == "L" else 2, SEED, 1, r["factor_id"], ka, ka, float(ka))
        B = synth.philox_matrix(0, SEED, 2, r["rhs_id"], r["m"], r["n"])
        if r["op"] == "trsm":
            e = orc.trsm_eta("L", r["uplo"], r["trans"], "N", 1.0, A, B, res)
            assert e <= (1e-12 if r["precision"] else 1e-13), (r, e)
        else:
            assert orc.trmm_eta("L", r["uplo"], r["trans"], "N", 1.0, A, B, res) <= 1e-13


@pytest.mark.parametrize("slots", [1, 3])
def test_serving_refined_requeued_per_correction(rt, h, orc, slots):
    """With refine_requeue, refined (mixed-precision) solves run one
    correction per turn and re-enter the queue between turns: each refined
    request takes as many turns as it makes corrections (the first also sets
    up its residual); with one slot and FP64 requests arriving throughout,
    FP64 work completes between the corrections of a refined request; with
    several, a solve's turns may run on different slots.  Every result is
    still bitwise the result of the same request alone."""
    g = synth.rng(synth.W_SERVE, 3)
    fac = [(3000 + f, int(synth.loguniform_int(g, 256, 1536, 1)[0]), "L" if f % 2 else "U") for f in range(12)]
    reqs = []
    for i in range(60):
        fid, ka, uplo = fac[i % 12]
        prec = (1 if i % 6 == 0 else 2) if i % 3 == 0 else 0
        reqs.append(dict(op="trsm", side="L", uplo=uplo, trans="N", diag="N", m=ka, n=int(g.integers(1, 96)),
                         alpha=1.0, precision=prec, factor_id=fid, rhs_id=70000 + i))
    say("serving refined re-queue", len(reqs), "slots", slots)
    results, comps, stats = _run_stream(rt, reqs, rate=3000.0, slots=slots, max_batch=8, small_max=128,
                                        refine_requeue=True)
    assert len(comps) == len(reqs)
    assert all(c["status"] == 0 for c in comps), [c for c in comps if c["status"] != 0][:3]
    by_ticket = {c["ticket"]: c for c in comps}
    refined = [(tk, r) for tk, (r, _) in results.items() if r["precision"]]
    assert stats["refine_turns"] == sum(by_ticket[tk]["iters"] for tk, _ in refined)
    assert all(by_ticket[tk]["iters"] >= 1 for tk, _ in refined)
    # some FP64 request started after a refined request's first turn and
    # completed before its last (the slot ran it between two corrections)
    interleaved = any(by_ticket[tk]["t_start"] < c["t_start"] and c["t_done"] < by_ticket[tk]["t_done"]
                      for tk, r in refined if by_ticket[tk]["iters"] >= 2
                      for c in comps if c["iters"] == 0)
    assert interleaved or slots > 1
    for tk, (r, res) in results.items():
        assert np.array_equal(res, _alone(rt, h, r)), r


@pytest.mark.parametrize("slots", [1, 3])
def test_serving_mixed_batch(rt, h, orc, slots):
    """With mixed_batch, small refined solves with FP32 updates run in lockstep
    batches when another such request is waiting (one batched FP32 solve and
    one batched FP64 residual product per round of corrections), else alone:
    every such request converges (eta <= 1e-12 against the oracle on the host
    twin of its inputs), at least one batch holds several of them, refined
    requests with BF16 updates still run alone, and FP64 results stay bitwise
    the alone results."""
    g = synth.rng(synth.W_SERVE, 4)
    fac = [(5000 + f, int(synth.loguniform_int(g, 16, 600, 1)[0]), "L" if f % 2 else "U") for f in range(10)]
    reqs = []
    for i in range(90):
        fid, ka, uplo = fac[int(g.integers(0, 10))]
        prec = 2 if i % 3 else (0 if i % 2 else 1)
        other = int(g.integers(1, 80))
        # refined requests with FP32 updates also on side R (factor order n)
        side = "R" if prec == 2 and i % 4 == 1 else "L"
        m, n = (ka, other) if side == "L" else (other, ka)
        reqs.append(dict(op="trsm", side=side, uplo=uplo, trans="N" if g.random() < 0.5 else "T", diag="N", m=m,
                         n=n, alpha=1.0 if i % 5 else -0.5, precision=prec, factor_id=fid, rhs_id=90000 + i))
    say("serving mixed batch", len(reqs), "slots", slots)
    results, comps, stats = _run_stream(rt, reqs, rate=20000.0, slots=slots, max_batch=16, small_max=1024,
                                        mixed_batch=True)
    assert len(comps) == len(reqs)
    assert all(c["status"] == 0 for c in comps), [c for c in comps if c["status"] != 0][:3]
    by_ticket = {c["ticket"]: c for c in comps}
    f32 = [tk for tk, (r, _) in results.items() if r["precision"] == 2]
    assert all(by_ticket[tk]["iters"] >= 1 for tk in f32)
    # at least one batch of several refined solves: completions sharing a start time
    starts = [by_ticket[tk]["t_start"] for tk in f32 if by_ticket[tk]["batched"]]
    assert starts and max(starts.count(t) for t in starts) >= 2
    # a request with no company waiting ran alone (one turn), as did every BF16-update one
    alone = sum(1 for tk in f32 if not by_ticket[tk]["batched"])
    assert stats["refine_turns"] == sum(1 for r, _ in results.values() if r["precision"] == 1) + alone
    for tk, (r, res) in results.items():
        if r["precision"] == 2:
            ka = r["m"] if r["side"] == "L" else r["n"]
            A = synth.philox_matrix(1 if r["uplo"] == "L" else 2, SEED, 1, r["factor_id"], ka, ka, float(ka))
            B = synth.philox_matrix(0, SEED, 2, r["rhs_id"], r["m"], r["n"])
            e = orc.trsm_eta(r["side"], r["uplo"], r["trans"], "N", r["alpha"], A, B, res)
            assert e <= 1e-12, (r, e)
        else:
            assert np.array_equal(res, _alone(rt, h, r)), r


def test_serving_small_budget(rt, h):
    """A 48 MB budget against about 150 MB of distinct factors (up to 19 MB
    each): factors are evicted and requests wait for memory; every result is
    still the alone result."""
    g = synth.rng(synth.W_SERVE, 2)
    reqs = _stream(150, g, m_hi=1536, n_hi=64, mixed_frac=0.0, n_factors=60)
    say("serving budget", len(reqs))
    results, comps, stats = _run_stream(rt, reqs, rate=2000.0, slots=3, hbm_budget=48 << 20, max_batch=16,
                                        small_max=512)
    assert all(c["status"] == 0 for c in comps)
    assert stats["evictions"] > 0
    assert stats["hbm_peak"] <= 48 << 20
    for tk, (r, res) in results.items():
        assert np.array_equal(res, _alone(rt, h, r)), r


@pytest.mark.timeout(60)
def test_serving_rejects(rt):
    srv = rt.Server(slots=1)
    with pytest.raises(rt.RtriError):
        srv.submit(op="trsm", side="L", uplo="X", m=4, n=4)
    with pytest.raises(rt.RtriError):
        srv.submit(op="trmm", m=8, n=2, precision=rt.PREC_MIXED_BF16)
    t = srv.now()
    srv.submit(op="trsm", m=64, n=2, factor_id=7, rhs_id=1, t_arrival=t)
    srv.drain()
    # the same factor id with another order is inconsistent
    srv.submit(op="trsm", m=65, n=2, factor_id=7, rhs_id=2, t_arrival=srv.now())
    srv.drain()
    comps = srv.poll()
    srv.close()
    assert sorted(c["status"] for c in comps) == [0, rt.ERR_INVALID]


def test_serving_large_mix_alone_equal(rt, h):
    """The bench's request mix at reduced orders: TRSM 80 % / TRMM 20 %, half of
    the TRSMs refined from BF16, orders log-uniform up to 3072, right-hand
    sides up to 512, factors shared; every request must succeed and equal its
    alone result bit for bit."""
    g = synth.rng(synth.W_SERVE, 3)
    reqs = _stream(240, g, m_hi=3072, n_hi=512, mixed_frac=0.5, n_factors=40)
    for r in reqs:
        if r["precision"] == 2:
            r["precision"] = 1
    say("serving large mix", len(reqs))
    results, comps, stats = _run_stream(rt, reqs, rate=3000.0, slots=4, max_batch=64, small_max=1024)
    bad = [(c["status"], c["iters"], c["eta"], results[c["ticket"]][0]) for c in comps if c["status"] != 0]
    assert not bad, bad[:4]
    diff = []
    for tk, (r, res) in results.items():
        if not np.array_equal(res, _alone(rt, h, r)):
            diff.append(r)
    assert not diff, (len(diff), diff[:4])
