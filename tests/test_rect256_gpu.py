"""The paper's narrow workload (its rectangular case, B m x 256, FP32) against
the CPU oracle, in the launch configuration the benchmark times: device-drawn
inputs (Philox fill), the shipped tuning rules, side L / lower / no transpose /
non-unit, m = 1024 ... 16384.  Narrow panels are where the GEMM updates are
short of tiles and split K, and where the TRMM runs all its leaves in one
launch with concurrent updates; every variant is also checked at m = 4096.
Results are checked on sampled columns: the oracle's compensated backward
error within 5e-5 (FP32) or 1e-13 (FP64)."""
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


@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("m", [1024, 2048, 4096, 8192, 16384])
def test_rect256_bench_config(rt, h, orc, op, m):
    n = 256
    say("rect256", op, m, "leaf", h.leaf("f32", op, m, n))
    Ad = torch.empty((m, m), dtype=torch.float32, device="cuda").t()
    Bd = torch.empty((n, m), dtype=torch.float32, device="cuda").t()
    rt.synth_fill(h, 1, synth.SEED, synth.W_SWEEP, 3, Ad, param=float(m))
    rt.synth_fill(h, 0, synth.SEED, synth.W_SWEEP, 4, Bd)
    idx = np.sort(synth.rng(synth.W_SWEEP, 256, m).choice(n, 16, replace=False))
    tidx = torch.as_tensor(idx, device="cuda")
    Bs = np.asfortranarray(Bd[:, tidx].cpu().numpy().astype(np.float64))
    (rt.trsm if op == "trsm" else rt.trmm)(h, "L", "L", "N", "N", 1.0, Ad, Bd)
    torch.cuda.synchronize()
    Xs = np.asfortranarray(Bd[:, tidx].cpu().numpy().astype(np.float64))
    A = rt.to_host(Ad).astype(np.float64)
    del Ad, Bd
    e = eta(orc, op, "L", "L", "N", "N", 1.0, A, Bs, Xs)
    Xo = oracle_op(orc, op, "L", "L", "N", "N", 1.0, A, Bs)
    fwd = float(np.max(np.abs(Xs - Xo)) / np.max(np.abs(Xo)))
    say("  eta", e, "fwd", fwd)
    assert e <= TOL["f32"], (op, m, e)
    assert fwd <= 100 * TOL["f32"]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("side,uplo,trans", VARIANTS_NT)
def test_rect256_variants_4096(rt, h, orc, dt, op, diag, side, uplo, trans):
    """Every variant on the narrow shape: the order-4096 factor against 256
    vectors (columns of B for side L, rows for side R)."""
    ka, nv = 4096, 256
    m, n = (ka, nv) if side == "L" else (nv, ka)
    say("rect256 variant", dt, op, side, uplo, trans, diag)
    g = synth.rng(synth.W_TEST, 6000, zlib.crc32(f"{dt}{op}{side}{uplo}{trans}{diag}".encode()) & 0xFFFF)
    A = rounded(synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress"), dt)
    B = rounded(synth.dense(m, n, g), dt)
    X = run_op(rt, h, op, side, uplo, trans, diag, 0.5, A, B, dt)
    idx = np.sort(g.choice(nv, 12, replace=False))
    if side == "L":
        Bs, Xs = np.asfortranarray(B[:, idx]), np.asfortranarray(X[:, idx])
    else:
        Bs, Xs = np.asfortranarray(B[idx, :]), np.asfortranarray(X[idx, :])
    e = eta(orc, op, side, uplo, trans, diag, 0.5, A, Bs, Xs)
    assert e <= TOL[dt], (dt, op, side, uplo, trans, diag, e)


@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("m,n,uplo,trans", [(5000, 256, "L", "N"), (5000, 256, "U", "T"), (9001, 200, "L", "T"),
                                            (9001, 200, "U", "N")])
def test_rect256_ragged(rt, h, orc, op, m, n, uplo, trans):
    """Narrow panels whose order is not a multiple of the tiles or leaves, with
    200 or 256 vectors: the grouped TRMM launch with edge tiles (tile order by
    CU rounds, two k-steps per LDS stage, a last stage ending inside K) and the
    TRSM's split-K updates, FP32, against the oracle on sampled columns."""
    say("rect256 ragged", op, m, n, uplo, trans, "leaf", h.leaf("f32", op, m, n))
    g = synth.rng(synth.W_TEST, 6100, m, n, ord(uplo) + 2 * ord(trans), 1 if op == "trsm" else 2)
    A = rounded(synth.tri(m, uplo, g, "base"), "f32")
    B = rounded(synth.dense(m, n, g), "f32")
    X = run_op(rt, h, op, "L", uplo, trans, "N", -1.25, A, B, "f32")
    idx = np.sort(g.choice(n, 12, replace=False))
    Bs, Xs = np.asfortranarray(B[:, idx]), np.asfortranarray(X[:, idx])
    e = eta(orc, op, "L", uplo, trans, "N", -1.25, A, Bs, Xs)
    assert e <= TOL["f32"], (op, m, n, uplo, trans, e)
