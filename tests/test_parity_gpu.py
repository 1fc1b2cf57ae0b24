"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: FP64 normwise backward error <= 1e-13; FP32 <= 5e-5 (the same
margin, 7*sqrt(16384)*u, at u = 2^-24).  Exact-integer inputs must agree bit
for bit.  Every test prints its case before the GPU call."""
import zlib

import numpy as np
import pytest

import synth
from dense_ref import VARIANTS
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
    yield hd
    hd.close()


def G(*k):
    return synth.rng(synth.W_TEST, 1000, *k)


# ---- the GEMM update on its own ------------------------------------------------

GEMM_SHAPES = [(1, 1, 1), (37, 50, 19), (64, 64, 16), (128, 128, 16), (200, 300, 70), (257, 129, 513),
               (512, 384, 256)]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("tp,tq", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
@pytest.mark.parametrize("shape", GEMM_SHAPES)
@pytest.mark.parametrize("tile", [0, 1, 2, 3])
def test_gemm_update(rt, h, orc, dt, tp, tq, shape, tile):
    M, N, K = shape
    say("gemm", dt, tp, tq, shape, tile)
    g = G(1, M, N, K)
    P = rounded(synth.dense(K, M, g) if tp == "T" else synth.dense(M, K, g), dt)
    Q = rounded(synth.dense(N, K, g) if tq == "T" else synth.dense(K, N, g), dt)
    C = rounded(synth.dense(M, N, g), dt)
    opP = P.T if tp == "T" else P
    opQ = Q.T if tq == "T" else Q
    h.set_option(rt.OPT_GEMM_TILE, tile)
    from gpu_util import torch_dtype
    td = torch_dtype(dt)
    for beta in (0.0, 1.5):
        Pd, Qd, Cd = rt.to_device(P, td), rt.to_device(Q, td), rt.to_device(C, td)
        rt.gemm_update(h, tp, tq, -0.75, Pd, Qd, beta, Cd)
        torch.cuda.synchronize()
        got = rt.to_host(Cd).astype(np.float64)
        want = beta * C + (-0.75) * (opP @ opQ)
        bound = np.abs(beta * C) + 0.75 * (np.abs(opP) @ np.abs(opQ))
        u = 2.0 ** -53 if dt == "f64" else 2.0 ** -24
        assert np.all(np.abs(got - want) <= 2 * (K + 2) * u * bound + 1e-300), (dt, tp, tq, shape, beta)


# ---- all variants against the oracle ---------------------------------------------

def _inputs(side, uplo, diag, m, n, dt, g, kind=None):
    ka = m if side == "L" else n
    kind = kind or ("unit" if diag == "U" else "stress")
    A = rounded(synth.tri(ka, uplo, g, kind), dt)
    B = rounded(synth.dense(m, n, g), dt)
    return A, B


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
def test_variant_parity(rt, h, orc, dt, op, diag, side, uplo, trans):
    m, n = (200, 77) if side == "L" else (77, 200)
    say(op, dt, side, uplo, trans, diag, m, n)
    A, B = _inputs(side, uplo, diag, m, n, dt, G(2, m))
    alpha = -1.5
    X = run_op(rt, h, op, side, uplo, trans, diag, alpha, A, B, dt)
    Xo = oracle_op(orc, op, side, uplo, trans, diag, alpha, A, B)
    e = eta(orc, op, side, uplo, trans, diag, alpha, A, B, X)
    assert e <= TOL[dt], (op, dt, side, uplo, trans, diag, e)
    assert np.max(np.abs(X - Xo)) <= 50 * TOL[dt] * np.max(np.abs(Xo))


# ---- exact integers: bit-for-bit with the oracle ---------------------------------

@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("side,uplo,trans", [v for v in VARIANTS if v[2] != "C"])
def test_exact_bitwise(rt, h, orc, dt, op, diag, side, uplo, trans):
    # sizes that keep every intermediate exactly representable (see the oracle pins)
    ka = {("trsm", "f64"): 44, ("trsm", "f32"): 18, ("trmm", "f64"): 60, ("trmm", "f32"): 60}[(op, dt)]
    n = 9
    m, n = (ka, n) if side == "L" else (n, ka)
    say("exact", op, dt, side, uplo, trans, diag, m, n)
    g = G(3, ka)
    if op == "trsm":
        A = synth.exact_tri(ka, uplo, g, offdiag=(-1, 0, 1), diag=(1.0, -1.0))
    else:
        A = synth.exact_tri(ka, uplo, g, offdiag=(-2, -1, 0, 1, 2), diag=(1.0, -1.0, 2.0, -2.0))
    if diag == "U":
        A[np.diag_indices(ka)] = np.nan
    B = synth.exact_dense(m, n, g)
    h.set_option(rt.OPT_LEAF_F64 if dt == "f64" else rt.OPT_LEAF_F32, 16)
    X = run_op(rt, h, op, side, uplo, trans, diag, 2.0, A, B, dt)
    Xo = oracle_op(orc, op, side, uplo, trans, diag, 2.0, A, B)
    assert np.array_equal(X, Xo)


# ---- blocked leaves (128 / 256 rows: several wavefronts per panel) ---------------

@pytest.mark.parametrize("leaf", [128, 256])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("side,uplo,trans", [v for v in VARIANTS if v[2] != "C"])
def test_blocked_leaf_variants(rt, h, orc, leaf, dt, op, diag, side, uplo, trans):
    """Orders 600 (full blocks plus a ragged one of 88 rows) against 130
    vectors (a ragged last workgroup of 2 vectors)."""
    m, n = (600, 130) if side == "L" else (130, 600)
    say("bleaf", leaf, op, dt, side, uplo, trans, diag, m, n)
    A, B = _inputs(side, uplo, diag, m, n, dt, G(12, m))
    h.set_option(rt.OPT_LEAF_F64 if dt == "f64" else rt.OPT_LEAF_F32, leaf)
    X = run_op(rt, h, op, side, uplo, trans, diag, -1.5, A, B, dt)
    e = eta(orc, op, side, uplo, trans, diag, -1.5, A, B, X)
    assert e <= TOL[dt], (leaf, op, dt, side, uplo, trans, diag, e)


@pytest.mark.parametrize("leaf", [16, 64, 128, 256])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("side,uplo,trans", [("L", "L", "N"), ("L", "U", "T"), ("R", "L", "N")])
def test_leaf_ill_conditioned(rt, h, orc, leaf, dt, side, uplo, trans):
    """Diagonal 4.5 + U(0,1) against off-diagonal U(-1,1): cond_1 ~ 1.7e6 at
    order 1024, and 16 x 16 diagonal tiles far from the identity.  The
    matrix-core leaves apply FP64 inverses of those tiles; the backward error
    must still meet the tolerance."""
    m, n = (1024, 96) if side == "L" else (96, 1024)
    say("ill-conditioned leaf", leaf, dt, side, uplo, trans)
    g = G(15, leaf)
    A = rounded(synth.tri(1024, uplo, g, "cond", c=4.5), dt)
    B = rounded(synth.dense(m, n, g), dt)
    h.set_option(rt.OPT_LEAF_F64 if dt == "f64" else rt.OPT_LEAF_F32, leaf)
    X = run_op(rt, h, "trsm", side, uplo, trans, "N", 1.0, A, B, dt)
    e = eta(orc, "trsm", side, uplo, trans, "N", 1.0, A, B, X)
    assert e <= TOL[dt], (leaf, dt, e)


@pytest.mark.parametrize("leaf", [128, 256])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("side,uplo,trans", [("L", "L", "N"), ("L", "U", "T"), ("R", "U", "N"), ("R", "L", "T")])
def test_blocked_leaf_exact(rt, h, orc, leaf, op, side, uplo, trans):
    """One partial block with exact small integers (power-of-two diagonal, so
    the reciprocal is exact): bit for bit with the oracle."""
    ka = 44 if op == "trsm" else 60
    m, n = (ka, 70) if side == "L" else (70, ka)
    say("bleaf exact", leaf, op, side, uplo, trans)
    g = G(13, ka)
    if op == "trsm":
        A = synth.exact_tri(ka, uplo, g, offdiag=(-1, 0, 1), diag=(1.0, -1.0))
    else:
        A = synth.exact_tri(ka, uplo, g, offdiag=(-2, -1, 0, 1, 2), diag=(1.0, -1.0, 2.0, -2.0))
    B = synth.exact_dense(m, n, g)
    h.set_option(rt.OPT_LEAF_F64, leaf)
    X = run_op(rt, h, op, side, uplo, trans, "N", 2.0, A, B, "f64")
    assert np.array_equal(X, oracle_op(orc, op, side, uplo, trans, "N", 2.0, A, B))


@pytest.mark.parametrize("op", ["trsm", "trmm"])
def test_blocked_leaf_exact_full_blocks(rt, h, orc, op):
    """Exact integers over two full 128-row blocks and a ragged one: unit
    diagonal with off-diagonal entries in {-1, 0, 1} scaled so every
    intermediate stays an exact integer."""
    ka, n = 300, 65
    say("bleaf exact full", op)
    g = G(14, ka)
    A = synth.exact_tri(ka, "L", g, offdiag=(0.0, 0.0, 0.0, 1.0), diag=(1.0,))
    A[np.tril_indices(ka, -2)] = 0.0          # bidiagonal: solutions stay small integers
    B = synth.exact_dense(ka, n, g, bound=3)
    h.set_option(rt.OPT_LEAF_F64, 128)
    X = run_op(rt, h, op, "L", "L", "N", "N", 1.0, A, B, "f64")
    assert np.array_equal(X, oracle_op(orc, op, "L", "L", "N", "N", 1.0, A, B))


# ---- leaf sizes, padding, alpha, sentinels, determinism --------------------------

@pytest.mark.parametrize("dt,leaf", [("f64", 16), ("f64", 32), ("f64", 64), ("f64", 128), ("f64", 256),
                                     ("f32", 16), ("f32", 32), ("f32", 64), ("f32", 128), ("f32", 256)])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
def test_leaf_sizes(rt, h, orc, dt, leaf, op):
    m, n = 333, 130
    say("leaf", dt, leaf, op)
    A, B = _inputs("L", "U", "N", m, n, dt, G(4))
    h.set_option(rt.OPT_LEAF_F64 if dt == "f64" else rt.OPT_LEAF_F32, leaf)
    X = run_op(rt, h, op, "L", "U", "T", "N", 1.0, A, B, dt)
    assert eta(orc, op, "L", "U", "T", "N", 1.0, A, B, X) <= TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("side", "LR")
def test_leading_dimension_padding(rt, h, orc, dt, side):
    m, n = 150, 97
    say("pad", dt, side)
    A, B = _inputs(side, "L", "N", m, n, dt, G(5))
    ka = A.shape[0]
    for op in ("trsm", "trmm"):
        X = run_op(rt, h, op, side, "L", "N", "N", 0.5, A, B, dt, lda=ka + 3, ldb=m + 5)
        assert eta(orc, op, side, "L", "N", "N", 0.5, A, B, X) <= TOL[dt]


@pytest.mark.parametrize("dt,leaf", [("f64", 64), ("f64", 128), ("f64", 256), ("f32", 64), ("f32", 256)])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("m", [600, 601])
def test_vector_and_element_paths_agree(rt, h, orc, dt, leaf, op, uplo, m):
    """Side L with ldb = m (16-byte panel and C accesses where the alignment
    allows) and ldb = m + 1 (element by element, every vector misaligned):
    the same arithmetic, so the results agree bit for bit, and both pass the
    oracle's bound.  m = 600 ends in a ragged leaf of a multiple of 4 rows,
    m = 601 in one that is not."""
    n = 130
    say("vec/elem", dt, leaf, op, uplo, m)
    A, B = _inputs("L", uplo, "N", m, n, dt, G(16, m))
    h.set_option(rt.OPT_LEAF_F64 if dt == "f64" else rt.OPT_LEAF_F32, leaf)
    ld_vec = m + (-m) % 4
    X1 = run_op(rt, h, op, "L", uplo, "N", "N", 0.75, A, B, dt, ldb=ld_vec)
    X2 = run_op(rt, h, op, "L", uplo, "N", "N", 0.75, A, B, dt, ldb=ld_vec + 1)
    assert np.array_equal(X1, X2), (dt, leaf, op, uplo, m)
    assert eta(orc, op, "L", uplo, "N", "N", 0.75, A, B, X1) <= TOL[dt]


@pytest.mark.parametrize("dt,leaf", [("f64", 64), ("f64", 256), ("f32", 128)])
@pytest.mark.parametrize("side,uplo,trans", [("L", "L", "N"), ("L", "U", "T"), ("L", "U", "N"), ("R", "L", "N"),
                                             ("R", "U", "T")])
@pytest.mark.parametrize("shape", [(600, 130), (1000, 257), (301, 70)])
def test_trmm_leaf_schedules_agree(rt, h, orc, dt, leaf, side, uplo, trans, shape):
    """TRMM with one launch per leaf (recursion order) and with every leaf in
    one launch after saving the panel, then all updates in one grouped launch:
    the GEMM updates see the same operands and every entry the same MFMA
    sequence (no update of these orders splits K), so the results agree bit
    for bit; both pass the oracle's bound."""
    m, n = shape if side == "L" else shape[::-1]
    say("trmm schedules", dt, leaf, side, uplo, trans, m, n)
    A, B = _inputs(side, uplo, "N", m, n, dt, G(17, m, n))
    h.set_option(rt.OPT_LEAF_F64 if dt == "f64" else rt.OPT_LEAF_F32, leaf)
    out = []
    for mode in (1, 2):
        h.set_option(rt.OPT_TRMM_LEAVES, mode)
        out.append(run_op(rt, h, "trmm", side, uplo, trans, "N", -1.25, A, B, dt))
    h.set_option(rt.OPT_TRMM_LEAVES, 0)
    assert np.array_equal(out[0], out[1]), (dt, leaf, side, uplo, trans, shape)
    assert eta(orc, "trmm", side, uplo, trans, "N", -1.25, A, B, out[1]) <= TOL[dt]


@pytest.mark.parametrize("op", ["trsm", "trmm"])
def test_alpha_zero_reads_nothing(rt, h, op):
    m, n = 70, 33
    say("alpha0", op)
    A = np.full((m, m), np.nan, order="F")
    B = synth.dense(m, n, G(6))
    X = run_op(rt, h, op, "L", "L", "N", "N", 0.0, A, B, "f64")
    assert np.array_equal(X, np.zeros((m, n)))


@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("side,uplo,trans", [("L", "L", "N"), ("L", "U", "T"), ("R", "U", "N"), ("R", "L", "T")])
def test_nan_sentinels_not_read(rt, h, orc, op, side, uplo, trans):
    m, n = 150, 90
    say("sentinel", op, side, uplo, trans)
    g = G(7)
    ka = m if side == "L" else n
    A = synth.tri(ka, uplo, g, "unit", fill=np.nan)   # NaN off the triangle and on the diagonal
    B = synth.dense(m, n, g)
    X = run_op(rt, h, op, side, uplo, trans, "U", 1.0, A, B, "f64")
    assert np.all(np.isfinite(X))
    assert eta(orc, op, side, uplo, trans, "U", 1.0, A, B, X) <= TOL["f64"]


def test_deterministic(rt, h):
    m = n = 700
    say("determinism")
    A, B = _inputs("L", "L", "N", m, n, "f64", G(8))
    X1 = run_op(rt, h, "trsm", "L", "L", "N", "N", 1.0, A, B, "f64")
    X2 = run_op(rt, h, "trsm", "L", "L", "N", "N", 1.0, A, B, "f64")
    assert np.array_equal(X1, X2)


def test_empty_is_noop(rt, h):
    A = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    for shape in [(0, 4), (4, 0)]:
        B = torch.zeros(shape, dtype=torch.float64, device="cuda")
        assert rt.rtri_dtrsm(h.ptr, 0, 0, 0, 0, shape[0], shape[1], 1.0, A.data_ptr(), 4, B.data_ptr(),
                             max(1, shape[0])) == 0


# ---- the m = n = 512 FP64 case and the square sweep (column-sampled) --------------

@pytest.mark.parametrize("op", ["trsm", "trmm"])
def test_small_config_512(rt, h, orc, op):
    """FP64 left / lower / no-trans / non-unit, m = n = 512, alpha = 1, base generator."""
    m = n = 512
    say("c512", op)
    g = synth.rng(synth.W_SMALL, 0)
    A = synth.tri(m, "L", g, "base")
    B = synth.dense(m, n, g)
    X = run_op(rt, h, op, "L", "L", "N", "N", 1.0, A, B, "f64")
    Xo = oracle_op(orc, op, "L", "L", "N", "N", 1.0, A, B)
    assert eta(orc, op, "L", "L", "N", "N", 1.0, A, B, X) <= 1e-13
    assert np.max(np.abs(X - Xo)) <= 1e-13 * np.max(np.abs(Xo))


def _sampled_check(rt, h, orc, op, side, uplo, trans, diag, m, dt, kind, nsamp=16):
    n = m
    g = synth.rng(synth.W_SWEEP, m, zlib.crc32(f"{side}{uplo}{trans}{diag}{dt}".encode()) & 0xFFFF)
    A = rounded(synth.tri(m, uplo, g, kind), dt)
    B = rounded(synth.dense(m, n, g), dt)
    X = run_op(rt, h, op, side, uplo, trans, diag, 1.0, A, B, dt)
    idx = np.sort(synth.rng(synth.W_SWEEP, m, 77).choice(n if side == "L" else m, nsamp, replace=False))
    if side == "L":
        Bs, Xs = np.asfortranarray(B[:, idx]), np.asfortranarray(X[:, idx])
    else:
        Bs, Xs = np.asfortranarray(B[idx, :]), np.asfortranarray(X[idx, :])
    e = eta(orc, op, side, uplo, trans, diag, 1.0, A, Bs, Xs)
    Xo = oracle_op(orc, op, side, uplo, trans, diag, 1.0, A, Bs)
    return e, np.max(np.abs(Xs - Xo)) / np.max(np.abs(Xo))


@pytest.mark.parametrize("m", [1024, 2048, 4096])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("op", ["trsm", "trmm"])
def test_sweep_sampled(rt, h, orc, m, dt, op):
    for (side, uplo, trans, diag) in [("L", "L", "N", "N"), ("R", "U", "T", "N"), ("L", "U", "N", "U")]:
        say("sweep", m, dt, op, side, uplo, trans, diag)
        kind = "unit" if diag == "U" else "stress"
        e, fwd = _sampled_check(rt, h, orc, op, side, uplo, trans, diag, m, dt, kind)
        assert e <= TOL[dt], (m, dt, op, side, uplo, trans, diag, e)
        assert fwd <= 100 * TOL[dt]


@pytest.mark.parametrize("op", ["trsm", "trmm"])
def test_full_size_16384_sampled(rt, h, orc, op):
    """The headline workload: FP64 L/L/N/N at m = n = 16384 (base generator), in the
    launch configuration the benchmark times; checked on sampled columns."""
    say("c16384", op)
    e, fwd = _sampled_check(rt, h, orc, op, "L", "L", "N", "N", 16384, "f64", "base", nsamp=8)
    assert e <= 1e-13, e
    assert fwd <= 1e-12
