"""The FP64 TRSM that allocates nothing (rtri_dtrsm_noalloc) against the
allocating entry point (rtri_dtrsm) and the oracle.

The two entry points build the same plan and run the same kernels, only the
workspace differs (a fixed device array against the handle's allocations), so
their results must agree bit for bit; each result must also meet the FP64
backward-error bound against the oracle (eta <= 1e-13).  Two calls in a row on
one handle, the second smaller than the first, so the second runs on the
array the first left behind."""
import numpy as np
import pytest

import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_13821_amd as rt
    return rt


# (side, uplo, trans, diag, m, n): the first spans several 256-row leaves and a
# narrow panel whose long updates split K; the second is smaller and ragged
CASES = [("L", "L", "N", "N", 4133, 300), ("R", "U", "T", "U", 777, 129)]


def _inputs(side, uplo, diag, m, n, seed):
    g = synth.rng(synth.W_TEST, 7100, seed)
    ka = m if side == "L" else n
    A = synth.tri(ka, uplo, g, "unit" if diag == "U" else "base")
    B = synth.dense(m, n, g)
    return A, B


def test_noalloc_matches_dtrsm_twice(rt, orc):
    h = rt.Handle()
    try:
        for i, (side, uplo, trans, diag, m, n) in enumerate(CASES):
            say("noalloc", i, side, uplo, trans, diag, m, n)
            A, B = _inputs(side, uplo, diag, m, n, i)
            alpha = -1.5 if i == 0 else 0.75
            Ad = rt.to_device(A, torch.float64)
            B1 = rt.to_device(B, torch.float64)
            B2 = rt.to_device(B, torch.float64)
            rt.trsm_noalloc(h, side, uplo, trans, diag, alpha, Ad, B1)
            rt.trsm(h, side, uplo, trans, diag, alpha, Ad, B2)
            torch.cuda.synchronize()
            X1, X2 = rt.to_host(B1), rt.to_host(B2)
            assert np.array_equal(X1, X2), (i, float(np.max(np.abs(X1 - X2))))
            # oracle on sampled vectors (columns for side L, rows for side R)
            k = 16
            if side == "L":
                idx = np.linspace(0, n - 1, k).astype(int)
                e = orc.trsm_eta(side, uplo, trans, diag, alpha, A, B[:, idx], X1[:, idx])
            else:
                idx = np.linspace(0, m - 1, k).astype(int)
                e = orc.trsm_eta(side, uplo, trans, diag, alpha, A, B[idx, :], X1[idx, :])
            say("noalloc", i, "eta", e)
            assert e <= 1e-13, (i, e)
    finally:
        h.close()


def test_noalloc_alpha_zero_and_empty(rt):
    h = rt.Handle()
    try:
        say("noalloc alpha=0 / empty")
        A = torch.full((64, 64), float("nan"), dtype=torch.float64, device="cuda").t()
        B = torch.ones((64, 40), dtype=torch.float64, device="cuda").t().contiguous().t()
        rt.trsm_noalloc(h, "L", "L", "N", "N", 0.0, A, B)
        torch.cuda.synchronize()
        assert torch.count_nonzero(B).item() == 0
        E = torch.zeros((64, 0), dtype=torch.float64, device="cuda")
        rt.trsm_noalloc(h, "L", "L", "N", "N", 1.0, A, E)
        torch.cuda.synchronize()
    finally:
        h.close()
