"""Complex FP64 TRSM / TRMM on the GPU (rtri_ztrsm / rtri_ztrmm: op(A) = A,
A^T or conj(A^T), eqs. (1)-(4)) against the complex oracle.

Tolerance: the normwise backward error of the FP64 real paths, eta <= 1e-13
(complex products and Smith's division add a few units of roundoff per
operation, far inside that margin).  Exact Gaussian-integer inputs with
power-of-two real diagonals keep every intermediate exact, so the GPU must
equal the oracle bit for bit there."""
import numpy as np
import pytest

import synth
from dense_ref import VARIANTS
from gpu_util import say

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
    return synth.rng(synth.W_TEST, 7600, *k)


def ztri(n, uplo, g, kind="stress"):
    re = synth.tri(n, uplo, g, kind)
    im = synth.tri(n, uplo, g, kind)
    if kind != "unit":
        im[np.diag_indices(n)] = 0.5 * g.random(n)
    return np.asfortranarray(re + 1j * im)


def zdense(m, n, g):
    return np.asfortranarray(synth.dense(m, n, g) + 1j * synth.dense(m, n, g))


def _run(rt, h, op, side, uplo, trans, diag, alpha, A, B):
    Ad = rt.to_device(A, torch.complex128)
    Bd = rt.to_device(B, torch.complex128)
    (rt.ztrsm if op == "trsm" else rt.ztrmm)(h, side, uplo, trans, diag, alpha, Ad, Bd)
    torch.cuda.synchronize()
    return rt.to_host(Bd)


def _eta(orc, op, *args):
    return (orc.ztrsm_eta if op == "trsm" else orc.ztrmm_eta)(*args)


@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("diag", "NU")
@pytest.mark.parametrize("side,uplo,trans", VARIANTS)
def test_complex_variants(rt, h, orc, op, diag, side, uplo, trans):
    m, n = (150, 70) if side == "L" else (70, 150)
    say("complex", op, side, uplo, trans, diag)
    g = G(1, m, ord(side), ord(uplo), ord(trans))
    ka = m if side == "L" else n
    A = ztri(ka, uplo, g, "unit" if diag == "U" else "stress")
    B = zdense(m, n, g)
    alpha = 0.75 - 0.5j
    X = _run(rt, h, op, side, uplo, trans, diag, alpha, A, B)
    e = _eta(orc, op, side, uplo, trans, diag, alpha, A, B, X)
    assert e <= 1e-13, (op, side, uplo, trans, diag, e)


@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("side,uplo,trans,m,n", [("L", "L", "C", 1100, 130), ("L", "U", "N", 777, 300),
                                                  ("R", "U", "T", 90, 1030), ("R", "L", "C", 200, 600)])
def test_complex_several_levels(rt, h, orc, op, side, uplo, trans, m, n):
    """Orders spanning several leaves and GEMM levels, ragged."""
    say("complex levels", op, side, uplo, trans, m, n)
    g = G(2, m, n)
    ka = m if side == "L" else n
    A = ztri(ka, uplo, g, "stress")
    B = zdense(m, n, g)
    X = _run(rt, h, op, side, uplo, trans, "N", -1.5 + 0.25j, A, B)
    e = _eta(orc, op, side, uplo, trans, "N", -1.5 + 0.25j, A, B, X)
    assert e <= 1e-13, (op, e)


@pytest.mark.parametrize("op", ["trsm", "trmm"])
@pytest.mark.parametrize("side,uplo,trans", [("L", "L", "N"), ("L", "U", "C"), ("R", "L", "T"), ("R", "U", "C")])
def test_complex_exact_gaussian_integers(rt, h, orc, op, side, uplo, trans):
    """Off-diagonals in {-1, 0, 1} + i{-1, 0, 1}, diagonals in {+-1, +-2}
    (real), Gaussian-integer B: every partial sum and quotient is exact (the
    order stays small enough), so the GPU equals the oracle bit for bit."""
    ka = 24 if op == "trsm" else 96
    other = 9
    m, n = (ka, other) if side == "L" else (other, ka)
    say("complex exact", op, side, uplo, trans)
    g = G(3, ka, ord(side), ord(uplo), ord(trans))
    re = g.integers(-1, 2, size=(ka, ka)).astype(np.float64)
    im = g.integers(-1, 2, size=(ka, ka)).astype(np.float64)
    A = re + 1j * im
    A[np.diag_indices(ka)] = g.choice([1.0, -1.0, 2.0, -2.0] if op == "trmm" else [1.0, -1.0], size=ka)
    A = np.asfortranarray(A)
    B = np.asfortranarray(g.integers(-4, 5, size=(m, n)) + 1j * g.integers(-4, 5, size=(m, n))).astype(np.complex128)
    X = _run(rt, h, op, side, uplo, trans, "N", 1.0, A, B)
    want = (orc.ztrsm if op == "trsm" else orc.ztrmm)(side, uplo, trans, "N", 1.0, A, B)
    assert np.array_equal(X, want)


def test_complex_alpha_zero_and_empty(rt, h):
    say("complex alpha=0 / empty")
    A = torch.full((30, 30), complex(float("nan"), 0.0), dtype=torch.complex128, device="cuda").t()
    B = torch.ones((20, 30), dtype=torch.complex128, device="cuda").t()
    rt.ztrsm(h, "L", "L", "N", "N", 0.0, A, B)
    torch.cuda.synchronize()
    assert torch.count_nonzero(B).item() == 0
    E = torch.zeros((30, 0), dtype=torch.complex128, device="cuda")
    rt.ztrmm(h, "L", "L", "N", "N", 1.0, A, E)
    torch.cuda.synchronize()
