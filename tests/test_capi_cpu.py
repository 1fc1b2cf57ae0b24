"""The C-ABI library without a GPU: it loads, exports every function that
include/rtri.h declares, and validates arguments (BLAS position codes, quick
returns) before touching the device.  No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtri.h")
LIB = os.path.join(ROOT, "paper_2504_13821_amd", "librtri.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rtri_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_api():
    names = declared_functions()
    for must in ("rtri_create", "rtri_dtrsm", "rtri_strsm", "rtri_dtrmm", "rtri_strmm"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python paper_2504_13821_amd/build.py)"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rtri_[a-z0-9_]+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"


@pytest.fixture(scope="module")
def rt():
    import paper_2504_13821_amd as rt
    return rt


@pytest.fixture()
def handle(rt):
    h = ctypes.c_void_p()
    assert rt.rtri_create(ctypes.byref(h), None) == rt.OK
    yield h
    assert rt.rtri_destroy(h) == rt.OK


FAKE = 0x1000   # never dereferenced: every call below returns before launching work

BAD_ARGS = [
    # (side, uplo, trans, diag, m, n, A, lda, B, ldb) -> expected code
    ((2, 0, 0, 0, 4, 4, FAKE, 4, FAKE, 4), -1),
    ((0, 5, 0, 0, 4, 4, FAKE, 4, FAKE, 4), -2),
    ((0, 0, 3, 0, 4, 4, FAKE, 4, FAKE, 4), -3),
    ((0, 0, 0, -1, 4, 4, FAKE, 4, FAKE, 4), -4),
    ((0, 0, 0, 0, -1, 4, FAKE, 4, FAKE, 4), -5),
    ((0, 0, 0, 0, 4, -2, FAKE, 4, FAKE, 4), -6),
    ((0, 0, 0, 0, 4, 4, 0, 4, FAKE, 4), -8),
    ((0, 0, 0, 0, 4, 4, FAKE, 3, FAKE, 4), -9),       # side L: lda >= m
    ((1, 0, 0, 0, 4, 6, FAKE, 5, FAKE, 4), -9),       # side R: lda >= n
    ((0, 0, 0, 0, 4, 4, FAKE, 4, 0, 4), -10),
    ((0, 0, 0, 0, 4, 4, FAKE, 4, FAKE, 3), -11),
    ((0, 0, 0, 0, 0, 4, FAKE, 1, FAKE, 1), 0),        # quick return m = 0
    ((1, 1, 1, 1, 4, 0, FAKE, 1, FAKE, 4), 0),        # quick return n = 0
    ((0, 0, 0, 0, 0, 0, 0, 1, 0, 1), 0),              # empty with NULL pointers
]


@pytest.mark.parametrize("fname", ["rtri_dtrsm", "rtri_strsm", "rtri_dtrmm", "rtri_strmm", "rtri_dtrsm_noalloc",
                                   "rtri_dtrmm_ozaki"])
@pytest.mark.parametrize("args,code", BAD_ARGS)
def test_argument_codes(rt, handle, fname, args, code):
    side, uplo, trans, diag, m, n, A, lda, B, ldb = args
    fn = getattr(rt, fname)
    assert fn(handle, side, uplo, trans, diag, m, n, 1.0, A, lda, B, ldb) == code


def test_null_handle(rt):
    assert rt.rtri_dtrsm(None, 0, 0, 0, 0, 1, 1, 1.0, FAKE, 1, FAKE, 1) == rt.ERR_HANDLE
    assert rt.rtri_sync(None) == rt.ERR_HANDLE
    assert rt.rtri_destroy(None) == rt.ERR_HANDLE


def test_options(rt, handle):
    v = ctypes.c_int64()
    assert rt.rtri_set_option(handle, rt.OPT_LEAF_F64, 32) == rt.OK
    assert rt.rtri_get_option(handle, rt.OPT_LEAF_F64, ctypes.byref(v)) == rt.OK and v.value == 32
    assert rt.rtri_set_option(handle, rt.OPT_LEAF_F64, 48) == -3
    for leaf in (16, 64, 128, 256, 0):
        assert rt.rtri_set_option(handle, rt.OPT_LEAF_F32, leaf) == rt.OK
    assert rt.rtri_set_option(handle, rt.OPT_LEAF_F32, 512) == -3
    for mode in (0, 1, 2):
        assert rt.rtri_set_option(handle, rt.OPT_TRMM_LEAVES, mode) == rt.OK
        assert rt.rtri_get_option(handle, rt.OPT_TRMM_LEAVES, ctypes.byref(v)) == rt.OK and v.value == mode
    assert rt.rtri_set_option(handle, rt.OPT_TRMM_LEAVES, 3) == -3
    for opt, top in ((rt.OPT_GEMM16_TILE, 3), (rt.OPT_RESIDUAL, 1)):
        assert rt.rtri_get_option(handle, opt, ctypes.byref(v)) == rt.OK and v.value == 0
        for mode in range(top + 1):
            assert rt.rtri_set_option(handle, opt, mode) == rt.OK
            assert rt.rtri_get_option(handle, opt, ctypes.byref(v)) == rt.OK and v.value == mode
        assert rt.rtri_set_option(handle, opt, top + 1) == -3
        assert rt.rtri_set_option(handle, opt, -1) == -3
    assert rt.rtri_set_option(handle, 999, 1) == -2


def test_status_strings(rt):
    assert rt.rtri_status_string(0) == b"success"
    assert rt.rtri_status_string(-9) == b"lda too small"
    assert rt.rtri_status_string(rt.ERR_HIP) == b"HIP runtime error"


def test_tuning_db_load(rt, handle, tmp_path):
    good = tmp_path / "t.json"
    good.write_text('{"arch": "gfx950", "version": 1, "leaf": [{"dtype": "f64", "op": "trsm", "ka_max": 1024, '
                    '"n_max": 512, "leaf": 32}], "gemm_tile": [{"dtype": "f32", "m_max": 256, "n_max": 4096, "tile": 2}]}')
    assert rt.rtri_load_tuning(handle, str(good).encode()) == rt.OK
    bad = tmp_path / "b.json"
    bad.write_text('{"leaf": [{"dtype": "f64", "op": "trsm", "ka_max": 1024, "n_max": 512, "leaf": 48}]}')
    assert rt.rtri_load_tuning(handle, str(bad).encode()) == rt.ERR_INVALID
    assert rt.rtri_load_tuning(handle, str(tmp_path / "missing.json").encode()) == rt.ERR_INVALID
    (tmp_path / "trunc.json").write_text('{"leaf": [')
    assert rt.rtri_load_tuning(handle, str(tmp_path / "trunc.json").encode()) == rt.ERR_INVALID


def _leaf(rt, handle, dt, op, order, nvec):
    v = ctypes.c_int()
    assert rt.rtri_query_leaf(handle, dt, op, order, nvec, ctypes.byref(v)) == rt.OK
    return v.value


def test_leaf_policy(rt, handle, tmp_path):
    # untuned: 64-row leaves up to order 1024 (the batched kernel's size), 256 above
    assert _leaf(rt, handle, rt.F64, 0, 1024, 100) == 64
    assert _leaf(rt, handle, rt.F32, 1, 1025, 100) == 256
    # rules: the smallest bucket that covers the order, then the vector count
    db = tmp_path / "t.json"
    db.write_text('{"leaf": [{"dtype": "f64", "op": "trsm", "ka_max": 1024, "n_max": 512, "leaf": 32},'
                  '{"dtype": "f64", "op": "trsm", "ka_max": 1024, "n_max": 4096, "leaf": 128},'
                  '{"dtype": "f64", "op": "trsm", "ka_max": 4096, "n_max": 512, "leaf": 256}]}')
    assert rt.rtri_load_tuning(handle, str(db).encode()) == rt.OK
    assert _leaf(rt, handle, rt.F64, 0, 700, 100) == 32
    assert _leaf(rt, handle, rt.F64, 0, 700, 1000) == 128
    assert _leaf(rt, handle, rt.F64, 0, 3000, 10) == 256
    assert _leaf(rt, handle, rt.F64, 0, 99999, 10) == 256        # past the largest bucket: the largest
    # an explicit option wins over the rules
    assert rt.rtri_set_option(handle, rt.OPT_LEAF_F64, 16) == rt.OK
    assert _leaf(rt, handle, rt.F64, 0, 3000, 10) == 16
    v = ctypes.c_int()
    assert rt.rtri_query_leaf(handle, 7, 0, 1, 1, ctypes.byref(v)) == -2
    assert rt.rtri_query_leaf(handle, rt.F64, 2, 1, 1, ctypes.byref(v)) == -3
    assert rt.rtri_query_leaf(handle, rt.F64, 0, -1, 1, ctypes.byref(v)) == -4


def test_shipped_tuning_rules_load(rt, handle):
    assert rt.rtri_load_tuning(handle, rt.TUNING_DB.encode()) == rt.OK
    for dt in (rt.F64, rt.F32):
        for op in (0, 1):
            assert _leaf(rt, handle, dt, op, 16384, 16384) in (16, 32, 64, 128, 256)


# ---- the Python wrappers reject undersized operands before any C call --------

class _NoCall:
    """Stands in for every C entry point: a wrapper that reaches it fails the test."""

    def __init__(self, name):
        self.__name__ = name

    def __call__(self, *a):
        raise AssertionError(f"{self.__name__} was called")


@pytest.fixture()
def guarded(rt, monkeypatch):
    for name in ("rtri_dtrsm", "rtri_dtrmm", "rtri_strsm", "rtri_strmm", "rtri_trmm_ex", "rtri_dtrsm_mixed",
                 "rtri_gemm_update"):
        monkeypatch.setattr(rt, name, _NoCall(name))
    return rt


def _cm(torch, rows, cols, dtype=None):
    """A column-major (stride(0) == 1) CPU tensor of shape (rows, cols)."""
    return torch.zeros((cols, rows), dtype=dtype or torch.float64).t()


def test_wrappers_reject_bad_shapes(guarded):
    rt = guarded
    torch = pytest.importorskip("torch")
    h = None   # never reached
    A_small = _cm(torch, 8, 4)          # lda >= 8 but only 4 columns: an order-8 factor would be read past its end
    B = _cm(torch, 8, 5)
    for fn in (rt.trsm, rt.trmm):
        with pytest.raises(ValueError, match="A has shape"):
            fn(h, "L", "L", "N", "N", 1.0, A_small, B)
        with pytest.raises(ValueError, match="A has shape"):
            fn(h, "R", "L", "N", "N", 1.0, _cm(torch, 5, 4), B)
    with pytest.raises(ValueError, match="A has shape"):
        rt.trsm_mixed(h, "L", "L", "N", "N", 1.0, A_small, B)
    A16 = _cm(torch, 8, 8, torch.bfloat16)
    with pytest.raises(ValueError, match="B has shape"):
        rt.trmm_ex(h, "L", "L", "N", "N", 1.0, A16, _cm(torch, 8, 4, torch.bfloat16), _cm(torch, 8, 5, torch.float32))
    with pytest.raises(ValueError, match="A has shape"):
        rt.trmm_ex(h, "L", "L", "N", "N", 1.0, _cm(torch, 8, 7, torch.bfloat16), _cm(torch, 8, 5, torch.bfloat16),
                   _cm(torch, 8, 5, torch.float32))
    # GEMM update: C (M x N) = op(P) (M x K) op(Q) (K x N)
    C = _cm(torch, 6, 5)
    with pytest.raises(ValueError, match="Q has shape"):
        rt.gemm_update(h, "N", "N", 1.0, _cm(torch, 6, 4), _cm(torch, 3, 5), 0.0, C)
    with pytest.raises(ValueError, match="P has shape"):
        rt.gemm_update(h, "T", "N", 1.0, _cm(torch, 4, 5), _cm(torch, 4, 5), 0.0, C)
    # well-shaped host tensors pass the shape checks and stop at the device check
    with pytest.raises(ValueError, match="device tensor"):
        rt.trsm(h, "L", "L", "N", "N", 1.0, _cm(torch, 8, 8), B)


# ---- factor objects: argument codes (no device work is reached) -----------------

def test_factor_argument_codes(rt, handle):
    f = ctypes.c_void_p()
    create = rt.rtri_factor_create
    assert create(handle, 2, 0, 8, rt.F64, FAKE, 8, 0, ctypes.byref(f)) == -2
    assert create(handle, 0, 5, 8, rt.F64, FAKE, 8, 0, ctypes.byref(f)) == -3
    assert create(handle, 0, 0, -1, rt.F64, FAKE, 8, 0, ctypes.byref(f)) == -4
    assert create(handle, 0, 0, 8, rt.BF16, FAKE, 8, 0, ctypes.byref(f)) == -5
    assert create(handle, 0, 0, 8, rt.F64, None, 8, 0, ctypes.byref(f)) == -6
    assert create(handle, 0, 0, 8, rt.F64, FAKE, 7, 0, ctypes.byref(f)) == -7
    assert create(handle, 0, 0, 8, rt.F64, FAKE, 8, 4, ctypes.byref(f)) == -8
    assert create(handle, 0, 0, 8, rt.F64, FAKE, 8, 0, None) == -9
    assert create(None, 0, 0, 8, rt.F64, FAKE, 8, 0, ctypes.byref(f)) == rt.ERR_HANDLE
    # without the copy flag, creation does no device work
    assert create(handle, 0, 0, 8, rt.F64, FAKE, 8, 0, ctypes.byref(f)) == rt.OK
    trsm, trmm = rt.rtri_factor_trsm, rt.rtri_factor_trmm
    ok = (0, 0, 8, 3, 1.0, FAKE, 8)
    cases = [((2, 0, 8, 3, 1.0, FAKE, 8), -3), ((0, 3, 8, 3, 1.0, FAKE, 8), -4), ((0, 0, 7, 3, 1.0, FAKE, 8), -5),
             ((0, 0, -1, 3, 1.0, FAKE, 8), -5), ((1, 0, 3, 7, 1.0, FAKE, 3), -6), ((0, 0, 8, -1, 1.0, FAKE, 8), -6),
             ((0, 0, 8, 3, 1.0, None, 8), -8), ((0, 0, 8, 3, 1.0, FAKE, 7), -9)]
    for args, code in cases:
        assert trsm(handle, f, *args, 0, 1e-12, 10, None) == code, (args, code)
        assert trmm(handle, f, *args) == code, (args, code)
    assert trsm(handle, f, *ok, 7, 1e-12, 10, None) == -10
    assert trsm(handle, f, *ok, 2, -1.0, 10, None) == -11
    assert trsm(handle, f, *ok, 2, 1e-12, 0, None) == -12
    assert trsm(handle, None, *ok, 0, 1e-12, 10, None) == -2
    # quick returns: no vectors
    assert trsm(handle, f, 0, 0, 8, 0, 1.0, None, 8, 2, 1e-12, 10, None) == rt.OK
    assert trmm(handle, f, 1, 0, 0, 8, 1.0, None, 1) == rt.OK
    nb = ctypes.c_int64(-1)
    assert rt.rtri_factor_bytes(f, ctypes.byref(nb)) == rt.OK and nb.value == 0
    assert rt.rtri_factor_destroy(f) == rt.OK
    f32 = ctypes.c_void_p()
    assert create(handle, 1, 1, 8, rt.F32, FAKE, 8, 0, ctypes.byref(f32)) == rt.OK
    # a refined solve needs an FP64 factor
    assert trsm(handle, f32, *ok, 1, 1e-12, 10, None) == rt.ERR_UNSUPPORTED
    assert rt.rtri_factor_destroy(f32) == rt.OK


def test_solver_argument_codes(rt, handle):
    """TRTRI / POTRS / GETRS reject bad arguments (and bad pivots) before any
    device work; empty problems return at once."""
    for fn in (rt.rtri_dtrtri, rt.rtri_strtri):
        assert fn(handle, 2, 0, 4, FAKE, 4) == -2
        assert fn(handle, 0, 2, 4, FAKE, 4) == -3
        assert fn(handle, 0, 0, -1, FAKE, 4) == -4
        assert fn(handle, 0, 0, 4, None, 4) == -5
        assert fn(handle, 0, 0, 4, FAKE, 3) == -6
        assert fn(handle, 1, 1, 0, None, 1) == rt.OK
    for fn in (rt.rtri_dpotrs, rt.rtri_spotrs):
        assert fn(handle, 3, 4, 2, FAKE, 4, FAKE, 4) == -2
        assert fn(handle, 0, -1, 2, FAKE, 4, FAKE, 4) == -3
        assert fn(handle, 0, 4, -2, FAKE, 4, FAKE, 4) == -4
        assert fn(handle, 0, 4, 2, None, 4, FAKE, 4) == -5
        assert fn(handle, 0, 4, 2, FAKE, 3, FAKE, 4) == -6
        assert fn(handle, 0, 4, 2, FAKE, 4, None, 4) == -7
        assert fn(handle, 0, 4, 2, FAKE, 4, FAKE, 3) == -8
        assert fn(handle, 0, 4, 0, FAKE, 4, None, 4) == rt.OK
    piv = (ctypes.c_int32 * 4)(1, 2, 3, 4)
    badpiv = (ctypes.c_int32 * 4)(1, 5, 3, 4)
    zeropiv = (ctypes.c_int32 * 4)(0, 2, 3, 4)
    for fn in (rt.rtri_dgetrs, rt.rtri_sgetrs):
        assert fn(handle, 4, 4, 2, FAKE, 4, piv, FAKE, 4) == -2
        assert fn(handle, 0, -1, 2, FAKE, 4, piv, FAKE, 4) == -3
        assert fn(handle, 0, 4, -1, FAKE, 4, piv, FAKE, 4) == -4
        assert fn(handle, 0, 4, 2, None, 4, piv, FAKE, 4) == -5
        assert fn(handle, 0, 4, 2, FAKE, 3, piv, FAKE, 4) == -6
        assert fn(handle, 0, 4, 2, FAKE, 4, None, FAKE, 4) == -7
        assert fn(handle, 0, 4, 2, FAKE, 4, badpiv, FAKE, 4) == -7
        assert fn(handle, 1, 4, 2, FAKE, 4, zeropiv, FAKE, 4) == -7
        assert fn(handle, 0, 4, 2, FAKE, 4, piv, None, 4) == -8
        assert fn(handle, 0, 4, 2, FAKE, 4, piv, FAKE, 3) == -9
        assert fn(handle, 0, 4, 0, FAKE, 4, piv, None, 4) == rt.OK


def test_noalloc_rejects_problems_beyond_its_scratch(rt, handle):
    """rtri_dtrsm_noalloc refuses a factor whose packed blocks exceed its fixed
    array (ka = 40000 with 256-row leaves: 157 blocks of 278528 bytes) before
    any device work; the allocating entry point has no such limit."""
    assert rt.rtri_set_option(handle, rt.OPT_LEAF_F64, 256) == rt.OK
    big = 40000
    assert rt.rtri_dtrsm_noalloc(handle, 0, 0, 0, 0, big, 1, 1.0, FAKE, big, FAKE, big) == rt.ERR_TOO_LARGE
    assert rt.rtri_dtrsm_noalloc(handle, 1, 0, 0, 0, 1, big, 1.0, FAKE, big, FAKE, 1) == rt.ERR_TOO_LARGE
    assert b"scratch" in rt.rtri_status_string(rt.ERR_TOO_LARGE)
    # an open profile is refused (it would create events on demand)
    assert rt.rtri_profile_begin(handle) == rt.OK
    assert rt.rtri_dtrsm_noalloc(handle, 0, 0, 0, 0, 4, 4, 1.0, FAKE, 4, FAKE, 4) == rt.ERR_UNSUPPORTED


def test_ozaki_order_limit(rt, handle):
    """The INT8-product TRMM refuses orders whose exact INT32 sums could
    overflow (K > 2^17) before any device work."""
    big = (1 << 17) + 1
    assert rt.rtri_dtrmm_ozaki(handle, 0, 0, 0, 0, big, 1, 1.0, FAKE, big, FAKE, big) == rt.ERR_UNSUPPORTED


def test_call_plan_argument_codes(rt, handle):
    """rtri_call_plan_create rejects bad arguments before any device work: op,
    dtype, then the BLAS-list codes shifted by three, and a NULL out."""
    p = ctypes.c_void_p()
    make = rt.rtri_call_plan_create
    ok = (0, 0, 0, 0, 8, 4, 1.0, FAKE, 8, FAKE, 8)
    assert make(handle, 2, rt.F64, *ok, ctypes.byref(p)) == -2
    assert make(handle, 0, rt.BF16, *ok, ctypes.byref(p)) == -3
    assert make(handle, 0, rt.F64, 2, 0, 0, 0, 8, 4, 1.0, FAKE, 8, FAKE, 8, ctypes.byref(p)) == -4
    assert make(handle, 1, rt.F32, 0, 0, 0, 0, -1, 4, 1.0, FAKE, 8, FAKE, 8, ctypes.byref(p)) == -8
    assert make(handle, 0, rt.F64, 0, 0, 0, 0, 8, 4, 1.0, FAKE, 7, FAKE, 8, ctypes.byref(p)) == -12
    assert make(handle, 0, rt.F64, 0, 0, 0, 0, 8, 4, 1.0, FAKE, 8, FAKE, 7, ctypes.byref(p)) == -14
    assert make(handle, 0, rt.F64, *ok, None) == -15
    assert make(None, 0, rt.F64, *ok, ctypes.byref(p)) == rt.ERR_HANDLE
    assert rt.rtri_call_plan_run(None) == rt.ERR_HANDLE
    assert rt.rtri_call_plan_destroy(None) == -1
