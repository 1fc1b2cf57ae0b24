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


@pytest.mark.parametrize("fname", ["rtri_dtrsm", "rtri_strsm", "rtri_dtrmm", "rtri_strmm"])
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
