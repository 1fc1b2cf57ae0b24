"""Python binding of librtri.so, the recursive TRMM / TRSM library for MI355X.

The functions named ``rtri_*`` mirror the C ABI in ``include/rtri.h`` one to
one (integers for pointers and streams).  ``Handle``, ``trsm`` and ``trmm`` add
argument marshalling for PyTorch tensors: device memory and streams come from
PyTorch, every step of the computation runs in the library's HIP kernels.
There is no fallback: importing this package on a machine without the built
library raises ImportError.

Matrices are column-major, as in BLAS: an m-by-n matrix is a torch tensor of
shape (m, n) with ``stride(0) == 1`` and leading dimension ``stride(1)``; see
``to_device``/``to_host`` for numpy Fortran-order conversion.
"""
from __future__ import annotations

import ctypes
import os

try:  # load PyTorch's HIP runtime first so the library shares it (one runtime per process)
    import torch
except ImportError:  # pragma: no cover - the library itself does not need torch
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtri.so")
HEADER = os.path.join(_HERE, "..", "include", "rtri.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2504_13821_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)

LEFT, RIGHT = 0, 1
LOWER, UPPER = 0, 1
NOTRANS, TRANS, CONJTRANS = 0, 1, 2
NONUNIT, UNIT = 0, 1
F64, F32, BF16, F16 = 0, 1, 2, 3
OK, ERR_HANDLE, ERR_HIP, ERR_NOMEM, ERR_UNSUPPORTED, NOT_CONVERGED, ERR_INVALID, ERR_TOO_LARGE = range(8)
OPT_LEAF_F64, OPT_LEAF_F32, OPT_GEMM_TILE, OPT_TRMM_LEAVES, OPT_GEMM16_TILE, OPT_RESIDUAL = 1, 2, 3, 4, 5, 6

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_OPARGS = (_vp, _int, _int, _int, _int, _i64, _i64)
rtri_create = _sig("rtri_create", _int, ctypes.POINTER(_vp), _vp)
rtri_destroy = _sig("rtri_destroy", _int, _vp)
rtri_set_stream = _sig("rtri_set_stream", _int, _vp, _vp)
rtri_sync = _sig("rtri_sync", _int, _vp)
rtri_set_option = _sig("rtri_set_option", _int, _vp, _int, _i64)
rtri_get_option = _sig("rtri_get_option", _int, _vp, _int, ctypes.POINTER(_i64))
rtri_status_string = _sig("rtri_status_string", ctypes.c_char_p, _int)
rtri_last_hip_error = _sig("rtri_last_hip_error", _int, _vp)
rtri_dtrsm = _sig("rtri_dtrsm", _int, *_OPARGS, ctypes.c_double, _vp, _i64, _vp, _i64)
rtri_strsm = _sig("rtri_strsm", _int, *_OPARGS, ctypes.c_float, _vp, _i64, _vp, _i64)
rtri_dtrmm = _sig("rtri_dtrmm", _int, *_OPARGS, ctypes.c_double, _vp, _i64, _vp, _i64)
rtri_strmm = _sig("rtri_strmm", _int, *_OPARGS, ctypes.c_float, _vp, _i64, _vp, _i64)
rtri_dtrsm_noalloc = _sig("rtri_dtrsm_noalloc", _int, *_OPARGS, ctypes.c_double, _vp, _i64, _vp, _i64)
rtri_dtrmm_ozaki = _sig("rtri_dtrmm_ozaki", _int, *_OPARGS, ctypes.c_double, _vp, _i64, _vp, _i64)
rtri_call_plan_create = _sig("rtri_call_plan_create", _int, _vp, _int, _int, _int, _int, _int, _int, _i64, _i64,
                             ctypes.c_double, _vp, _i64, _vp, _i64, ctypes.POINTER(_vp))
rtri_call_plan_run = _sig("rtri_call_plan_run", _int, _vp)
rtri_call_plan_destroy = _sig("rtri_call_plan_destroy", _int, _vp)
rtri_trmm_ex = _sig("rtri_trmm_ex", _int, *_OPARGS, ctypes.c_float, _vp, _int, _i64, _vp, _int, _i64, _vp, _int, _i64)


class RefineInfo(ctypes.Structure):
    _fields_ = [("iters", _int), ("converged", _int), ("eta", ctypes.c_double), ("anorm", ctypes.c_double),
                ("eta_hist", ctypes.c_double * 32)]


rtri_dtrsm_mixed = _sig("rtri_dtrsm_mixed", _int, *_OPARGS, ctypes.c_double, _vp, _i64, _vp, _i64, _int,
                        ctypes.c_double, _int, ctypes.POINTER(RefineInfo))
_c2 = ctypes.c_double * 2
rtri_ztrsm = _sig("rtri_ztrsm", _int, *_OPARGS, ctypes.POINTER(ctypes.c_double), _vp, _i64, _vp, _i64)
rtri_ztrmm = _sig("rtri_ztrmm", _int, *_OPARGS, ctypes.POINTER(ctypes.c_double), _vp, _i64, _vp, _i64)
rtri_dtrtri = _sig("rtri_dtrtri", _int, _vp, _int, _int, _i64, _vp, _i64)
rtri_strtri = _sig("rtri_strtri", _int, _vp, _int, _int, _i64, _vp, _i64)
rtri_dpotrs = _sig("rtri_dpotrs", _int, _vp, _int, _i64, _i64, _vp, _i64, _vp, _i64)
rtri_spotrs = _sig("rtri_spotrs", _int, _vp, _int, _i64, _i64, _vp, _i64, _vp, _i64)
rtri_dgetrs = _sig("rtri_dgetrs", _int, _vp, _int, _i64, _i64, _vp, _i64, _vp, _vp, _i64)
rtri_sgetrs = _sig("rtri_sgetrs", _int, _vp, _int, _i64, _i64, _vp, _i64, _vp, _vp, _i64)
rtri_factor_create = _sig("rtri_factor_create", _int, _vp, _int, _int, _i64, _int, _vp, _i64, ctypes.c_uint,
                          ctypes.POINTER(_vp))
rtri_factor_trsm = _sig("rtri_factor_trsm", _int, _vp, _vp, _int, _int, _i64, _i64, ctypes.c_double, _vp, _i64, _int,
                        ctypes.c_double, _int, ctypes.POINTER(RefineInfo))
rtri_factor_trmm = _sig("rtri_factor_trmm", _int, _vp, _vp, _int, _int, _i64, _i64, ctypes.c_double, _vp, _i64)
rtri_factor_bytes = _sig("rtri_factor_bytes", _int, _vp, ctypes.POINTER(_i64))
rtri_factor_destroy = _sig("rtri_factor_destroy", _int, _vp)
FACTOR_COPY = 1


class BatchEntry(ctypes.Structure):
    _fields_ = [("op", _int), ("side", _int), ("uplo", _int), ("trans", _int), ("diag", _int), ("m", _i64),
                ("n", _i64), ("alpha", ctypes.c_double), ("A", _vp), ("lda", _i64), ("B", _vp), ("ldb", _i64)]


rtri_batch_plan_create = _sig("rtri_batch_plan_create", _int, _vp, _int, _int, ctypes.POINTER(BatchEntry),
                              ctypes.POINTER(_vp), ctypes.POINTER(_int))
rtri_batch_plan_run = _sig("rtri_batch_plan_run", _int, _vp)
rtri_batch_plan_chunks = _sig("rtri_batch_plan_chunks", _int, _vp, ctypes.POINTER(_i64))
rtri_batch_plan_destroy = _sig("rtri_batch_plan_destroy", _int, _vp)
rtri_batched = _sig("rtri_batched", _int, _vp, _int, _int, ctypes.POINTER(BatchEntry), ctypes.POINTER(_int))
rtri_synth_fill = _sig("rtri_synth_fill", _int, _vp, _int, _int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                       _i64, _i64, ctypes.c_double, _vp, _i64)


class ServerCfg(ctypes.Structure):
    _fields_ = [("slots", _int), ("hbm_budget", _i64), ("max_batch", _int), ("small_max", _i64),
                ("synth_seed", ctypes.c_uint64), ("refine_requeue", _int), ("mixed_batch", _int)]


class Request(ctypes.Structure):
    _fields_ = [("op", _int), ("side", _int), ("uplo", _int), ("trans", _int), ("diag", _int), ("m", _i64),
                ("n", _i64), ("alpha", ctypes.c_double), ("precision", _int), ("factor_id", ctypes.c_uint64),
                ("rhs_id", ctypes.c_uint64), ("result", _vp), ("t_arrival", ctypes.c_double)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", _int), ("batched", _int), ("iters", _int),
                ("eta", ctypes.c_double), ("t_arrival", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class Counters(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("failed", _i64), ("launches", _i64),
                ("batched_launches", _i64), ("batched_requests", _i64), ("factor_hits", _i64),
                ("factor_misses", _i64), ("evictions", _i64), ("hbm_in_use", _i64), ("hbm_peak", _i64),
                ("useful_flops", ctypes.c_double), ("refine_turns", _i64)]


PREC_F64, PREC_MIXED_BF16, PREC_MIXED_F32 = 0, 1, 2
rtri_server_create = _sig("rtri_server_create", _int, ctypes.POINTER(ServerCfg), ctypes.POINTER(_vp))
rtri_server_register_factor = _sig("rtri_server_register_factor", _int, _vp, ctypes.c_uint64, _i64, _int, _vp, _i64)
rtri_server_submit = _sig("rtri_server_submit", _int, _vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64))
rtri_server_poll = _sig("rtri_server_poll", _int, _vp, ctypes.POINTER(Completion), _int, ctypes.POINTER(_int))
rtri_server_drain = _sig("rtri_server_drain", _int, _vp)
rtri_server_stats = _sig("rtri_server_stats", _int, _vp, ctypes.POINTER(Counters))
rtri_server_now = _sig("rtri_server_now", ctypes.c_double, _vp)
rtri_server_destroy = _sig("rtri_server_destroy", _int, _vp)
rtri_tune = _sig("rtri_tune", _int, _vp, _int, _i64, ctypes.c_char_p)
rtri_load_tuning = _sig("rtri_load_tuning", _int, _vp, ctypes.c_char_p)
rtri_query_leaf = _sig("rtri_query_leaf", _int, _vp, _int, _int, _i64, _i64, ctypes.POINTER(_int))
TUNING_DB = os.path.join(_HERE, "tuning", "gfx950.json")
rtri_gemm_update = _sig("rtri_gemm_update", _int, _vp, _int, _int, _int, _i64, _i64, _i64, ctypes.c_double, _vp,
                        _i64, _vp, _i64, ctypes.c_double, _vp, _i64)


class KernelStat(ctypes.Structure):
    _fields_ = [("kclass", _int), ("dtype", _int), ("launches", _i64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


KCLASS_NAMES = {0: "gemm", 1: "leaf_solve", 2: "leaf_mult", 3: "other", 4: "batched"}
DTYPE_NAMES = {0: "f64", 1: "f32", 2: "bf16", 3: "f16", 4: "i8"}
rtri_profile_begin = _sig("rtri_profile_begin", _int, _vp)
rtri_profile_end = _sig("rtri_profile_end", _int, _vp, ctypes.POINTER(KernelStat), _int, ctypes.POINTER(_int))


class RtriError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = rtri_status_string(code).decode()
        super().__init__(f"{what}: rtri status {code} ({msg})" if what else f"rtri status {code} ({msg})")
        self.code = code


def check(code: int, what: str = "") -> int:
    if code != OK:
        raise RtriError(code, what)
    return code


_SIDE = {"L": LEFT, "R": RIGHT}
_UPLO = {"L": LOWER, "U": UPPER}
_TRANS = {"N": NOTRANS, "T": TRANS, "C": CONJTRANS}
_DIAG = {"N": NONUNIT, "U": UNIT}


def codes(side: str, uplo: str, trans: str, diag: str):
    """BLAS letters -> C ABI codes; an unknown letter maps to -1, which the
    library rejects with the argument's error code."""
    return (_SIDE.get(side.upper(), -1), _UPLO.get(uplo.upper(), -1), _TRANS.get(trans.upper(), -1),
            _DIAG.get(diag.upper(), -1))


class Handle:
    """An rtri handle bound to a torch CUDA/HIP stream (default: the current one)."""

    def __init__(self, stream=None):
        if torch is not None and stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        self.stream = stream
        raw = getattr(stream, "cuda_stream", stream) if stream is not None else None
        h = _vp()
        check(rtri_create(ctypes.byref(h), _vp(raw) if raw else None), "rtri_create")
        self._h = h

    @property
    def ptr(self):
        return self._h

    def set_option(self, option: int, value: int):
        check(rtri_set_option(self._h, option, value), "rtri_set_option")

    def get_option(self, option: int) -> int:
        v = _i64()
        check(rtri_get_option(self._h, option, ctypes.byref(v)), "rtri_get_option")
        return v.value

    def sync(self):
        check(rtri_sync(self._h), "rtri_sync")

    def tune(self, dtype="f64", max_order=16384, db_path=None):
        """Run the tuning sweep (blocking) and keep its rules; optionally write them as JSON."""
        check(rtri_tune(self._h, {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}[dtype], max_order,
                        db_path.encode() if db_path else None), "rtri_tune")

    def load_tuning(self, path=TUNING_DB):
        check(rtri_load_tuning(self._h, path.encode()), "rtri_load_tuning")

    def leaf(self, dtype="f64", op="trsm", order=1, nvec=1) -> int:
        """The leaf size this handle would use for such a problem."""
        v = _int()
        check(rtri_query_leaf(self._h, {"f64": F64, "f32": F32}[dtype], {"trsm": 0, "trmm": 1}[op], order, nvec,
                              ctypes.byref(v)), "rtri_query_leaf")
        return v.value

    def profile_begin(self):
        check(rtri_profile_begin(self._h), "rtri_profile_begin")

    def profile_end(self) -> list:
        """Per kernel class: dicts with launches, ms, flops, bytes (waits for the stream)."""
        buf = (KernelStat * 16)()
        n = _int()
        check(rtri_profile_end(self._h, buf, 16, ctypes.byref(n)), "rtri_profile_end")
        return [dict(kclass=KCLASS_NAMES[b.kclass], dtype=DTYPE_NAMES[b.dtype], launches=b.launches, ms=b.ms,
                     flops=b.flops, bytes=b.bytes) for b in buf[:n.value]]

    def close(self):
        if self._h:
            rtri_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _colmajor(t, name):
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.shape[0] > 1 and t.stride(0) != 1:
        raise ValueError(f"{name} must be a column-major view (stride(0) == 1)")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    return max(1, t.stride(1) if t.shape[1] > 1 else t.shape[0])


def _need_shape(t, name, rows, cols):
    """Reject a tensor smaller than the rows x cols the call will read or write
    (the C ABI sees only pointers and leading dimensions, so an undersized
    tensor would be read past its end)."""
    if t.dim() != 2 or t.shape[0] < rows or t.shape[1] < cols:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, needs at least ({rows}, {cols})")


def _same_device(**ts):
    devs = {str(t.device) for t in ts.values()}
    if len(devs) > 1:
        raise ValueError("tensors on different devices: " + ", ".join(f"{k} on {t.device}" for k, t in ts.items()))


def _factor_order(side, B):
    return B.shape[0] if str(side).upper() == "L" else B.shape[1]


def _call(h: Handle, solve: bool, side, uplo, trans, diag, alpha, A, B):
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    m, n = B.shape
    ka = _factor_order(side, B)
    _need_shape(A, "A", ka, ka)
    _same_device(A=A, B=B)
    lda = _colmajor(A, "A")
    ldb = _colmajor(B, "B")
    if A.dtype != B.dtype:
        raise TypeError("A and B must have the same dtype")
    if B.dtype == torch.float64:
        fn = rtri_dtrsm if solve else rtri_dtrmm
    elif B.dtype == torch.float32:
        fn = rtri_strsm if solve else rtri_strmm
    else:
        raise TypeError(f"unsupported dtype {B.dtype}")
    rc = fn(h.ptr, *codes(side, uplo, trans, diag), m, n, alpha, A.data_ptr(), lda, B.data_ptr(), ldb)
    check(rc, fn.__name__)
    return B


def trsm(h: Handle, side, uplo, trans, diag, alpha, A, B):
    """In place: B := X with op(A) X = alpha B (side 'L') or X op(A) = alpha B (side 'R')."""
    return _call(h, True, side, uplo, trans, diag, alpha, A, B)


def trmm(h: Handle, side, uplo, trans, diag, alpha, A, B):
    """In place: B := alpha op(A) B (side 'L') or alpha B op(A) (side 'R')."""
    return _call(h, False, side, uplo, trans, diag, alpha, A, B)


def trsm_noalloc(h: Handle, side, uplo, trans, diag, alpha, A, B):
    """As trsm for FP64, through rtri_dtrsm_noalloc: no device memory is allocated by the call (its
    workspace is the library's fixed device array)."""
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    m, n = B.shape
    ka = _factor_order(side, B)
    _need_shape(A, "A", ka, ka)
    _same_device(A=A, B=B)
    lda = _colmajor(A, "A")
    ldb = _colmajor(B, "B")
    if A.dtype != torch.float64 or B.dtype != torch.float64:
        raise TypeError("trsm_noalloc takes float64 A and B")
    rc = rtri_dtrsm_noalloc(h.ptr, *codes(side, uplo, trans, diag), m, n, alpha, A.data_ptr(), lda, B.data_ptr(),
                            ldb)
    check(rc, "rtri_dtrsm_noalloc")
    return B


class CallPlan:
    """One TRSM ('trsm') or TRMM ('trmm') on fixed tensors A and B (FP64 or FP32), planned once and
    captured in a HIP graph; run() replays it on the handle's stream (rtri_call_plan_*)."""

    def __init__(self, h: Handle, op, side, uplo, trans, diag, alpha, A, B):
        if B.dim() != 2:
            raise ValueError("B must be 2-D")
        m, n = B.shape
        ka = _factor_order(side, B)
        _need_shape(A, "A", ka, ka)
        _same_device(A=A, B=B)
        lda, ldb = _colmajor(A, "A"), _colmajor(B, "B")
        if A.dtype != B.dtype:
            raise TypeError("A and B must have the same dtype")
        dt = {torch.float64: F64, torch.float32: F32}.get(B.dtype)
        if dt is None:
            raise TypeError(f"unsupported dtype {B.dtype}")
        p = _vp()
        check(rtri_call_plan_create(h.ptr, {"trsm": 0, "trmm": 1}[op], dt, *codes(side, uplo, trans, diag), m, n,
                                    alpha, A.data_ptr(), lda, B.data_ptr(), ldb, ctypes.byref(p)),
              "rtri_call_plan_create")
        self._p = p
        self._keep = (A, B)

    def run(self):
        check(rtri_call_plan_run(self._p), "rtri_call_plan_run")

    def close(self):
        if self._p:
            rtri_call_plan_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trmm_ozaki(h: Handle, side, uplo, trans, diag, alpha, A, B):
    """As trmm for FP64, through rtri_dtrmm_ozaki: the product from exact INT8 matrix-core products
    (modular Ozaki scheme), FP64-accurate."""
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    m, n = B.shape
    ka = _factor_order(side, B)
    _need_shape(A, "A", ka, ka)
    _same_device(A=A, B=B)
    lda = _colmajor(A, "A")
    ldb = _colmajor(B, "B")
    if A.dtype != torch.float64 or B.dtype != torch.float64:
        raise TypeError("trmm_ozaki takes float64 A and B")
    rc = rtri_dtrmm_ozaki(h.ptr, *codes(side, uplo, trans, diag), m, n, alpha, A.data_ptr(), lda, B.data_ptr(), ldb)
    check(rc, "rtri_dtrmm_ozaki")
    return B


def gemm_update(h: Handle, trans_p: str, trans_q: str, s, P, Q, beta, C):
    """In place: C := beta C + s op(P) op(Q) (the recursion's GEMM update on its own)."""
    tp, tq = _TRANS[trans_p.upper()], _TRANS[trans_q.upper()]
    if C.dim() != 2 or P.dim() != 2:
        raise ValueError("P, Q and C must be 2-D")
    M, N = C.shape
    K = P.shape[0] if tp else P.shape[1]
    _need_shape(P, "P", K if tp else M, M if tp else K)
    _need_shape(Q, "Q", N if tq else K, K if tq else N)
    _same_device(P=P, Q=Q, C=C)
    ldp, ldq, ldc = _colmajor(P, "P"), _colmajor(Q, "Q"), _colmajor(C, "C")
    if P.dtype in (torch.bfloat16, torch.float16):
        # 16-bit P and Q, FP32 C (FP32 accumulation)
        if Q.dtype != P.dtype or C.dtype != torch.float32:
            raise TypeError("16-bit P needs Q of the same type and a float32 C")
        dt = BF16 if P.dtype == torch.bfloat16 else F16
    else:
        if not (P.dtype == Q.dtype == C.dtype):
            raise TypeError("P, Q and C must have the same dtype")
        dt = {torch.float64: F64, torch.float32: F32}[C.dtype]
    check(rtri_gemm_update(h.ptr, dt, tp, tq, M, N, K, s, P.data_ptr(), ldp, Q.data_ptr(), ldq, beta,
                           C.data_ptr(), ldc), "rtri_gemm_update")
    return C


def trmm_ex(h: Handle, side, uplo, trans, diag, alpha, A, B, C):
    """Out of place: C := alpha op(A) B (side 'L') or alpha B op(A) (side 'R'); A, B bfloat16 or float16
    (same type), C float32; FP32 accumulation."""
    if C.dim() != 2:
        raise ValueError("C must be 2-D")
    m, n = C.shape
    ka = _factor_order(side, C)
    _need_shape(A, "A", ka, ka)
    _need_shape(B, "B", m, n)
    _same_device(A=A, B=B, C=C)
    lda, ldb, ldc = _colmajor(A, "A"), _colmajor(B, "B"), _colmajor(C, "C")
    t = {torch.bfloat16: BF16, torch.float16: F16}[A.dtype]
    tb = {torch.bfloat16: BF16, torch.float16: F16}[B.dtype]
    if C.dtype != torch.float32:
        raise TypeError("C must be float32")
    check(rtri_trmm_ex(h.ptr, *codes(side, uplo, trans, diag), m, n, alpha, A.data_ptr(), t, lda, B.data_ptr(), tb,
                       ldb, C.data_ptr(), F32, ldc), "rtri_trmm_ex")
    return C


def trsm_mixed(h: Handle, side, uplo, trans, diag, alpha, A, B, gemm="bf16", tol=1e-12, max_iter=20,
               allow_not_converged=False):
    """In place, FP64: B := X with op(A) X = alpha B (or X op(A) = alpha B) by iterative refinement
    around a low-precision recursive solve (GEMM updates in 'bf16' or 'f32').  Returns the refinement
    record as a dict."""
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    m, n = B.shape
    ka = _factor_order(side, B)
    _need_shape(A, "A", ka, ka)
    _same_device(A=A, B=B)
    lda, ldb = _colmajor(A, "A"), _colmajor(B, "B")
    if A.dtype != torch.float64 or B.dtype != torch.float64:
        raise TypeError("A and B must be float64")
    info = RefineInfo()
    rc = rtri_dtrsm_mixed(h.ptr, *codes(side, uplo, trans, diag), m, n, alpha, A.data_ptr(), lda, B.data_ptr(),
                          ldb, {"bf16": BF16, "f32": F32}[gemm], tol, max_iter, ctypes.byref(info))
    if not (rc == OK or (allow_not_converged and rc == NOT_CONVERGED)):
        check(rc, "rtri_dtrsm_mixed")
    return dict(status=rc, iters=info.iters, converged=bool(info.converged), eta=info.eta, anorm=info.anorm,
                eta_hist=list(info.eta_hist[:info.iters]))


def ztrsm(h: Handle, side, uplo, trans, diag, alpha, A, B):
    """Complex (complex128) in place: B := X with op(A) X = alpha B or X op(A) = alpha B; trans 'C' is
    conj(A^T)."""
    return _zcall(h, True, side, uplo, trans, diag, alpha, A, B)


def ztrmm(h: Handle, side, uplo, trans, diag, alpha, A, B):
    """Complex (complex128) in place: B := alpha op(A) B or alpha B op(A)."""
    return _zcall(h, False, side, uplo, trans, diag, alpha, A, B)


def _zcall(h, solve, side, uplo, trans, diag, alpha, A, B):
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    m, n = B.shape
    ka = _factor_order(side, B)
    _need_shape(A, "A", ka, ka)
    _same_device(A=A, B=B)
    lda, ldb = _colmajor(A, "A"), _colmajor(B, "B")
    if A.dtype != torch.complex128 or B.dtype != torch.complex128:
        raise TypeError("A and B must be complex128")
    a = complex(alpha)
    al = _c2(a.real, a.imag)
    fn = rtri_ztrsm if solve else rtri_ztrmm
    check(fn(h.ptr, *codes(side, uplo, trans, diag), m, n, al, A.data_ptr(), lda, B.data_ptr(), ldb), fn.__name__)
    return B


def trtri(h: Handle, uplo, diag, A):
    """In place: the triangle of A named by uplo (and its diagonal unless diag='U') becomes that
    triangle of inv(A)."""
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError(f"A must be square, got {tuple(A.shape)}")
    lda = _colmajor(A, "A")
    fn = {torch.float64: rtri_dtrtri, torch.float32: rtri_strtri}.get(A.dtype)
    if fn is None:
        raise TypeError(f"unsupported dtype {A.dtype}")
    check(fn(h.ptr, _UPLO.get(uplo.upper(), -1), _DIAG.get(diag.upper(), -1), A.shape[0], A.data_ptr(), lda),
          fn.__name__)
    return A


def potrs(h: Handle, uplo, A, B):
    """In place: B := X with (L L^T) X = B (uplo 'L') or (U^T U) X = B (uplo 'U'), the factor in A."""
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    n, nrhs = B.shape
    _need_shape(A, "A", n, n)
    _same_device(A=A, B=B)
    lda, ldb = _colmajor(A, "A"), _colmajor(B, "B")
    if A.dtype != B.dtype:
        raise TypeError("A and B must have the same dtype")
    fn = {torch.float64: rtri_dpotrs, torch.float32: rtri_spotrs}.get(B.dtype)
    if fn is None:
        raise TypeError(f"unsupported dtype {B.dtype}")
    check(fn(h.ptr, _UPLO.get(uplo.upper(), -1), n, nrhs, A.data_ptr(), lda, B.data_ptr(), ldb), fn.__name__)
    return B


def getrs(h: Handle, trans, LU, ipiv, B):
    """In place: B := X with S X = B (trans 'N') or S^T X = B (trans 'T') for P S = L U packed in LU;
    ipiv: LAPACK's 1-based interchange sequence (host integers)."""
    import numpy as np
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    n, nrhs = B.shape
    _need_shape(LU, "LU", n, n)
    _same_device(LU=LU, B=B)
    lda, ldb = _colmajor(LU, "LU"), _colmajor(B, "B")
    if LU.dtype != B.dtype:
        raise TypeError("LU and B must have the same dtype")
    piv = np.ascontiguousarray(np.asarray(ipiv), dtype=np.int32)
    if piv.shape != (n,):
        raise ValueError(f"ipiv must have {n} entries")
    fn = {torch.float64: rtri_dgetrs, torch.float32: rtri_sgetrs}.get(B.dtype)
    if fn is None:
        raise TypeError(f"unsupported dtype {B.dtype}")
    check(fn(h.ptr, _TRANS.get(trans.upper(), -1), n, nrhs, LU.data_ptr(), lda, piv.ctypes.data, B.data_ptr(), ldb),
          fn.__name__)
    return B


_PREC = {"f64": 0, "mixed_bf16": 1, "mixed_f32": 2}


class Factor:
    """A triangular factor kept for repeated solves and multiplies (see
    rtri_factor_*): packed diagonal blocks, and for refined solves the GEMM-type
    copy of A and |op(A)|, are made on first use and kept on the device.
    Without copy=True the tensor A must stay unchanged while the factor lives
    (the factor keeps a reference to it)."""

    def __init__(self, h: Handle, uplo, diag, A, copy=False):
        if A.dim() != 2 or A.shape[0] != A.shape[1]:
            raise ValueError(f"A must be square, got {tuple(A.shape)}")
        lda = _colmajor(A, "A")
        dt = {torch.float64: F64, torch.float32: F32}.get(A.dtype)
        if dt is None:
            raise TypeError(f"unsupported dtype {A.dtype}")
        self.dtype = A.dtype
        self.order = A.shape[0]
        u, d = _UPLO.get(uplo.upper(), -1), _DIAG.get(diag.upper(), -1)
        p = _vp()
        check(rtri_factor_create(h.ptr, u, d, self.order, dt, A.data_ptr(), lda, FACTOR_COPY if copy else 0,
                                 ctypes.byref(p)), "rtri_factor_create")
        self._f = p
        self._A = None if copy else A

    @property
    def ptr(self):
        return self._f

    def _b(self, side, B):
        if B.dim() != 2:
            raise ValueError("B must be 2-D")
        if B.dtype != self.dtype:
            raise TypeError("B must have the factor's dtype")
        ka = _factor_order(side, B)
        if ka != self.order:
            raise ValueError(f"B has shape {tuple(B.shape)}: side {side} needs order {self.order}")
        return _colmajor(B, "B")

    def trsm(self, h: Handle, side, trans, alpha, B, precision="f64", tol=1e-12, max_iter=30,
             allow_not_converged=False):
        """In place: B := X with op(A) X = alpha B (or X op(A) = alpha B); precision 'f64' (the factor's
        own type), 'mixed_bf16' or 'mixed_f32' (refined to tol, FP64 factors).  Returns the refinement
        record as a dict."""
        ldb = self._b(side, B)
        m, n = B.shape
        info = RefineInfo()
        rc = rtri_factor_trsm(h.ptr, self._f, _SIDE.get(side.upper(), -1), _TRANS.get(trans.upper(), -1), m, n, alpha,
                              B.data_ptr(), ldb, _PREC[precision], tol, max_iter, ctypes.byref(info))
        if not (rc == OK or (allow_not_converged and rc == NOT_CONVERGED)):
            check(rc, "rtri_factor_trsm")
        return dict(status=rc, iters=info.iters, converged=bool(info.converged), eta=info.eta, anorm=info.anorm,
                    eta_hist=list(info.eta_hist[:info.iters]))

    def trmm(self, h: Handle, side, trans, alpha, B):
        """In place: B := alpha op(A) B (or alpha B op(A))."""
        ldb = self._b(side, B)
        m, n = B.shape
        check(rtri_factor_trmm(h.ptr, self._f, _SIDE.get(side.upper(), -1), _TRANS.get(trans.upper(), -1), m, n,
                               alpha, B.data_ptr(), ldb), "rtri_factor_trmm")
        return B

    def bytes(self) -> int:
        v = _i64()
        check(rtri_factor_bytes(self._f, ctypes.byref(v)), "rtri_factor_bytes")
        return v.value

    def close(self):
        if self._f:
            rtri_factor_destroy(self._f)
            self._f = _vp()
            self._A = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_entries(problems):
    """problems: iterable of (op 'trsm'|'trmm', side, uplo, trans, diag, alpha, A, B) with column-major
    device tensors of one dtype.  Returns (ctypes array of BatchEntry, dtype code)."""
    problems = list(problems)
    arr = (BatchEntry * max(1, len(problems)))()
    dt = None
    for i, (op, side, uplo, trans, diag, alpha, A, B) in enumerate(problems):
        if B.dim() != 2:
            raise ValueError(f"problem {i}: B must be 2-D")
        ka = _factor_order(side, B)
        _need_shape(A, f"problem {i}: A", ka, ka)
        _same_device(A=A, B=B)
        lda, ldb = _colmajor(A, "A"), _colmajor(B, "B")
        d = {torch.float64: F64, torch.float32: F32}[B.dtype]
        if dt is None:
            dt = d
        elif d != dt or A.dtype != B.dtype:
            raise TypeError("one dtype per batch")
        s, u, t, g = codes(side, uplo, trans, diag)
        arr[i] = BatchEntry({"trsm": 0, "trmm": 1}[op], s, u, t, g, B.shape[0], B.shape[1], alpha, A.data_ptr(), lda,
                            B.data_ptr(), ldb)
    return arr, (dt if dt is not None else F64), len(problems)


class BatchPlan:
    """A reusable batch plan (graph-captured persistent launch)."""

    def __init__(self, h: Handle, problems):
        self.h = h
        arr, dt, n = batch_entries(problems)
        self._arr = arr
        p = _vp()
        bad = _int(-1)
        rc = rtri_batch_plan_create(h.ptr, dt, n, arr, ctypes.byref(p), ctypes.byref(bad))
        if rc != OK:
            raise RtriError(rc, f"rtri_batch_plan_create (entry {bad.value})")
        self._p = p

    def run(self):
        check(rtri_batch_plan_run(self._p), "rtri_batch_plan_run")

    def chunks(self) -> int:
        c = _i64()
        check(rtri_batch_plan_chunks(self._p, ctypes.byref(c)), "rtri_batch_plan_chunks")
        return c.value

    def close(self):
        if self._p:
            rtri_batch_plan_destroy(self._p)
            self._p = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batched(h: Handle, problems):
    """One-shot batch (blocking)."""
    arr, dt, n = batch_entries(problems)
    bad = _int(-1)
    rc = rtri_batched(h.ptr, dt, n, arr, ctypes.byref(bad))
    if rc != OK:
        raise RtriError(rc, f"rtri_batched (entry {bad.value})")


def synth_fill(h: Handle, kind: int, seed: int, stream: int, ident: int, X, param: float = 0.0):
    """On-device Philox4x32-10 fill of a column-major tensor (see rtri_synth_fill)."""
    ldx = _colmajor(X, "X")
    dt = {torch.float64: F64, torch.float32: F32}[X.dtype]
    check(rtri_synth_fill(h.ptr, dt, kind, seed, stream, ident, X.shape[0], X.shape[1], param, X.data_ptr(), ldx),
          "rtri_synth_fill")
    return X


class Server:
    """Continuous-batching server (see rtri_server_*).  Requests are dicts with
    the rtri_request fields; 'result' may be a float64 numpy array (m x n,
    Fortran order) that receives the result."""

    def __init__(self, slots=4, hbm_budget=64 << 30, max_batch=256, small_max=1024, seed=250413821,
                 refine_requeue=False, mixed_batch=False):
        cfg = ServerCfg(slots, hbm_budget, max_batch, small_max, seed, 1 if refine_requeue else 0,
                        1 if mixed_batch else 0)
        p = _vp()
        check(rtri_server_create(ctypes.byref(cfg), ctypes.byref(p)), "rtri_server_create")
        self._s = p
        self._keep = {}

    def now(self) -> float:
        return rtri_server_now(self._s)

    def submit(self, op="trsm", side="L", uplo="L", trans="N", diag="N", m=1, n=1, alpha=1.0, precision=PREC_F64,
               factor_id=1, rhs_id=1, result=None, t_arrival=0.0) -> int:
        s, u, t, d = codes(side, uplo, trans, diag)
        ptr = None
        if result is not None:
            if result.dtype.name != "float64" or not result.flags["F_CONTIGUOUS"] or result.shape != (m, n):
                raise ValueError("result must be a Fortran-ordered float64 m x n array")
            ptr = result.ctypes.data
        req = Request({"trsm": 0, "trmm": 1}[op], s, u, t, d, m, n, alpha, precision, factor_id, rhs_id, ptr,
                      t_arrival)
        tk = ctypes.c_uint64()
        check(rtri_server_submit(self._s, ctypes.byref(req), ctypes.byref(tk)), "rtri_server_submit")
        if result is not None:
            self._keep[tk.value] = result
        return tk.value

    def poll(self, max_n=4096) -> list:
        buf = (Completion * max_n)()
        n = _int()
        check(rtri_server_poll(self._s, buf, max_n, ctypes.byref(n)), "rtri_server_poll")
        out = []
        for c in buf[:n.value]:
            self._keep.pop(c.ticket, None)
            out.append(dict(ticket=c.ticket, status=c.status, batched=bool(c.batched), iters=c.iters, eta=c.eta,
                            t_arrival=c.t_arrival, t_start=c.t_start, t_done=c.t_done))
        return out

    def drain(self):
        check(rtri_server_drain(self._s), "rtri_server_drain")

    def stats(self) -> dict:
        c = Counters()
        check(rtri_server_stats(self._s, ctypes.byref(c)), "rtri_server_stats")
        return {f: getattr(c, f) for f, _ in Counters._fields_}

    def close(self):
        if self._s:
            rtri_server_destroy(self._s)
            self._s = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_device(a, dtype=None, device="cuda", ld=None):
    """numpy (any order) -> column-major device tensor of shape (m, n); optional padded leading dimension."""
    import numpy as np
    a = np.asarray(a)
    m, n = a.shape
    ld = m if ld is None else ld
    dt = dtype if dtype is not None else {np.dtype("float64"): torch.float64, np.dtype("float32"): torch.float32,
                                          np.dtype("complex128"): torch.complex128}[a.dtype]
    store = torch.zeros((n, ld), dtype=dt, device=device)
    # narrower types are rounded by torch (round to nearest even)
    store[:, :m] = torch.from_numpy(np.ascontiguousarray(a.T)).to(device=device).to(dtype=dt)
    return store.t()[:m, :]


def to_host(t):
    """column-major device tensor -> numpy Fortran-order array (16-bit types widened to float32)."""
    x = t.t().contiguous()
    if x.dtype in (torch.bfloat16, torch.float16):
        x = x.float()
    return x.cpu().numpy().T
