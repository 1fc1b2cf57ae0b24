"""Benchmark of the recursive TRSM / TRMM path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--m 16384] [--no-cpu]

Workload (one "step"): FP64 TRSM then FP64 TRMM, side = L, uplo = L, trans = N,
diag = N, m = n = 16384, alpha = 1, in place on one B.  A is lower-triangular
with off-diagonal entries U(-1,1) and diagonal entries m + U(0,1); B is U(-1,1);
column-major, seeded (Philox4x32-10).  TRSM followed by TRMM on the same A is a
round trip, so every timed step sees data of the same scale.  Inputs are
resident in HBM before the timed region starts.

Printed: one JSON line.  value = useful TFLOP/s of the step (m^2 n flops per
operation, the BLAS convention); roofline = the FP64 GEMM-update kernel class,
from per-launch HIP events recorded by the library on its own stream in a second
pass of the same steps; cpu_baseline = the CPU oracle on a sample of columns.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0, "i8": 5000.0}   # MI355X dense MFMA, TFLOP/s (TOP/s for i8)
HBM_PEAK = 8000.0                                                    # GB/s

# HBM-side bytes per FP64 GEMM-update launch of this step, from two rocprofv3
# PMC passes (FETCH_SIZE x 2 + WRITE_SIZE x 1, factors from a 2 GiB copy in the
# same process; profiles/gemm_f64_16384_traffic.txt).  Valid only for the GEMM
# sources they were taken on: reported as null once those change.
GEMM_TRAFFIC = {"bytes_per_launch": 1.0394e9, "sources_sha256_16": "6ee4c57ad51e1707"}


def gemm_sources_digest():
    import hashlib
    d = hashlib.sha256()
    for f in ("gemm.hip", "gemm_core.h"):
        with open(os.path.join(ROOT, "paper_2504_13821_amd", "csrc", f), "rb") as fh:
            d.update(fh.read())
    return d.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=16384)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--leaf", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true", help="only the headline step")
    ap.add_argument("--extras", default="mixed,rect256,solvers,small,trmm16,batched,serving",
                    help="comma-separated extra sections to run (default: all but 'vendor', the rocBLAS "
                         "comparison, and 'residual', the residual product alone, which run only when named)")
    ap.add_argument("--serve-requests", type=int, default=5000)
    ap.add_argument("--serve-rates", default="0.1,0.25,0.5,0.75,0.9,1.0,1.2",
                    help="open-loop arrival rates as fractions of the measured saturation throughput")
    ap.add_argument("--tuning", default="", help="tuning database (default: the package's, if present)")
    return ap.parse_args()


def progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library runs each problem on a single MI355X "
              "(how the path would shard over several GPUs is described in the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2504_13821_amd as rt
    import synth

    m = n = args.m
    g = synth.rng(synth.W_SWEEP, m, 0)
    A = synth.tri(m, "L", g, "base", fill=0.0)
    B0 = synth.dense(m, n, g)
    Ad = rt.to_device(A, torch.float64)
    B0d = rt.to_device(B0, torch.float64)
    Bd = rt.to_device(B0, torch.float64)
    h = rt.Handle()
    tuning = args.tuning or (rt.TUNING_DB if os.path.exists(rt.TUNING_DB) else "")
    if tuning:
        h.load_tuning(tuning)
    if args.leaf:
        h.set_option(rt.OPT_LEAF_F64, args.leaf)

    progress("inputs resident", m, n)

    def step():
        rt.trsm(h, "L", "L", "N", "N", 1.0, Ad, Bd)
        rt.trmm(h, "L", "L", "N", "N", 1.0, Ad, Bd)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    progress("timed steps done", round(ms_step, 3), "ms/step")
    flops_step = 2.0 * m * m * n
    value = flops_step / (ms_step * 1e-3) / 1e12

    # each operation alone (event-timed, B restored outside the timed call)
    def time_op(fn, reps=3):
        ts = []
        for _ in range(reps):
            Bd.copy_(B0d)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn(h, "L", "L", "N", "N", 1.0, Ad, Bd)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return min(ts)
    t_trsm = time_op(rt.trsm)
    t_trmm = time_op(rt.trmm)

    # second pass of the same steps with per-launch events: the dominant kernel
    h.profile_begin()
    for _ in range(args.steps):
        step()
    stats = h.profile_end()
    by = {(s["kclass"], s["dtype"]): s for s in stats}
    gem = by[("gemm", "f64")]
    gemm_avg_ms = gem["ms"] / gem["launches"]
    traffic = GEMM_TRAFFIC["bytes_per_launch"] if gemm_sources_digest() == GEMM_TRAFFIC["sources_sha256_16"] else None
    achieved = gem["flops"] / (gem["ms"] * 1e-3) / 1e12
    prof_total_ms = sum(s["ms"] for s in stats) / args.steps
    kernels = {f"{s['kclass']}_{s['dtype']}": {"launches_per_step": s["launches"] / args.steps,
                                               "ms_per_step": round(s["ms"] / args.steps, 4),
                                               "tflops": round(s["flops"] / max(s["ms"], 1e-9) / 1e9, 2)}
               for s in stats}

    out = {
        "metric": "TRSM/TRMM TFLOP/s at m=n=16384 (FP64 vs mixed+IR); served solves/s, p99 latency",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 TRSM + TRMM, side=L uplo=L trans=N diag=N, m=n={m}, alpha=1, "
                               "A: off-diagonal U(-1,1), diagonal m+U(0,1); B: U(-1,1)",
                   "m": m, "n": n, "leaf": {"trsm": h.leaf("f64", "trsm", m, n), "trmm": h.leaf("f64", "trmm", m, n)}},
        "trsm_ms": round(t_trsm, 3), "trsm_tflops": round(m * m * n / (t_trsm * 1e-3) / 1e12, 3),
        "trmm_ms": round(t_trmm, 3), "trmm_tflops": round(m * m * n / (t_trmm * 1e-3) / 1e12, 3),
        "fraction_of_fp64_peak": round(value / PEAK["f64"], 4),
        "roofline": {
            "kernel": "gemm_kernel<double> (GEMM update, all launches of a step)",
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": PEAK["f64"],
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK["f64"], 4),
            "traffic": traffic,
            "traffic_unit": "bytes per launch (HBM side, PMC)",
            "algorithmic_bytes_per_launch": round(gem["bytes"] / gem["launches"]),
            "algorithmic_flops_per_launch": round(gem["flops"] / gem["launches"]),
            "avg_launch_ms": round(gemm_avg_ms, 5),
            "launches_per_step": gem["launches"] / args.steps,
        },
        "kernels": kernels,
        "profiled_kernel_ms_per_step": round(prof_total_ms, 3),
    }

    out["tuning_db"] = os.path.basename(tuning) if tuning else None
    if not args.no_cpu:
        out["cpu_baseline"], out["eta_sampled"] = cpu_baseline(rt, torch, h, A, B0, B0d, Ad, Bd, m, n)
        progress("cpu baseline done")
    del Ad, Bd, B0d
    torch.cuda.empty_cache()
    extras = set() if args.no_extras else set(x.strip() for x in args.extras.split(",") if x.strip())
    if "mixed" in extras:
        out["mixed"], sample_mx = bench_mixed(rt, torch, h)
        if not args.no_cpu:
            cpu_check_mixed(out["mixed"], sample_mx)
        del sample_mx
        progress("mixed done")
    if "rect256" in extras:
        out["rect256"], sample_r = bench_rect256(rt, torch, h)
        if not args.no_cpu:
            cpu_check_rect256(out["rect256"], sample_r)
        del sample_r
        progress("rect256 done")
    if "solvers" in extras:
        out["solvers"], sample_s = bench_solvers(rt, torch, h)
        if not args.no_cpu:
            cpu_check_solvers(out["solvers"], sample_s)
        del sample_s
        progress("solvers done")
    if "residual" in extras:   # the residual product alone (part of "mixed" too)
        import synth
        mm = 8192
        Ad = rt.synth_fill(h, 1, synth.SEED, synth.W_MIXED, 1, torch.empty((mm, mm), dtype=torch.float64,
                                                                           device="cuda").t(), param=45.0)
        B0 = rt.synth_fill(h, 0, synth.SEED, synth.W_MIXED, 2, torch.empty((mm, mm), dtype=torch.float64,
                                                                           device="cuda").t())
        out["residual_product"] = bench_residual_product(rt, torch, h, Ad, B0)
        del Ad, B0
        progress("residual done")
    if "small" in extras:
        out["small"] = bench_small(rt, torch, h)
        progress("small done")
    if "trmm16" in extras:
        out["trmm16"], sample16 = bench_trmm16(rt, torch, h)
        if not args.no_cpu:
            cpu_check_trmm16(out["trmm16"], sample16)
        del sample16
        progress("16-bit trmm done")
    if "batched" in extras:
        out["batched"] = bench_batched(rt, torch, h)
        progress("batched done")
    if "serving" in extras:
        out["serving"] = bench_serving(rt, args.serve_requests,
                                       [float(x) for x in args.serve_rates.split(",") if x.strip()])
        progress("serving done")
    if "vendor" in extras:
        out["vendor_context"] = bench_vendor(rt, torch, h, m)
        progress("vendor context done")
    print(json.dumps(out), flush=True)


def _event_ms(torch, fn, prep=None, reps=3):
    ts = []
    for _ in range(reps):
        if prep is not None:
            prep()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return min(ts)


class _RocBlas:
    """rocBLAS trsm / trmm through its C API (context only: the paper compares
    its recursive kernels against the vendor library on the same hardware)."""
    SIDE_L, FILL_L, OP_N, DIAG_N = 141, 122, 111, 131

    def __init__(self, torch):
        import ctypes
        self.ct = ctypes
        self.lib = ctypes.CDLL(os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "librocblas.so"))
        self.h = ctypes.c_void_p()
        self._ok(self.lib.rocblas_create_handle(ctypes.byref(self.h)), "create_handle")
        self._ok(self.lib.rocblas_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
                 "set_stream")

    def _ok(self, st, what):
        if st != 0:
            raise RuntimeError(f"rocblas_{what} returned {st}")

    def trsm(self, A, B):
        ct = self.ct
        f64 = A.dtype.itemsize == 8
        al = (ct.c_double if f64 else ct.c_float)(1.0)
        fn = self.lib.rocblas_dtrsm if f64 else self.lib.rocblas_strsm
        m, n = B.shape
        self._ok(fn(self.h, self.SIDE_L, self.FILL_L, self.OP_N, self.DIAG_N, ct.c_int(m), ct.c_int(n), ct.byref(al),
                    ct.c_void_p(A.data_ptr()), ct.c_int(A.stride(1)), ct.c_void_p(B.data_ptr()),
                    ct.c_int(B.stride(1))), "trsm")

    def trmm(self, A, B, C):
        ct = self.ct
        f64 = A.dtype.itemsize == 8
        al = (ct.c_double if f64 else ct.c_float)(1.0)
        fn = self.lib.rocblas_dtrmm if f64 else self.lib.rocblas_strmm
        m, n = B.shape
        self._ok(fn(self.h, self.SIDE_L, self.FILL_L, self.OP_N, self.DIAG_N, ct.c_int(m), ct.c_int(n), ct.byref(al),
                    ct.c_void_p(A.data_ptr()), ct.c_int(A.stride(1)), ct.c_void_p(B.data_ptr()),
                    ct.c_int(B.stride(1)), ct.c_void_p(C.data_ptr()), ct.c_int(C.stride(1))), "trmm")

    def close(self):
        self.lib.rocblas_destroy_handle(self.h)


def bench_vendor(rt, torch, h, m):
    """rocBLAS beside this library on the same device-drawn inputs, side=L
    uplo=L trans=N diag=N, alpha = 1: FP64 at m = n = 16384, and the paper's
    FP32 shapes (B m x 256 and m x m).  ratio = rocBLAS time / this library's time, the paper's
    convention (above 1: this library is faster).  Context, not a target."""
    import synth
    try:
        rb = _RocBlas(torch)
    except (OSError, RuntimeError) as e:
        return {"skipped": f"rocBLAS not usable: {e}"}
    res = {"library": "rocBLAS (ROCm install)", "convention": "ratio = rocBLAS time / this library's time"}
    try:
        A = torch.empty((m, m), dtype=torch.float64, device="cuda").t()
        B0 = torch.empty((m, m), dtype=torch.float64, device="cuda").t()
        rt.synth_fill(h, 1, synth.SEED, synth.W_SWEEP, 1, A, param=float(m))
        rt.synth_fill(h, 0, synth.SEED, synth.W_SWEEP, 2, B0)
        B = B0.clone()
        C = torch.empty_like(B0)
        o_s = _event_ms(torch, lambda: rt.trsm(h, "L", "L", "N", "N", 1.0, A, B), lambda: B.copy_(B0), reps=2)
        o_m = _event_ms(torch, lambda: rt.trmm(h, "L", "L", "N", "N", 1.0, A, B), lambda: B.copy_(B0), reps=2)
        v_s = _event_ms(torch, lambda: rb.trsm(A, B), lambda: B.copy_(B0), reps=2)
        v_m = _event_ms(torch, lambda: rb.trmm(A, B0, C), reps=2)
        fl = float(m) ** 3
        res["f64_square"] = {"m": m, "n": m,
                             "trsm": {"ours_ms": round(o_s, 3), "rocblas_ms": round(v_s, 3),
                                      "ours_tflops": round(fl / (o_s * 1e-3) / 1e12, 3),
                                      "rocblas_tflops": round(fl / (v_s * 1e-3) / 1e12, 3),
                                      "ratio": round(v_s / o_s, 3)},
                             "trmm": {"ours_ms": round(o_m, 3), "rocblas_ms": round(v_m, 3),
                                      "ours_tflops": round(fl / (o_m * 1e-3) / 1e12, 3),
                                      "rocblas_tflops": round(fl / (v_m * 1e-3) / 1e12, 3),
                                      "ratio": round(v_m / o_m, 3)}}
        del A, B0, B, C
        torch.cuda.empty_cache()
        rows = []
        for shape in ("rect256", "square"):
            for mm in (1024, 2048, 4096, 8192, 16384):
                n = 256 if shape == "rect256" else mm
                A = torch.empty((mm, mm), dtype=torch.float32, device="cuda").t()
                B0 = torch.empty((n, mm), dtype=torch.float32, device="cuda").t()
                rt.synth_fill(h, 1, synth.SEED, synth.W_SWEEP, 3, A, param=float(mm))
                rt.synth_fill(h, 0, synth.SEED, synth.W_SWEEP, 4, B0)
                B = B0.clone()
                C = torch.empty_like(B0)
                reps = 5 if mm * mm * n < 1e12 else 2
                o_s = _event_ms(torch, lambda: rt.trsm(h, "L", "L", "N", "N", 1.0, A, B), lambda: B.copy_(B0), reps)
                o_m = _event_ms(torch, lambda: rt.trmm(h, "L", "L", "N", "N", 1.0, A, B), lambda: B.copy_(B0), reps)
                v_s = _event_ms(torch, lambda: rb.trsm(A, B), lambda: B.copy_(B0), reps)
                v_m = _event_ms(torch, lambda: rb.trmm(A, B0, C), reps=reps)
                fl = mm * mm * n
                rows.append({"shape": shape, "m": mm, "n": n,
                             "trsm_ms": [round(o_s, 3), round(v_s, 3)], "trsm_ratio": round(v_s / o_s, 3),
                             "trsm_tflops": [round(fl / (o_s * 1e-3) / 1e12, 2), round(fl / (v_s * 1e-3) / 1e12, 2)],
                             "trmm_ms": [round(o_m, 3), round(v_m, 3)], "trmm_ratio": round(v_m / o_m, 3),
                             "trmm_tflops": [round(fl / (o_m * 1e-3) / 1e12, 2), round(fl / (v_m * 1e-3) / 1e12, 2)]})
                del A, B0, B, C
                torch.cuda.empty_cache()
        res["f32_paper_shapes"] = {"columns": "ms / tflops pairs are [this library, rocBLAS]", "rows": rows}
    finally:
        rb.close()
    return res


def mixed_cond_labels():
    """Diagonal offset c of the m = 8192 mixed-precision factors (diagonal
    c + U(0,1), off-diagonal U(-1,1), device Philox fill, id 1) -> 1-norm
    condition number, as computed by the CPU oracle on the bit-identical host
    twin (tests/golden/make_c3_cond.py writes the file)."""
    with open(os.path.join(ROOT, "tests", "golden", "c3_cond.json")) as f:
        return [(case["c"], case["cond1"]) for case in json.load(f)["cases"]]


def bench_mixed(rt, torch, h, m=8192, ns=8):
    """Mixed-precision refined TRSM against the plain FP64 TRSM on the same
    system: m = n = 8192, lower factor with off-diagonal U(-1,1) and diagonal
    c + U(0,1) for three condition classes, dense right-hand sides U(-1,1);
    plus the headline order m = n = 16384 on its own factor (diagonal
    m + U(0,1)).  Inputs drawn on the device (Philox).  Returns the timings
    and, for the CPU leg, sampled columns of every input and result."""
    import synth
    res = {"workload": f"FP64-accurate TRSM L/L/N/N m=n={m}, diagonal c+U(0,1), tol 1e-12; "
                       "and m=n=16384, diagonal m+U(0,1)", "cases": []}
    samples = []
    cases = [(m, c, kappa) for c, kappa in mixed_cond_labels()] + [(16384, 16384.0, None)]
    for mm, c, kappa in cases:
        Ad = torch.empty((mm, mm), dtype=torch.float64, device="cuda").t()
        B0 = torch.empty((mm, mm), dtype=torch.float64, device="cuda").t()
        w = synth.W_MIXED if mm == m else synth.W_SWEEP
        rt.synth_fill(h, 0, synth.SEED, w, 2, B0)
        rt.synth_fill(h, 1, synth.SEED, w, 1, Ad, param=c)
        Bd = B0.clone()
        idx = np.sort(synth.rng(synth.W_MIXED, 3, mm, int(c)).choice(mm, ns, replace=False))
        tidx = torch.as_tensor(idx, device="cuda")
        smp = {"m": mm, "c": c, "A": rt.to_host(Ad), "B": np.asfortranarray(B0[:, tidx].cpu().numpy())}
        t_plain = _event_ms(torch, lambda: rt.trsm(h, "L", "L", "N", "N", 1.0, Ad, Bd), lambda: Bd.copy_(B0))
        case = {"m": mm, "c": c, "cond1": kappa, "fp64_ms": round(t_plain, 3),
                "fp64_tflops": round(mm ** 3 / (t_plain * 1e-3) / 1e12, 3)}
        smp["fp64"] = np.asfortranarray(Bd[:, tidx].cpu().numpy())
        variants = [("bf16", 0), ("f32", 0), ("bf16", 1), ("f32", 1)] if mm == m else [("f32", 0), ("f32", 1)]
        for gemm, resid in variants:
            info = {}
            key = gemm if resid == 0 else f"{gemm}_int8res"

            def run():
                info.update(rt.trsm_mixed(h, "L", "L", "N", "N", 1.0, Ad, Bd, gemm=gemm, tol=1e-12, max_iter=30,
                                          allow_not_converged=True))
            h.set_option(rt.OPT_RESIDUAL, resid)
            t = _event_ms(torch, run, lambda: Bd.copy_(B0))
            h.set_option(rt.OPT_RESIDUAL, 0)
            case[key] = {"ms": round(t, 3), "speedup_vs_fp64": round(t_plain / t, 3), "iters": info["iters"],
                         "eta_library": info["eta"], "converged": info["converged"],
                         "residual_product": "INT8 (Ozaki scheme)" if resid else "FP64 MFMA",
                         "useful_tflops": round(mm ** 3 / (t * 1e-3) / 1e12, 3)}
            smp[key] = np.asfortranarray(Bd[:, tidx].cpu().numpy())
        if mm == m:
            case["residual_product"] = bench_residual_product(rt, torch, h, Ad, B0)
        res["cases"].append(case)
        samples.append(smp)
        del Ad, B0, Bd
        torch.cuda.empty_cache()
    return res, samples


def bench_residual_product(rt, torch, h, Ad, B0):
    """The refined solve's residual product op(A) X on its own (FP64 accuracy
    both ways): the FP64 recursive TRMM against the INT8-product TRMM (modular
    Ozaki scheme), with the latter's per-class kernel profile; the INT8 GEMM
    class is reported against the dense INT8 MFMA peak (ops = 2 m n K per
    modulus, K over the triangle's half: m^2 n per modulus)."""
    mm = Ad.shape[0]
    W = B0.clone()
    out = {"m": mm, "n": B0.shape[1]}
    for name, fn in (("fp64_trmm", rt.trmm), ("int8_trmm", rt.trmm_ozaki)):
        t = _event_ms(torch, lambda: fn(h, "L", "L", "N", "N", 1.0, Ad, W), lambda: W.copy_(B0))
        out[name + "_ms"] = round(t, 3)
    W.copy_(B0)
    h.profile_begin()
    rt.trmm_ozaki(h, "L", "L", "N", "N", 1.0, Ad, W)
    prof = h.profile_end()
    out["int8_kernels"] = {f"{x['kclass']}_{x['dtype']}": {"launches": x["launches"], "ms": round(x["ms"], 4)}
                           for x in prof}
    g = [x for x in prof if x["kclass"] == "gemm" and x["dtype"] == "i8"]
    if g:
        tops = g[0]["flops"] / (g[0]["ms"] * 1e-3) / 1e12
        out["int8_gemm"] = {"bound": "mfma", "achieved": round(tops, 1), "peak": PEAK["i8"], "unit": "TOP/s",
                            "frac": round(tops / PEAK["i8"], 4), "moduli": int(round(g[0]["flops"] / (mm ** 2 * W.shape[1])))}
    del W
    return out


def cpu_check_mixed(res, samples):
    """CPU leg: every refined solve (and the plain FP64 solve beside it) on its
    sampled columns against the oracle: the compensated backward error and the
    forward error relative to the oracle's own solution."""
    import oracle
    for case, smp in zip(res["cases"], samples):
        Xo = oracle.trsm("L", "L", "N", "N", 1.0, smp["A"], smp["B"])
        for key in ("fp64", "bf16", "f32", "bf16_int8res", "f32_int8res"):
            if key not in smp:
                continue
            X = smp[key]
            err = {"columns": int(X.shape[1]),
                   "eta_oracle": oracle.trsm_eta("L", "L", "N", "N", 1.0, smp["A"], smp["B"], X),
                   "forward_error": float(np.max(np.abs(X - Xo)) / np.max(np.abs(Xo)))}
            if key == "fp64":
                case["fp64_error_vs_oracle"] = err
            else:
                case[key]["error_vs_oracle"] = err


def bench_rect256(rt, torch, h, ns=16):
    """The paper's narrow workload (its Sec. 4.1-4.2 rectangular case): FP32
    TRSM and TRMM, side L, lower, no transpose, non-unit, alpha = 1, A m x m
    (off-diagonal U(-1,1), diagonal m + U(0,1)), B m x 256 U(-1,1), for
    m = 1024 ... 16384, the shipped tuning rules loaded.  Per m: event-timed
    call (median of 5, B restored outside the timed region), TFLOP/s at
    m^2 * 256 flops, and the per-class kernel profile of one more call (the
    GEMM-update class is the roofline kernel: MFMA-bound, FP32 peak).  Returns
    the timings and, for the CPU leg, sampled columns of inputs and results."""
    import synth
    res = {"workload": "FP32 TRSM / TRMM L/L/N/N, A m x m (diagonal m+U(0,1)), B m x 256, alpha 1", "rows": []}
    samples = []
    for mm in (1024, 2048, 4096, 8192, 16384):
        n = 256
        Ad = torch.empty((mm, mm), dtype=torch.float32, device="cuda").t()
        B0 = torch.empty((n, mm), dtype=torch.float32, device="cuda").t()
        rt.synth_fill(h, 1, synth.SEED, synth.W_SWEEP, 3, Ad, param=float(mm))
        rt.synth_fill(h, 0, synth.SEED, synth.W_SWEEP, 4, B0)
        Bd = B0.clone()
        idx = np.sort(synth.rng(synth.W_SWEEP, 256, mm).choice(n, ns, replace=False))
        tidx = torch.as_tensor(idx, device="cuda")
        smp = {"m": mm, "A": rt.to_host(Ad).astype(np.float64),
               "B": np.asfortranarray(B0[:, tidx].cpu().numpy().astype(np.float64))}
        fl = float(mm) * mm * n
        row = {"m": mm, "n": n}
        for op, fn in (("trsm", rt.trsm), ("trmm", rt.trmm)):
            ts = []
            for _ in range(5):
                ts.append(_event_ms(torch, lambda: fn(h, "L", "L", "N", "N", 1.0, Ad, Bd), lambda: Bd.copy_(B0),
                                    reps=1))
            t = float(np.median(ts))
            Bd.copy_(B0)
            h.profile_begin()
            fn(h, "L", "L", "N", "N", 1.0, Ad, Bd)
            st = {(x["kclass"], x["dtype"]): x for x in h.profile_end()}
            smp[op] = np.asfortranarray(Bd[:, tidx].cpu().numpy().astype(np.float64))
            tf = fl / (t * 1e-3) / 1e12
            r = {"ms": round(t, 4), "tflops": round(tf, 2), "fraction_of_peak": round(tf / PEAK["f32"], 4),
                 "leaf": h.leaf("f32", op, mm, n), "kernels": {}}
            for (kc, dt), x in st.items():
                r["kernels"][f"{kc}_{dt}"] = {"launches": x["launches"], "ms": round(x["ms"], 4),
                                              "tflops": round(x["flops"] / max(x["ms"], 1e-9) / 1e9, 2)}
            g = st.get(("gemm", "f32"))
            if g is not None:
                gt = g["flops"] / (g["ms"] * 1e-3) / 1e12
                r["roofline"] = {"kernel": "GEMM update class (FP32 MFMA)", "bound": "mfma", "achieved": round(gt, 2),
                                 "peak": PEAK["f32"], "unit": "TFLOP/s", "frac": round(gt / PEAK["f32"], 4),
                                 "avg_launch_ms": round(g["ms"] / g["launches"], 5)}
            row[op] = r
        res["rows"].append(row)
        samples.append(smp)
        del Ad, B0, Bd
        torch.cuda.empty_cache()
    return res, samples


def cpu_check_rect256(res, samples):
    """CPU leg: sampled columns of every narrow-panel result against the oracle
    (compensated backward error; FP32 bound 5e-5)."""
    import oracle
    for row, smp in zip(res["rows"], samples):
        row["trsm"]["eta_oracle"] = oracle.trsm_eta("L", "L", "N", "N", 1.0, smp["A"], smp["B"], smp["trsm"])
        row["trmm"]["eta_oracle"] = oracle.trmm_eta("L", "L", "N", "N", 1.0, smp["A"], smp["B"], smp["trmm"])


def bench_small(rt, torch, h, reps=100):
    """Calls whose kernels take microseconds, where host planning and launches
    dominate: the small parity case (FP64 L/L/N/N, m = n = 512) and the
    narrow panel (FP32, m = 16384, n = 256), each as a plain call and as a
    call plan (the same kernels captured once in a HIP graph and replayed).
    Latency = host wall time from the call to the end of a stream
    synchronisation, median of reps (B restored outside the timed region)."""
    import time
    import synth
    res = {"workload": "FP64 L/L/N/N m=n=512 (base recipe); FP32 L/L/N/N m=16384, n=256", "cases": []}
    for (label, td, mm, nn) in (("fp64_512", torch.float64, 512, 512), ("fp32_16384x256", torch.float32, 16384, 256)):
        dcode = 0 if td == torch.float64 else 1
        Ad = rt.synth_fill(h, 1, synth.SEED, synth.W_SWEEP, 21, torch.empty((mm, mm), dtype=td, device="cuda").t(),
                           param=float(mm))
        B0 = rt.synth_fill(h, 0, synth.SEED, synth.W_SWEEP, 22, torch.empty((nn, mm), dtype=td, device="cuda").t())
        Bd = B0.clone()
        case = {"case": label, "m": mm, "n": nn}
        h.set_option(rt.OPT_TRMM_LEAVES, 1)   # the schedule a plan captures, for both ways of calling
        for op in ("trsm", "trmm"):
            fn = rt.trsm if op == "trsm" else rt.trmm
            plan = rt.CallPlan(h, op, "L", "L", "N", "N", 1.0, Ad, Bd)
            out = {}
            for way, call in (("plain", lambda: fn(h, "L", "L", "N", "N", 1.0, Ad, Bd)), ("plan", plan.run)):
                ts = []
                for r in range(reps + 3):
                    Bd.copy_(B0)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    call()
                    torch.cuda.synchronize()
                    if r >= 3:
                        ts.append((time.perf_counter() - t0) * 1e3)
                ms = float(np.median(ts))
                out[way] = {"latency_ms": round(ms, 4), "tflops": round(mm * mm * nn / (ms * 1e-3) / 1e12, 3)}
            out["speedup"] = round(out["plain"]["latency_ms"] / out["plan"]["latency_ms"], 3)
            case[op] = out
            plan.close()
        h.set_option(rt.OPT_TRMM_LEAVES, 0)
        res["cases"].append(case)
        del Ad, B0, Bd
    return res


def bench_solvers(rt, torch, h, n=16384, ns=8):
    """The operations built on the recursive TRSM, FP64, order n = 16384:
    TRTRI (lower, non-unit; n^3/3 flops), POTRS (lower Cholesky-type factor,
    n right-hand sides; 2 n^3 flops) and GETRS (P S = L U, unit lower L with
    off-diagonal U(-1,1)/n, upper U with diagonal n + U(0,1), local row
    interchanges; n right-hand sides, trans N; 2 n^3 flops).  Factors: the
    sweep recipe (off-diagonal U(-1,1), diagonal n + U(0,1)), device-drawn.
    Returns timings and, for the CPU leg, sampled columns."""
    import synth
    res = {"workload": f"FP64, order {n}: TRTRI lower non-unit; POTRS lower, {n} rhs; GETRS trans N, {n} rhs"}
    smp = {}
    idx = np.sort(synth.rng(synth.W_SWEEP, 77, n).choice(n, ns, replace=False))
    tidx = torch.as_tensor(idx, device="cuda")
    A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    rt.synth_fill(h, 1, synth.SEED, synth.W_SWEEP, 11, A0, param=float(n))
    A = A0.clone()
    t = _event_ms(torch, lambda: rt.trtri(h, "L", "N", A), lambda: A.copy_(A0))
    smp["A"] = rt.to_host(A0)
    smp["trtri"] = np.asfortranarray(A[:, tidx].cpu().numpy())
    res["trtri"] = {"ms": round(t, 3), "tflops": round(n ** 3 / 3 / (t * 1e-3) / 1e12, 3),
                    "fraction_of_peak": round(n ** 3 / 3 / (t * 1e-3) / 1e12 / PEAK["f64"], 4)}
    del A
    B0 = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    rt.synth_fill(h, 0, synth.SEED, synth.W_SWEEP, 12, B0)
    B = B0.clone()
    smp["B"] = np.asfortranarray(B0[:, tidx].cpu().numpy())
    t = _event_ms(torch, lambda: rt.potrs(h, "L", A0, B), lambda: B.copy_(B0))
    smp["potrs"] = np.asfortranarray(B[:, tidx].cpu().numpy())
    res["potrs"] = {"ms": round(t, 3), "tflops": round(2.0 * n ** 3 / (t * 1e-3) / 1e12, 3),
                    "fraction_of_peak": round(2.0 * n ** 3 / (t * 1e-3) / 1e12 / PEAK["f64"], 4)}
    # LU: unit lower part scaled by 1/n (a unit triangle with O(1) entries grows
    # exponentially), upper part of the sweep recipe
    LU = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    rt.synth_fill(h, 2, synth.SEED, synth.W_SWEEP, 13, LU, param=float(n))
    Ltmp = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    rt.synth_fill(h, 1, synth.SEED, synth.W_SWEEP, 14, Ltmp, param=0.0)
    LU += torch.tril(Ltmp, -1) / n
    del Ltmp
    g = synth.rng(synth.W_SWEEP, 15, n)
    ipiv = np.array([i + 1 + int(g.integers(0, min(8, n - i))) for i in range(n)], dtype=np.int32)
    t = _event_ms(torch, lambda: rt.getrs(h, "N", LU, ipiv, B), lambda: B.copy_(B0))
    smp["getrs"] = np.asfortranarray(B[:, tidx].cpu().numpy())
    smp["LU"] = rt.to_host(LU)
    smp["ipiv"] = ipiv
    res["getrs"] = {"ms": round(t, 3), "tflops": round(2.0 * n ** 3 / (t * 1e-3) / 1e12, 3),
                    "fraction_of_peak": round(2.0 * n ** 3 / (t * 1e-3) / 1e12 / PEAK["f64"], 4)}
    smp["idx"] = idx
    del A0, B0, B, LU
    torch.cuda.empty_cache()
    return res, smp


def cpu_check_solvers(res, smp):
    """CPU leg: sampled columns against the oracle.  TRTRI: column j of the
    inverse solves A x = e_j, so its backward error is the TRSM's on e_j.
    POTRS / GETRS: the oracle's own two substitutions on the sampled
    right-hand sides, forward error relative to them."""
    import oracle
    n = smp["A"].shape[0]
    E = np.zeros((n, len(smp["idx"])), order="F")
    E[smp["idx"], np.arange(len(smp["idx"]))] = 1.0
    Xt = np.tril(smp["trtri"][:, :])
    for c, j in enumerate(smp["idx"]):
        Xt[:j, c] = 0.0   # the strictly upper part of the column is not part of the lower inverse
    res["trtri"]["eta_oracle"] = oracle.trsm_eta("L", "L", "N", "N", 1.0, smp["A"], E, Xt)
    Xo = oracle.trsm("L", "L", "N", "N", 1.0, smp["A"], E)
    res["trtri"]["forward_error"] = float(np.max(np.abs(Xt - Xo)) / np.max(np.abs(Xo)))
    Xo = oracle.potrs("L", smp["A"], smp["B"])
    res["potrs"]["forward_error_vs_oracle"] = float(np.max(np.abs(smp["potrs"] - Xo)) / np.max(np.abs(Xo)))
    Xo = oracle.getrs("N", smp["LU"], smp["ipiv"], smp["B"])
    res["getrs"]["forward_error_vs_oracle"] = float(np.max(np.abs(smp["getrs"] - Xo)) / np.max(np.abs(Xo)))
    res["columns_checked"] = int(len(smp["idx"]))


def bench_trmm16(rt, torch, h, m=8192, ns=16):
    """TRMM with 16-bit inputs and FP32 accumulation, m = n = 8192, L/L/N/N:
    lower factor with off-diagonal U(-1,1) and diagonal c + U(0,1) (c = 45),
    B U(-1,1), drawn in FP64 on the device and rounded to BF16 / FP16.  Returns
    the timings and, for the CPU check, the sampled columns of the inputs and
    results (the error against the oracle is computed in the CPU leg)."""
    import synth
    Ad = torch.empty((m, m), dtype=torch.float64, device="cuda").t()
    B0 = torch.empty((m, m), dtype=torch.float64, device="cuda").t()
    rt.synth_fill(h, 1, synth.SEED, synth.W_MIXED, 1, Ad, param=45.0)
    rt.synth_fill(h, 0, synth.SEED, synth.W_MIXED, 2, B0)
    idx = np.sort(synth.rng(synth.W_MIXED, 16, 1).choice(m, ns, replace=False))
    tidx = torch.as_tensor(idx, device="cuda")
    res = {"workload": f"TRMM L/L/N/N m=n={m}, 16-bit A and B, FP32 accumulation and output; "
                       "diagonal 45+U(0,1), off-diagonal U(-1,1), B U(-1,1)"}
    sample = {"idx": idx, "A": rt.to_host(Ad), "B": np.asfortranarray(rt.to_host(B0)[:, idx])}
    C = torch.empty((m, m), dtype=torch.float32, device="cuda").t()
    for dt, td in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        A16 = torch.empty((m, m), dtype=td, device="cuda").t()
        B16 = torch.empty((m, m), dtype=td, device="cuda").t()
        A16.copy_(Ad)
        B16.copy_(B0)
        t = _event_ms(torch, lambda: rt.trmm_ex(h, "L", "L", "N", "N", 1.0, A16, B16, C))
        h.profile_begin()
        rt.trmm_ex(h, "L", "L", "N", "N", 1.0, A16, B16, C)
        st = {(x["kclass"], x["dtype"]): x for x in h.profile_end()}
        g = st.get(("gemm", dt))
        row = {"ms": round(t, 3), "tflops": round(m ** 3 / (t * 1e-3) / 1e12, 3),
               "fraction_of_peak": round(m ** 3 / (t * 1e-3) / 1e12 / PEAK[dt], 4)}
        if g is not None:
            gt = g["flops"] / (g["ms"] * 1e-3) / 1e12
            row["gemm16"] = {"ms": round(g["ms"], 3), "launches": g["launches"], "tflops": round(gt, 2),
                             "frac": round(gt / PEAK[dt], 4)}
        res[dt] = row
        sample[dt] = {"A": rt.to_host(A16).astype(np.float64),
                      "B": np.asfortranarray(rt.to_host(B16)[:, idx].astype(np.float64)),
                      "C": np.asfortranarray(C[:, tidx].cpu().numpy().astype(np.float64))}
        del A16, B16
    del Ad, B0, C
    torch.cuda.empty_cache()
    return res, sample


def cpu_check_trmm16(res, sample):
    """CPU leg: the 16-bit TRMM's sampled columns against the oracle, both on the
    original FP64 inputs (the rounding of A and B included) and on the rounded
    16-bit values widened exactly (the FP32 accumulation alone)."""
    import oracle
    for dt in ("bf16", "f16"):
        s = sample[dt]
        res[dt]["error_vs_oracle"] = {
            "columns": int(len(sample["idx"])),
            "eta_vs_fp64_inputs": oracle.trmm_eta("L", "L", "N", "N", 1.0, sample["A"], sample["B"], s["C"]),
            "eta_vs_rounded_inputs": oracle.trmm_eta("L", "L", "N", "N", 1.0, s["A"], s["B"], s["C"]),
        }


def bench_batched(rt, torch, h, count=4096):
    """4096 independent problems, m log-uniform [16,1024], nrhs uniform [1,128],
    uplo 50/50, factors with diagonal m + U(0,1); one graph-replayed persistent
    launch per dtype and op.  TRSM and TRMM run in place on the same operands, so
    the values stay bounded across repetitions."""
    import synth
    res = {"workload": f"{count} problems, m log-uniform [16,1024], nrhs uniform [1,128], side L, trans N"}
    for dt, td, es in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        g = synth.rng(synth.W_BATCH, 0)
        shapes = synth.batch_shapes(count, g)
        As, Bs = [], []
        for i, (mm, nn, u) in enumerate(shapes):
            As.append(rt.synth_fill(h, 1 if u == "L" else 2, synth.SEED, synth.W_BATCH, 2 * i,
                                    torch.empty((mm, mm), dtype=td, device="cuda").t(), param=float(mm)))
            Bs.append(rt.synth_fill(h, 0, synth.SEED, synth.W_BATCH, 2 * i + 1,
                                    torch.empty((nn, mm), dtype=td, device="cuda").t()))
        flops = sum(mm * mm * nn for (mm, nn, u) in shapes)
        byts = sum(es * (mm * (mm + 1) / 2 + 2 * mm * nn) for (mm, nn, u) in shapes)
        peak = 78.6e12 if dt == "f64" else 157.3e12
        bound_ms = sum(max(mm * mm * nn / peak, es * (mm * (mm + 1) / 2 + 2 * mm * nn) / 8e12)
                       for (mm, nn, u) in shapes) * 1e3
        # the longest problem alone: its chain of dependent leaves and updates
        # bounds the whole batch from below as well
        big = max(range(len(shapes)), key=lambda i: shapes[i][0] ** 2 * shapes[i][1])
        for op in ("trsm", "trmm"):
            plan = rt.BatchPlan(h, [(op, "L", u, "N", "N", 1.0, As[i], Bs[i]) for i, (mm, nn, u) in enumerate(shapes)])
            plan.run()
            torch.cuda.synchronize()
            t = _event_ms(torch, plan.run, reps=5)
            one = rt.BatchPlan(h, [(op, "L", shapes[big][2], "N", "N", 1.0, As[big], Bs[big])])
            one.run()
            torch.cuda.synchronize()
            t_chain = _event_ms(torch, one.run, reps=5)
            one.close()
            lb = max(bound_ms, t_chain)
            res[f"{op}_{dt}"] = {"ms": round(t, 4), "tflops": round(flops / (t * 1e-3) / 1e12, 3),
                                 "bound_ms": round(bound_ms, 4), "frac_of_bound": round(bound_ms / t, 3),
                                 "longest_problem_alone_ms": round(t_chain, 4),
                                 "frac_of_max_bound_and_longest": round(lb / t, 3),
                                 "chunks": plan.chunks(), "algorithmic_GB": round(byts / 1e9, 3)}
            plan.close()
        del As, Bs
    return res


def serving_stream(count, seed_key=0):
    """TRSM 80 % / TRMM 20 %; m log-uniform [32,8192]; nrhs log-uniform [1,512];
    FP64 or mixed precision 50/50 for TRSM (refinement around FP32 GEMM updates:
    two corrections where BF16 updates need four, so fewer launches and FP64
    residuals per request); factors shared by 1-16 requests spread over a
    256-request window; uplo and trans 50/50; side L."""
    import numpy as np
    import synth
    g = synth.rng(synth.W_SERVE, 1000, seed_key)
    reqs = [None] * count
    slots = list(range(count))
    fid = 0
    free = list(range(count))
    g.shuffle(free)
    order = np.argsort(g.random(count))
    i = 0
    pos = 0
    while pos < count:
        fid += 1
        uses = int(g.integers(1, 17))
        ka = int(synth.loguniform_int(g, 32, 8192, 1)[0])
        uplo = "L" if g.random() < 0.5 else "U"
        start = pos
        idxs = [start]
        for _ in range(uses - 1):
            j = start + int(g.integers(1, 256))
            if j < count:
                idxs.append(j)
        for j in idxs:
            while j < count and reqs[j] is not None:
                j += 1
            if j >= count:
                continue
            op = "trsm" if g.random() < 0.8 else "trmm"
            prec = (0 if g.random() < 0.5 else 2) if op == "trsm" else 0
            reqs[j] = dict(op=op, side="L", uplo=uplo, trans="N" if g.random() < 0.5 else "T", diag="N", m=ka,
                           n=int(synth.loguniform_int(g, 1, 512, 1)[0]), alpha=1.0, precision=prec, factor_id=fid,
                           rhs_id=j + 1)
        while pos < count and reqs[pos] is not None:
            pos += 1
    return reqs


def bench_serving(rt, count, rates=(0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2)):
    """Closed-loop saturation, then open-loop Poisson arrivals at fractions of
    it.  Latency = completion seen on the host minus the scheduled arrival (no
    coordinated omission), overall and per tag (FP64 TRSM, FP64 TRMM, refined
    TRSM).  (Served results are checked against the oracle in the GPU tests.)"""
    import numpy as np
    import synth
    reqs = serving_stream(count)
    flops = sum(r["m"] * r["m"] * r["n"] for r in reqs)
    res = {"workload": f"{count} requests (TRSM 80%/TRMM 20%, m log-uniform [32,8192], nrhs log-uniform [1,512], "
                       "FP64 or mixed+IR (FP32 GEMM updates) 50/50 for TRSM, factors shared by 1-16 requests), 64 GB budget",
           "requests": count}

    def tag(r):
        return "mixed_trsm" if r["precision"] else f"fp64_{r['op']}"

    def pct(v):
        return {"p50_ms": round(float(np.percentile(v, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(v, 99)) * 1e3, 3), "count": len(v)}

    def run(rate, keep=()):
        srv = rt.Server(slots=4, hbm_budget=64 << 30, max_batch=128, small_max=1024)
        t0 = srv.now() + 0.02
        if rate is None:
            arr = np.full(count, t0)
        else:
            arr = t0 + np.cumsum(synth.rng(synth.W_SERVE, 2000, int(rate)).exponential(1.0 / rate, count))
        kept = {}
        tickets = []
        for i, (r, ta) in enumerate(zip(reqs, arr)):
            out = np.zeros((r["m"], r["n"]), order="F") if i in keep else None
            tk = srv.submit(t_arrival=float(ta), result=out, **r)
            tickets.append(tk)
            if out is not None:
                kept[i] = out
        index = {tk: i for i, tk in enumerate(tickets)}
        srv.drain()
        comps = srv.poll(count + 16)
        st = srv.stats()
        srv.close()
        lat = np.array([c["t_done"] - c["t_arrival"] for c in comps])
        span = max(c["t_done"] for c in comps) - t0
        by_tag = {}
        for c in comps:
            by_tag.setdefault(tag(reqs[index[c["ticket"]]]), []).append(c["t_done"] - c["t_arrival"])
        bad = sum(1 for c in comps if c["status"] != 0)
        by_status = {}
        failed = []
        for c in comps:
            if c["status"] != 0:
                by_status[str(c["status"])] = by_status.get(str(c["status"]), 0) + 1
                r = reqs[index[c["ticket"]]]
                if len(failed) < 8:
                    failed.append({"status": c["status"], "op": r["op"], "m": r["m"], "n": r["n"],
                                   "precision": r["precision"], "trans": r["trans"], "uplo": r["uplo"],
                                   "iters": c["iters"], "eta": c["eta"], "factor_id": r["factor_id"]})
        out = dict(pct(lat), solves_per_s=round(count / span, 1), busy_tflops=round(flops / span / 1e12, 3),
                   per_tag={k: pct(v) for k, v in sorted(by_tag.items())},
                   errors=bad, errors_by_status=by_status, failed_sample=failed,
                   batched_requests=st["batched_requests"], launches=st["launches"], refine_turns=st["refine_turns"],
                   factor_hits=st["factor_hits"], factor_misses=st["factor_misses"],
                   evictions=st["evictions"], hbm_peak_GB=round(st["hbm_peak"] / 1e9, 2))
        out.pop("count")
        return out, kept

    sat, _ = run(None)
    progress("serving saturation", sat["solves_per_s"], "solves/s")
    res["saturation"] = sat
    mu = sat["solves_per_s"]
    res["rates"] = {}
    for frac in rates:
        r, _ = run(frac * mu)
        res["rates"][str(frac)] = dict(r, rate_per_s=round(frac * mu, 1))
        progress("serving rate", frac)
    return res


def cpu_baseline(rt, torch, h, A, B0, B0d, Ad, Bd, m, n):
    """The CPU oracle on a seeded sample of columns of the same workload (columns
    are independent for side = L, so a sample costs exactly its share), plus the
    backward error of the GPU result on those columns."""
    import oracle
    import synth
    threads = oracle.num_threads()
    ns = int(min(128, 4 * threads))
    idx = np.sort(synth.rng(synth.W_SWEEP, m, 99).choice(n, ns, replace=False))
    Bs = np.asfortranarray(B0[:, idx])
    t0 = time.perf_counter()
    Xo = oracle.trsm("L", "L", "N", "N", 1.0, A, Bs)
    t1 = time.perf_counter()
    Co = oracle.trmm("L", "L", "N", "N", 1.0, A, Bs)
    t2 = time.perf_counter()
    rate = 2.0 * m * m * ns / (t2 - t0) / 1e12
    # GPU results on the same columns
    Bd.copy_(B0d)
    rt.trsm(h, "L", "L", "N", "N", 1.0, Ad, Bd)
    torch.cuda.synchronize()
    Xg = np.asfortranarray(Bd[:, torch.as_tensor(idx, device=Bd.device)].cpu().numpy())
    Bd.copy_(B0d)
    rt.trmm(h, "L", "L", "N", "N", 1.0, Ad, Bd)
    torch.cuda.synchronize()
    Cg = np.asfortranarray(Bd[:, torch.as_tensor(idx, device=Bd.device)].cpu().numpy())
    eta = {"trsm": oracle.trsm_eta("L", "L", "N", "N", 1.0, A, Bs, Xg),
           "trmm": oracle.trmm_eta("L", "L", "N", "N", 1.0, A, Bs, Cg),
           "trsm_max_abs_diff_vs_oracle": float(np.max(np.abs(Xg - Xo))),
           "columns": int(ns)}
    # one core, a whole small problem: FP64 TRSM L/L/N/N at m = n = 1024
    g1 = synth.rng(synth.W_SWEEP, 1024, 0)
    A1 = synth.tri(1024, "L", g1, "base", fill=0.0)
    B1 = synth.dense(1024, 1024, g1)
    oracle.set_threads(1)
    try:
        t3 = time.perf_counter()
        oracle.trsm("L", "L", "N", "N", 1.0, A1, B1)
        t4 = time.perf_counter()
    finally:
        oracle.set_threads(threads)
    base = {"value": round(rate, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{ns} seeded columns of the m=n={m} FP64 TRSM and TRMM (same A), "
                      f"{t2 - t0:.1f} s of CPU time, scaled to TFLOP/s with m^2 flops per column",
            "seconds": round(t2 - t0, 2),
            "one_core_trsm_1024": {"seconds": round(t4 - t3, 3),
                                   "gflops": round(1024.0 ** 3 / (t4 - t3) / 1e9, 3)}}
    return base, eta


if __name__ == "__main__":
    main()
