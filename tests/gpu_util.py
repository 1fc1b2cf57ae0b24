"""Shared helpers of the GPU tests: device transfer and running one call."""
from __future__ import annotations

import sys

import numpy as np

import synth

TOL = {"f64": 1e-13, "f32": 5e-5}


def torch_dtype(name):
    import torch
    return {"f64": torch.float64, "f32": torch.float32}[name]


def rounded(x: np.ndarray, dt: str) -> np.ndarray:
    """Inputs as the GPU sees them, as exact float64 values (NaN kept)."""
    return synth.round_to(x, dt)


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def run_op(rt, h, op, side, uplo, trans, diag, alpha, A, B, dt, lda=None, ldb=None):
    """Run one TRSM/TRMM on the GPU and return the result as float64 numpy."""
    import torch
    td = torch_dtype(dt)
    Ad = rt.to_device(A, td, ld=lda)
    Bd = rt.to_device(B, td, ld=ldb)
    fn = rt.trsm if op == "trsm" else rt.trmm
    fn(h, side, uplo, trans, diag, alpha, Ad, Bd)
    torch.cuda.synchronize()
    return rt.to_host(Bd).astype(np.float64)


def eta(orc, op, side, uplo, trans, diag, alpha, A, B, X):
    if op == "trsm":
        return orc.trsm_eta(side, uplo, trans, diag, alpha, A, B, X)
    return orc.trmm_eta(side, uplo, trans, diag, alpha, A, B, X)


def oracle_op(orc, op, *args):
    return (orc.trsm if op == "trsm" else orc.trmm)(*args)
