"""Write c3_cond.json: the 1-norm condition numbers of the m = 8192 factors of
the mixed-precision workload, computed by the CPU oracle alone.

The factors are lower triangular with off-diagonal entries U(-1,1) and
diagonal c + U(0,1) (the reading of "cond(A) in {1e2, 1e4, 1e6}": the 1-norm
condition number, set by the diagonal offset c).  They are regenerated here
with the host twin of the on-device Philox4x32-10 fill (synth.philox_matrix,
kind 1, workload W_MIXED, id 1), bit for bit the matrices the benchmark and
the GPU tests draw on the device.  kappa_1 = |A|_1 |A^-1|_1 with the inverse
taken column by column by the oracle's substitution.

    python tests/golden/make_c3_cond.py            (several minutes on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

M = 8192
OFFSETS = (450.0, 45.0, 17.0)   # target classes 1e2, 1e4, 1e6


def main():
    out = {"m": M, "generator": "synth.philox_matrix(1, SEED, W_MIXED, 1, m, m, c)", "norm": "1-norm",
           "cases": []}
    for c in OFFSETS:
        t0 = time.perf_counter()
        A = synth.philox_matrix(1, synth.SEED, synth.W_MIXED, 1, M, M, c)
        k = oracle.cond_one("L", "N", A)
        out["cases"].append({"c": c, "cond1": k})
        print(f"c = {c}: cond_1 = {k:.4e} ({time.perf_counter() - t0:.0f} s)", flush=True)
        del A
    with open(os.path.join(HERE, "c3_cond.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
