"""Planted mistakes: each mutant is a copy of the oracle source with one
plausible slip (a dropped term, a wrong sign or index, a transposed operand,
a lost alpha).  The mutant is compiled on the CPU and run through a small
battery of the pins; every mutant must fail at least one of them.  This shows
the pins can tell a wrong oracle from a right one."""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg.blas as sblas

import oracle
import synth
from dense_ref import VARIANTS_NT, exact_trmm, exact_trsm, frac_to_f64_exact

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, replacement); each original must occur in the source
MUTANTS = [
    ("trsm_sign", "s += elem_opA(A, lda, trans, i, k) * x[k];", "s -= elem_opA(A, lda, trans, i, k) * x[k];"),
    ("trsm_transposed_operand", "s += elem_opA(A, lda, trans, i, k) * x[k];",
     "s += elem_opA(A, lda, trans, k, i) * x[k];"),
    ("trsm_dropped_term", "int64_t k0 = low ? 0 : i + 1, k1 = low ? i - 1 : m - 1;",
     "int64_t k0 = low ? 1 : i + 1, k1 = low ? i - 1 : m - 1;"),
    ("trsm_upper_bound", "int64_t k0 = low ? 0 : i + 1, k1 = low ? i - 1 : m - 1;",
     "int64_t k0 = low ? 0 : i + 1, k1 = low ? i - 1 : m - 2;"),
    ("trsm_no_alpha", "double v = alpha * x[i] - s;", "double v = x[i] - s;"),
    ("trsm_mul_not_div", "x[i] = (diag == 1) ? v : v / elem_opA(A, lda, trans, i, i);",
     "x[i] = (diag == 1) ? v : v * elem_opA(A, lda, trans, i, i);"),
    ("trsm_unit_ignored", "x[i] = (diag == 1) ? v : v / elem_opA(A, lda, trans, i, i);",
     "x[i] = v / elem_opA(A, lda, trans, i, i);"),
    ("trsmR_order", "int64_t j = low ? n - 1 - r : r;", "int64_t j = low ? r : n - 1 - r;"),
    ("trsmR_index", "s += B[i + k * ldb] * elem_opA(A, lda, trans, k, j);",
     "s += B[i + k * ldb] * elem_opA(A, lda, trans, j, k);"),
    ("eff_lower_flip", "return (uplo == 0) != (trans != 0);", "return (uplo == 0) == (trans != 0);"),
    ("trans_ignored", "return trans == 0 ? A[i + k * lda] : A[k + i * lda];", "return A[i + k * lda];"),
    ("trmm_dropped_diag", "int64_t k0 = low ? 0 : i, k1 = low ? i : m - 1;\n                double s = 0.0;",
     "int64_t k0 = low ? 0 : i, k1 = low ? i - 1 : m - 1;\n                double s = 0.0;"),
    ("trmm_unit_ignored", "if (i == k && diag == 1)\n        return 1.0;", "if (i == k && diag == 7)\n        return 1.0;"),
    ("trmmR_range", "int64_t k0 = low ? j : 0, k1 = low ? n - 1 : j;\n                double s = 0.0;",
     "int64_t k0 = low ? j + 1 : 0, k1 = low ? n - 1 : j;\n                double s = 0.0;"),
    ("trmm_alpha_sq", "c[i] = alpha * s;", "c[i] = alpha * alpha * s;"),
]


def _battery(orc) -> list:
    """A fast subset of the pins; returns the names of the checks that failed."""
    failed = []
    g = synth.rng(synth.W_TEST, 99)
    for side, uplo, trans in VARIANTS_NT:
        for diag in "NU":
            m, n = (9, 4) if side == "L" else (4, 9)
            ka = m if side == "L" else n
            A = synth.exact_tri(ka, uplo, g, offdiag=(-1, 0, 1), diag=(1.0, 2.0, -2.0, 4.0))
            if diag == "U":
                np.fill_diagonal(A, np.nan)
            B = synth.exact_dense(m, n, g)
            for alpha in (1.0, 2.0):
                try:
                    w = frac_to_f64_exact(exact_trsm(side, uplo, trans, diag, alpha, A, B))
                    if not np.array_equal(orc.trsm(side, uplo, trans, diag, alpha, A, B), w):
                        failed.append(("exact_trsm", side, uplo, trans, diag))
                    w = frac_to_f64_exact(exact_trmm(side, uplo, trans, diag, alpha, A, B))
                    if not np.array_equal(orc.trmm(side, uplo, trans, diag, alpha, A, B), w):
                        failed.append(("exact_trmm", side, uplo, trans, diag))
                except AssertionError:
                    failed.append(("exact_repr", side, uplo, trans, diag))
    # random data against the host BLAS
    for side, uplo, trans in VARIANTS_NT:
        m, n = 12, 7
        ka = m if side == "L" else n
        A = synth.tri(ka, uplo, g, "stress")
        B = synth.dense(m, n, g)
        kw = dict(side=int(side == "R"), lower=int(uplo == "L"), trans_a=int(trans == "T"), diag=0)
        ref = sblas.dtrsm(0.5, np.nan_to_num(A), B, **kw)
        if not np.allclose(orc.trsm(side, uplo, trans, "N", 0.5, A, B), ref, rtol=1e-12, atol=1e-13):
            failed.append(("blas_trsm", side, uplo, trans))
        ref = sblas.dtrmm(0.5, np.nan_to_num(A), B, **kw)
        if not np.allclose(orc.trmm(side, uplo, trans, "N", 0.5, A, B), ref, rtol=1e-12, atol=1e-13):
            failed.append(("blas_trmm", side, uplo, trans))
    return failed


def test_battery_passes_on_real_oracle():
    oracle.lib()
    assert _battery(oracle) == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, monkeypatch, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    cfile = tmp_path / "mut.c"
    cfile.write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-o", str(so),
                    str(cfile), "-lm"], check=True)
    oracle.lib()
    real = oracle._lib
    mut = ctypes.CDLL(str(so))
    for fn in ("oracle_trsm", "oracle_trmm"):
        getattr(mut, fn).argtypes = getattr(real, fn).argtypes
        getattr(mut, fn).restype = None
    monkeypatch.setattr(oracle, "_lib", mut)
    assert _battery(oracle), f"mutant {name} survived every pin"
