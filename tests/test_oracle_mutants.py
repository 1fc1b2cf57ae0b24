"""Planted mistakes: each mutant is a copy of the oracle source with one
plausible slip (a dropped term, a wrong sign or index, a transposed operand,
a lost alpha).  The mutant is compiled on the CPU and run through a small
battery of the pins; every mutant must fail at least one of them.  This shows
the pins can tell a wrong oracle from a right one."""
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg.blas as sblas

import oracle
import synth
from dense_ref import (VARIANTS_NT, dense_op, exact_trmm, exact_trsm, exact_ztrmm, exact_ztrsm, frac_solve,
                       frac_to_f64_exact, grat_to_c128_exact, to_frac, zdense_op)

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
    # the error metrics: compensated residual and product, norms, eta
    ("resid_sign", "dot2_add_prod(&acc, -tri_val(A, lda, trans, diag, i, k), X[k + j * ldx]);",
     "dot2_add_prod(&acc, tri_val(A, lda, trans, diag, i, k), X[k + j * ldx]);"),
    ("resid_no_alpha", "dot2_add_prod(&acc, alpha, B[i + j * ldb]);", "dot2_add_prod(&acc, 1.0, B[i + j * ldb]);"),
    ("residR_transposed", "dot2_add_prod(&acc, -X[i + k * ldx], tri_val(A, lda, trans, diag, k, j));",
     "dot2_add_prod(&acc, -X[i + k * ldx], tri_val(A, lda, trans, diag, j, k));"),
    ("dot2_compensation_dropped", "acc->c += ep + es;", "acc->c += es;"),
    ("two_sum_sign", "*e = (a - (x - z)) + (b - z);", "*e = (a - (x - z)) - (b - z);"),
    ("trmm_dot2_transposed", "dot2_add_prod(&acc, tri_val(A, lda, trans, diag, i, k), B[k + j * ldb]);",
     "dot2_add_prod(&acc, tri_val(A, lda, trans, diag, k, i), B[k + j * ldb]);"),
    ("trmm_dot2R_transposed", "dot2_add_prod(&acc, B[i + k * ldb], tri_val(A, lda, trans, diag, k, j));",
     "dot2_add_prod(&acc, B[i + k * ldb], tri_val(A, lda, trans, diag, j, k));"),
    ("opnorm_inf_no_abs", "s += fabs(tri_val(A, lda, trans, diag, i, k));", "s += tri_val(A, lda, trans, diag, i, k);"),
    ("opnorm_inf_columns", "s += fabs(tri_val(A, lda, trans, diag, i, k));",
     "s += fabs(tri_val(A, lda, trans, diag, k, i));"),
    ("opnorm_one_drops_diag", "int64_t i0 = low ? k : 0, i1 = low ? ka - 1 : k;",
     "int64_t i0 = low ? k + 1 : 0, i1 = low ? ka - 1 : k;"),
    ("eta_side_norm_swapped", "double an = side == 0 ? oracle_opnorm_inf(uplo, trans, diag, ka, A, lda)",
     "double an = side == 1 ? oracle_opnorm_inf(uplo, trans, diag, ka, A, lda)"),
    ("eta_no_b_term", "double den = an * xn + fabs(alpha) * bn;", "double den = an * xn;"),
    ("eta_x_norm_from_b", "xn = vnorm_inf(X + v * ldx, m, 1);", "xn = vnorm_inf(B + v * ldb, m, 1);"),
    ("trmm_eta_no_alpha", "double den = fabs(alpha) * an * bn;", "double den = an * bn;"),
    # the triangular inverse
    ("trtri_sign", "s += A[i + k * lda] * x[k];", "s -= A[i + k * lda] * x[k];"),
    ("trtri_lower_start", "for (int64_t k = j; k < i; ++k)", "for (int64_t k = j + 1; k < i; ++k)"),
    ("trtri_upper_end", "for (int64_t k = i + 1; k <= j; ++k)", "for (int64_t k = i + 1; k < j; ++k)"),
    ("trtri_unit_ignored", "x[i] = (diag == 1) ? v : v / A[i + i * lda];", "x[i] = v / A[i + i * lda];"),
    ("trtri_rhs", "double v = (i == j ? 1.0 : 0.0) - s;", "double v = 1.0 - s;"),
    ("trtri_writes_unit_diag", "if (i != j || diag != 1)", "if (1)"),
    ("trtri_transposed", "s += A[i + k * lda] * x[k];", "s += A[k + i * lda] * x[k];"),
    # complex arithmetic
    ("z_conj_dropped", "if (trans == 2)\n        a.im = -a.im;", "if (trans == 7)\n        a.im = -a.im;"),
    ("z_mul_sign", "cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};",
     "cplx r = {a.re * b.re + a.im * b.im, a.re * b.im + a.im * b.re};"),
    ("z_div_imag", "r.im = (a.im - a.re * q) / den;", "r.im = (a.im + a.re * q) / den;"),
    ("z_div_other_branch", "r.im = (a.im * q - a.re) / den;", "r.im = (a.re * q - a.im) / den;"),
    ("ztrsm_alpha_dropped", "cplx v = c_mul(alpha, c_ld(B, i, j, ldb));", "cplx v = c_ld(B, i, j, ldb);"),
    ("ztrmm_alpha_conj", "c_st(C, i, j, m, c_mul(alpha, s));",
     "c_st(C, i, j, m, c_mul((cplx){alpha.re, -alpha.im}, s));"),
    ("z_transposed_index", "cplx a = trans == 0 ? c_ld(A, i, k, lda) : c_ld(A, k, i, lda);",
     "cplx a = trans == 0 ? c_ld(A, k, i, lda) : c_ld(A, k, i, lda);"),
    ("zresid_imag_sign", "a.re = -a.re;\n                    a.im = -a.im;", "a.re = -a.re;"),
    ("zopnorm_rows_as_cols", "int64_t k0 = low ? 0 : l, k1 = low ? l : ka - 1;",
     "int64_t k0 = low ? l : 0, k1 = low ? ka - 1 : l;"),
]

FUNCS = ("oracle_trsm", "oracle_trmm", "oracle_trmm_dot2", "oracle_trsm_residual", "oracle_trsm_eta",
         "oracle_trmm_eta", "oracle_opnorm_inf", "oracle_opnorm_one", "oracle_trtri", "oracle_ztrmm", "oracle_ztrsm",
         "oracle_ztrsm_residual", "oracle_ztrmm_dot2", "oracle_ztrsm_eta", "oracle_ztrmm_eta", "oracle_zopnorm")


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


def _exact_resid(side, uplo, trans, diag, alpha, A, B, X):
    """alpha B - op(A) X (or alpha B - X op(A)) in exact rationals, with the
    Dot2 error bound of Ogita, Rump and Oishi (2005) for each entry."""
    T = to_frac(dense_op(A, uplo, trans, diag))
    Bf, Xf = to_frac(B), to_frac(X)
    a = Fraction(float(alpha))
    m, n = B.shape
    ka = len(T)
    u = 2.0 ** -53
    gam = (ka + 1) * u / (1 - (ka + 1) * u)
    ex = np.empty((m, n))
    bound = np.empty((m, n))
    for i in range(m):
        for j in range(n):
            terms = [T[i][k] * Xf[k][j] for k in range(ka)] if side == "L" else [Xf[i][k] * T[k][j] for k in range(ka)]
            v = a * Bf[i][j] - sum(terms, Fraction(0))
            ex[i, j] = float(v)
            bound[i, j] = u * abs(float(v)) + gam * gam * (abs(float(a * Bf[i][j])) + sum(abs(float(t)) for t in terms))
    return ex, bound


def _metric_battery(orc) -> list:
    """Pins of the error metrics (compensated residual and product, operator
    norms, backward errors, condition number) against exact rationals and
    closed forms; returns the names of the checks that failed."""
    failed = []
    g = synth.rng(synth.W_TEST, 98)
    for side in "LR":
        for uplo, trans, diag in (("L", "N", "N"), ("U", "T", "N"), ("U", "N", "U"), ("L", "T", "U")):
            m, n = (9, 4) if side == "L" else (4, 9)
            ka = m if side == "L" else n
            A = synth.tri(ka, uplo, g, "unit" if diag == "U" else "stress")
            B = synth.dense(m, n, g)
            T = dense_op(A, uplo, trans, diag)
            alpha = 1.5
            # a near solution from numpy (not the oracle): the residual cancels heavily
            X = (np.linalg.solve(T, alpha * B) if side == "L" else np.linalg.solve(T.T, alpha * B.T).T).copy(order="F")
            R = orc.trsm_residual(side, uplo, trans, diag, alpha, A, B, X)
            ex, bound = _exact_resid(side, uplo, trans, diag, alpha, A, B, X)
            if not np.all(np.abs(R - ex) <= bound):
                failed.append(("residual", side, uplo, trans, diag))
            # compensated product: alpha op(A) B = alpha B - (alpha B - op(A) B) in exact terms
            C = orc.trmm_dot2(side, uplo, trans, diag, alpha, A, B)
            exC, bC = _exact_resid(side, uplo, trans, diag, alpha, A, np.zeros_like(B), B)
            if not np.all(np.abs(C + alpha * exC) <= 2 * abs(alpha) * bC):
                failed.append(("trmm_dot2", side, uplo, trans, diag))
            # operator norms against the explicitly formed op(A)
            ninf, none = np.abs(T).sum(axis=1).max(), np.abs(T).sum(axis=0).max()
            if not (abs(orc.opnorm_inf(uplo, trans, diag, A) - ninf) <= 1e-14 * ninf):
                failed.append(("opnorm_inf", uplo, trans, diag))
            if not (abs(orc.opnorm_one(uplo, trans, diag, A) - none) <= 1e-14 * none):
                failed.append(("opnorm_one", uplo, trans, diag))
            # eta: one planted perturbation of an exact solution, closed form
            Ae = synth.exact_tri(ka, uplo, g, offdiag=(-1, 0, 1), diag=(1.0, 2.0))
            if diag == "U":
                np.fill_diagonal(Ae, np.nan)
            Be = synth.exact_dense(m, n, g)
            Te = dense_op(Ae, uplo, trans, diag)
            Xe = frac_to_f64_exact(exact_trsm(side, uplo, trans, diag, 2.0, Ae, Be))
            if orc.trsm_eta(side, uplo, trans, diag, 2.0, Ae, Be, Xe) != 0.0:
                failed.append(("eta_exact", side, uplo, trans, diag))
            d = 2.0 ** -20
            Xp = Xe.copy(order="F")
            if side == "L":
                Xp[2, 1] += d
                r = np.abs(Te[:, 2]).max() * d
                den = np.abs(Te).sum(axis=1).max() * np.abs(Xp[:, 1]).max() + 2.0 * np.abs(Be[:, 1]).max()
            else:
                Xp[1, 2] += d
                r = np.abs(Te[2, :]).max() * d
                den = np.abs(Te).sum(axis=0).max() * np.abs(Xp[1, :]).max() + 2.0 * np.abs(Be[1, :]).max()
            if not (abs(orc.trsm_eta(side, uplo, trans, diag, 2.0, Ae, Be, Xp) - r / den) <= 1e-12 * r / den):
                failed.append(("eta_closed_form", side, uplo, trans, diag))
            Ce = frac_to_f64_exact(exact_trmm(side, uplo, trans, diag, 2.0, Ae, Be))
            Cp = Ce.copy(order="F")
            if side == "L":
                Cp[3, 0] += 1.0
                den = 2.0 * np.abs(Te).sum(axis=1).max() * np.abs(Be[:, 0]).max()
            else:
                Cp[0, 3] += 1.0
                den = 2.0 * np.abs(Te).sum(axis=0).max() * np.abs(Be[0, :]).max()
            if not (abs(orc.trmm_eta(side, uplo, trans, diag, 2.0, Ae, Be, Cp) - 1.0 / den) <= 1e-12 / den):
                failed.append(("trmm_eta_closed_form", side, uplo, trans, diag))
    return failed


def _trtri_battery(orc) -> list:
    """The triangular inverse against exact rationals (every variant, NaN in
    the triangle it must not touch and on a unit diagonal)."""
    failed = []
    g = synth.rng(synth.W_TEST, 97)
    for uplo in "LU":
        for diag in "NU":
            n = 8
            A = synth.exact_tri(n, uplo, g, offdiag=(-1, 0, 1), diag=(1.0, -1.0, 2.0))
            if diag == "U":
                np.fill_diagonal(A, np.nan)
            T = dense_op(A, uplo, "N", diag)
            want = frac_to_f64_exact(frac_solve(to_frac(T), to_frac(np.eye(n))))
            got = orc.trtri(uplo, diag, A)
            tri = np.tril if uplo == "L" else np.triu
            mask = tri(np.ones((n, n), bool), -1 if uplo == "L" else 1) | (np.eye(n, dtype=bool) & (diag == "N"))
            if not (np.array_equal(got[mask], want[mask]) and np.all(np.isnan(got[~mask]))):
                failed.append(("trtri", uplo, diag))
    return failed


def _complex_battery(orc) -> list:
    """The complex oracle against exact Gaussian rationals (every variant,
    complex alpha, unit-modulus diagonals so quotients are exact, and a
    non-unit-modulus divisor for both branches of the quotient), and its
    metrics against closed forms."""
    failed = []
    g = synth.rng(synth.W_TEST, 96)
    for side, uplo, trans in [(s_, u_, t_) for s_ in "LR" for u_ in "LU" for t_ in "NTC"]:
        m, n = (7, 3) if side == "L" else (3, 7)
        ka = m if side == "L" else n
        A = np.asfortranarray(g.integers(-1, 2, size=(ka, ka)) + 1j * g.integers(-1, 2, size=(ka, ka)))
        A[np.diag_indices(ka)] = np.array([1, 1j, -1, -1j, 2, 2j, 1 + 1j])[:ka]
        mask = np.triu(np.ones((ka, ka), bool), 1) if uplo == "L" else np.tril(np.ones((ka, ka), bool), -1)
        A[mask] = np.nan
        B = np.asfortranarray(g.integers(-4, 5, size=(m, n)) + 1j * g.integers(-4, 5, size=(m, n)))
        try:
            want = grat_to_c128_exact(exact_ztrmm(side, uplo, trans, "N", 1 - 1j, A, B))
            if not np.array_equal(orc.ztrmm(side, uplo, trans, "N", 1 - 1j, A, B), want):
                failed.append(("ztrmm", side, uplo, trans))
            want = grat_to_c128_exact(exact_ztrsm(side, uplo, trans, "N", 1 - 1j, A, B))
            got = orc.ztrsm(side, uplo, trans, "N", 1 - 1j, A, B)
            if not np.allclose(got, want, rtol=1e-14, atol=1e-14):
                failed.append(("ztrsm", side, uplo, trans))
            if orc.ztrsm_eta(side, uplo, trans, "N", 1 - 1j, A, B, want) > 1e-15:
                failed.append(("ztrsm_eta", side, uplo, trans))
            T = zdense_op(A, uplo, trans, "N")
            if abs(orc.zopnorm(uplo, trans, "N", A, True) - np.abs(T).sum(axis=1).max()) > 1e-14 * np.abs(T).sum():
                failed.append(("zopnorm", uplo, trans))
            C = orc.ztrmm_dot2(side, uplo, trans, "N", 1 - 1j, A, B)
            if not np.array_equal(C, grat_to_c128_exact(exact_ztrmm(side, uplo, trans, "N", 1 - 1j, A, B))):
                failed.append(("ztrmm_dot2", side, uplo, trans))
            Xp = want.copy(order="F")
            Xp[0, 0] += 1e-6
            R = orc.ztrsm_residual(side, uplo, trans, "N", 1 - 1j, A, B, Xp)
            Rx = (1 - 1j) * B - (T @ Xp if side == "L" else Xp @ T)
            if not np.allclose(R, Rx, rtol=1e-12, atol=1e-12):
                failed.append(("ztrsm_residual", side, uplo, trans))
        except AssertionError:
            failed.append(("exact_repr", side, uplo, trans))
    return failed


def test_battery_passes_on_real_oracle():
    oracle.lib()
    assert _battery(oracle) == []
    assert _metric_battery(oracle) == []
    assert _trtri_battery(oracle) == []
    assert _complex_battery(oracle) == []


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
    for fn in FUNCS:
        getattr(mut, fn).argtypes = getattr(real, fn).argtypes
        getattr(mut, fn).restype = getattr(real, fn).restype
    monkeypatch.setattr(oracle, "_lib", mut)
    assert _battery(oracle) or _metric_battery(oracle) or _trtri_battery(oracle) or _complex_battery(oracle), \
        f"mutant {name} survived every pin"
