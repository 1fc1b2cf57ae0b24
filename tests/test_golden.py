"""Hand-worked examples of eqs. (1)-(4) (tests/golden/worked_3x3.json) against the oracle."""
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FIX = json.load(open(os.path.join(HERE, "golden", "worked_3x3.json")))


@pytest.mark.parametrize("case", FIX["cases"], ids=lambda c: f"{c['op']}_{c['side']}{c['uplo']}{c['trans']}{c['diag']}")
def test_worked_example(orc, case):
    A = np.asfortranarray(np.array(FIX["A_lower"], dtype=np.float64))
    A[np.triu_indices(3, 1)] = np.nan        # unreferenced triangle
    if case["diag"] == "U":
        A[np.diag_indices(3)] = np.nan       # unit diagonal is not read
        A = np.asfortranarray(A)
    B = np.asfortranarray(np.array(case["B"], dtype=np.float64))
    want = np.array(case["X"], dtype=np.float64)
    fn = orc.trsm if case["op"] == "trsm" else orc.trmm
    got = fn(case["side"], case["uplo"], case["trans"], case["diag"], case["alpha"], A, B)
    assert np.array_equal(got, want)


def test_c3_condition_labels():
    """The mixed-precision workload's factors (written by make_c3_cond.py with
    the oracle alone): each 1-norm condition number within a factor of two of
    its class 1e2 / 1e4 / 1e6, the classes in order of decreasing offset c."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "c3_cond.json")) as f:
        d = json.load(f)
    assert d["m"] == 8192
    cases = sorted(d["cases"], key=lambda c: -c["c"])
    for case, target in zip(cases, (1e2, 1e4, 1e6)):
        assert target / 2 <= case["cond1"] <= target * 2, (case, target)
