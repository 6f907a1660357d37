"""The binary64 oracle against stored exact-arithmetic fixtures (no GPU).

The fixtures in tests/golden/ were written by tests/golden/make_golden.py from
exact rational elimination (oracle/brute.py).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    rec = {}
    with open(os.path.join(HERE, name + ".txt")) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    it = iter(lines)
    for ln in it:
        key, *rest = ln.split()
        if key == "shape":
            m, n = int(rest[0]), int(rest[1])
        elif key in ("A", "LU"):
            rows = [next(it).split() for _ in range(m)]
            conv = float if key == "A" else (lambda s: float(Fraction(s)))
            rec[key] = np.array([[conv(v) for v in r] for r in rows])
        elif key == "ipiv":
            rec[key] = [int(v) for v in rest]
        elif key == "info":
            rec[key] = int(rest[0])
        elif key in ("b", "x"):
            rec[key] = np.array([float(Fraction(v)) for v in rest])
    return rec


@pytest.mark.parametrize("name", ["lu_4x4_swaps", "lu_wilkinson_8", "lu_panel_6x3"])
def test_oracle_matches_exact_fixture(name):
    rec = load(name)
    lu, piv, info = oracle.getrf(rec["A"])
    assert list(piv) == rec["ipiv"]
    assert info == rec["info"]
    assert np.max(np.abs(lu - rec["LU"])) <= 1e-14 * max(1, np.max(np.abs(rec["LU"])))
    if "x" in rec:
        x = oracle.getrs(lu, piv, rec["b"])
        assert np.max(np.abs(x - rec["x"])) <= 1e-14
