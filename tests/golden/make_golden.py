"""Writes the exact-arithmetic fixtures in this folder.

Calls only ``oracle.brute`` (exact rational Gaussian elimination with partial
pivoting; paper, section "High Performance Linpack": A = L U, L y = b, U x = y).
Each fixture is a small dyadic matrix, its exact pivot sequence and its exact
packed factors / solution, printed as fractions.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import brute  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = {
    # a 4x4 dyadic matrix whose pivot search swaps at every step
    "lu_4x4_swaps": [[0.125, 1.0, -2.0, 0.5],
                     [-1.5, 0.25, 1.0, 2.0],
                     [3.0, -0.5, 0.75, -1.0],
                     [0.5, 2.5, -0.25, 1.25]],
    # Wilkinson's growth matrix, n = 8: every pivot column is a tie of magnitudes
    "lu_wilkinson_8": [[1.0 if i == j or j == 7 else (-1.0 if i > j else 0.0)
                        for j in range(8)] for i in range(8)],
    # a 6x3 tall panel (the shape of one column panel of the blocked method)
    "lu_panel_6x3": [[0.5, -1.0, 2.0], [1.0, 0.25, -0.5], [-2.0, 1.5, 0.125],
                     [0.75, -0.25, 1.0], [1.5, 2.0, -1.25], [-0.5, 0.5, 0.5]],
}
RHS = {"lu_4x4_swaps": [1.0, -0.5, 0.25, 2.0]}


def write_case(name, a):
    lu, piv, info = brute.getrf_exact(a)
    with open(os.path.join(HERE, name + ".txt"), "w") as f:
        f.write("# exact Gaussian elimination with partial pivoting (lowest row on ties)\n")
        f.write("# source: oracle/brute.py via tests/golden/make_golden.py\n")
        f.write(f"shape {len(a)} {len(a[0])}\n")
        f.write("A\n")
        for row in a:
            f.write(" ".join(repr(v) for v in row) + "\n")
        f.write("ipiv " + " ".join(str(p) for p in piv) + "\n")
        f.write(f"info {info}\n")
        f.write("LU\n")
        for row in lu:
            f.write(" ".join(str(v) for v in row) + "\n")
        if name in RHS:
            x = brute.solve_exact(a, RHS[name])
            f.write("b " + " ".join(repr(v) for v in RHS[name]) + "\n")
            f.write("x " + " ".join(str(v) for v in x) + "\n")


if __name__ == "__main__":
    for k, v in CASES.items():
        write_case(k, v)
