"""Writes tests/golden/brute_small.txt: small seeded matrices with their R
factor computed by the high-precision brute-force oracle (exact rational Gram
matrix, 60-digit Cholesky).  Calls only ``oracle`` and the seeded input
generators.  Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import brute  # noqa: E402
from paper_1002_4250_amd import inputs  # noqa: E402

CASES = [(4, 4, 11), (9, 3, 12), (16, 5, 13), (33, 6, 14), (64, 8, 15)]


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "brute_small.txt")
    with open(out, "w") as f:
        f.write("# R factors of small seeded uniform[-1,1) matrices (inputs.uniform(m, n, seed)),\n")
        f.write("# from the brute-force oracle: exact rational A^T A, Cholesky at 60 digits\n")
        f.write("# (R^T R = A^T A with diag(R) > 0 defines R, section 2).  Values are\n")
        f.write("# float.hex(); A is listed column by column, R row by row (upper part).\n")
        for m, n, seed in CASES:
            A = inputs.uniform(m, n, seed)
            R = brute.r_factor(A)
            f.write(f"case {m} {n} {seed}\n")
            for j in range(n):
                f.write("A " + " ".join(float(A[i, j]).hex() for i in range(m)) + "\n")
            for i in range(n):
                f.write("R " + " ".join(float(R[i, j]).hex() for j in range(i, n)) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
