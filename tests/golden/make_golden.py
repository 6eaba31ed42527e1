"""Writes the stored expected values under tests/golden/ from the oracle only.

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fornberg  # noqa: E402


def main():
    with open(os.path.join(HERE, "fornberg_staggered.txt"), "w") as f:
        f.write("# Staggered Fornberg coefficients alpha^s_{m,n}, exact rationals, m = 1..8.\n")
        f.write("# Definition: Sec. 3 and Sec. 4.1, eq. eq_Fornberg_staggered (order 2m).\n")
        f.write("# Cross-check: alpha^s_{m,n}/2 are the 2m-point Lagrange weights at the midpoint.\n")
        f.write("# format: m n numerator denominator\n")
        for m in range(1, 9):
            for n, a in enumerate(fornberg.alpha_staggered(m), start=1):
                f.write(f"{m} {n} {a.numerator} {a.denominator}\n")


if __name__ == "__main__":
    main()
