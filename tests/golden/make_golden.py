#!/usr/bin/env python3
"""Writes the golden fixtures of this directory from the FP64 oracle only.

c1_rows.txt   the s = 32 rows chosen by the pivoted-QR rounds (Algorithm 3.1
              step 3, readings R3/R4) on the 2-D diffusion configuration
              (N = 64, r = 16, s = 32, seed 101), in selection order.
c1_y.txt      the SubApSnap coefficients y (eq. (3.3)) of its first 8 test
              parameters in the orthonormal basis, one parameter per line,
              17 significant digits.

Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import subap_inputs as si  # noqa: E402
from oracle import offline as O  # noqa: E402
from oracle import online as On  # noqa: E402


def main():
    w = si.diffusion2d()
    off = O.offline(w)
    P = w["test_params"][:8]
    Y = On.solve(off["family"], off["Q"], off["rows"], P)
    with open(os.path.join(HERE, "c1_rows.txt"), "w") as f:
        f.write("# oracle rows, 2-D diffusion N=64 r=16 s=32 seed 101 (tests/golden/make_golden.py)\n")
        f.write("\n".join(str(int(i)) for i in off["rows"]) + "\n")
    with open(os.path.join(HERE, "c1_y.txt"), "w") as f:
        f.write("# oracle y for test parameters 0..7 of the same configuration (tests/golden/make_golden.py)\n")
        for y in Y:
            f.write(" ".join(f"{v:.17g}" for v in y) + "\n")


if __name__ == "__main__":
    main()
