#!/usr/bin/env python3
"""Writes krr_c2_basis.npz from the FP64 oracle only.

The kernel ridge regression configuration (n = 16384 points in R^8, r = 32
snapshots, s = 128 rows, seed 202) takes the oracle about a quarter of an hour
to build: r dense Cholesky snapshot solves of order 16384 (Algorithm 3.1
step 1), the thin QR with diag(R) > 0 (step 2) and the pivoted-QR rounds on
(A(p_sel) Q)^T (step 3).  The GPU tests at that size take the oracle's basis
and rows from this file instead of rebuilding them.

Contents: Q (n x r, FP64, the orthonormal snapshot basis), rows (s, int64,
selection order) and fingerprint (a digest of the workload's inputs; the
tests refuse the file when the workload generator has changed).

Run from the repository root: python tests/golden/make_krr_basis.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import subap_inputs as si  # noqa: E402
from oracle import offline as O  # noqa: E402

PATH = os.path.join(HERE, "krr_c2_basis.npz")


def fingerprint(w) -> str:
    h = hashlib.sha256()
    for key in ("points", "rhs", "snap_params", "select_param"):
        h.update(np.ascontiguousarray(w[key], dtype=np.float64).tobytes())
    h.update(f"{w['n']} {w['r']} {w['s']} {w['lam']!r}".encode())
    return h.hexdigest()


def main():
    w = si.krr()
    off = O.offline(w)
    np.savez_compressed(PATH, Q=off["Q"], rows=off["rows"], fingerprint=np.array(fingerprint(w)))


if __name__ == "__main__":
    main()
