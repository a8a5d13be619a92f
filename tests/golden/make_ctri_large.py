"""Writes ctri_large.json: the CPU oracle's Algorithm 3 (Proposition 1,
`oracle.krylov.residual_alg3`, LAPACK eigendecomposition of the dense T) on
seeded symmetric negative definite band matrices of the projected matrix's
shape (`workloads.random_band_T`: a stiff Toeplitz band with a jittered
diagonal, bandwidth ell = 8) of order k = 6000 and k = 10000 -- sizes whose top divide-and-conquer merge takes the LDS-staged and
the global-memory secular-equation kernels.  Stored: the residual norm and
every 50th eigenvalue (plus the largest).  Calls only oracle/ and workloads/;
run from the repository root (about a minute on 8 cores):

    python3 tests/golden/make_ctri_large.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import krylov as K  # noqa: E402
from workloads import random_band_T  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = ((6000, 8, 1), (10000, 8, 2))
STRIDE = 50


def dense_of(band):
    k, l1 = band.shape
    T = np.zeros((k, k))
    for d in range(l1):
        idx = np.arange(k - d)
        T[idx + d, idx] = band[:k - d, d]
        T[idx, idx + d] = band[:k - d, d]
    return T


def main():
    out = {"source": "oracle/krylov.py residual_alg3 on workloads.random_band_T(k, ell, seed)",
           "stride": STRIDE, "cases": []}
    for k, ell, seed in CASES:
        band, gamma, tau = random_band_T(k, ell, seed)
        r = K.residual_alg3(dense_of(band), gamma, tau)
        sel = list(range(0, k, STRIDE)) + [k - 1]
        out["cases"].append({"k": k, "ell": ell, "seed": seed, "res": r.res,
                             "lam_idx": sel, "lam": [float(r.lam[i]) for i in sel]})
        print(k, r.res, r.lam[0], r.lam[-1], flush=True)
    json.dump(out, open(os.path.join(HERE, "ctri_large.json"), "w"), indent=0)


if __name__ == "__main__":
    main()
