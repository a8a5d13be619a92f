"""Writes example5_oracle.json: the CPU oracle's large-A / small-B method
(Section 5.2, Algorithm 5) on the paper's Example 5 operators -- centred
finite differences of (exp(-xy) u_x)_x + (exp(xy) u_y)_y + 10 u_zz on 148^3
interior points of the unit cube, split as A X + X B with A the x-y part
(21904 x 21904) and B the z part (148 x 148) -- with the seeded uniform
right-hand sides C1 = uniform_C(21904, s, 0), C2 = uniform_C(148, s, 1),
tol 1e-6, the residual checked at m = 10, 20, 40, 80 and at every step inside
a window before the oracle's own stop, plus 64 seeded entries of Z1 Z2^T.
Calls only oracle/ and workloads/; run from the repository root:

    python3 tests/golden/make_example5_oracle.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import smallb as SB  # noqa: E402
from workloads import fd1d_dense, fd2d_variable, uniform_C  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N = 148
WINDOW = {3: 240, 8: 190}  # every step checked from here on


def main():
    op = fd2d_variable(N, lambda x, y: np.exp(-x * y), lambda x, y: np.exp(x * y), "e1")
    A = op.to_scipy()
    B = fd1d_dense(N, 10.0)
    out = {"source": "oracle/smallb.py sylv_small_b on the Example 5 split (A: x-y part, B: 10 u_zz), "
                     "C1 = uniform_C(21904, s, 0), C2 = uniform_C(148, s, 1), tol 1e-6, residual of Algorithm 5 "
                     "at m = 10, 20, 40, 80 and at every step of the window; X_ij = (Z1 Z2^T)_ij at seeded (i, j)",
           "tol": 1e-6, "cases": {}}
    rng = np.random.default_rng([55])
    ii = rng.integers(0, op.n, size=64)
    jj = rng.integers(0, N, size=64)
    for s, lo in WINDOW.items():
        C1 = uniform_C(op.n, s, 0)
        C2 = uniform_C(N, s, 1)
        early = (10, 20, 40, 80)
        r = SB.sylv_small_b(A, B, C1, C2, tol=1e-6, check=lambda m, lo=lo: m >= lo or m in early, max_iter=400,
                            two_pass=False)
        assert r.converged and r.m > lo, (s, r.m, lo)
        X = np.einsum("ka,ka->k", r.Z1[ii, :], r.Z2[jj, :])
        out["cases"][str(s)] = {"m": r.m, "t": r.t, "window_start": lo,
                                "hist": [[h["m"], h["res"]] for h in r.hist],
                                "samples": [[int(a), int(b), float(x)] for a, b, x in zip(ii, jj, X)],
                                "x_absmax_samples": float(np.max(np.abs(X)))}
        print(s, r.m, r.t, flush=True)
    json.dump(out, open(os.path.join(HERE, "example5_oracle.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
