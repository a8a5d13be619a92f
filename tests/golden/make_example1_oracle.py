"""Writes example1_oracle.json: the CPU oracle's Algorithm 1 on the paper's
Example 1 operator (Section 6: centred conservative finite differences of
(exp(-xy) u_x)_x + (exp(xy) u_y)_y on 148 x 148 interior points) with the
seeded uniform right-hand sides of `workloads.uniform_C`, tol 1e-6, the
residual checked at m = 10, 20, 40, 80 and at every step inside a window around
the iteration counts of Table 1.  Calls only oracle/ and workloads/; run from the repository root:

    python3 tests/golden/make_example1_oracle.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import krylov as K  # noqa: E402
from workloads import fd2d_variable, uniform_C  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    paper = json.load(open(os.path.join(HERE, "paper_example1.json")))
    op = fd2d_variable(148, lambda x, y: np.exp(-x * y), lambda x, y: np.exp(x * y), "e1")
    A = op.to_scipy()
    out = {"source": "oracle/krylov.py lyap_std on the Example 1 operator, C = uniform_C(n, s, 0), tol 1e-6, "
                     "residual of Proposition 1 at m = 10, 20, 40, 80 and at every step of the window",
           "tol": 1e-6, "cases": {}}
    for s in (1, 4, 8):
        ref = paper["iterations"][str(s)]
        lo = int(0.9 * ref)
        C = uniform_C(op.n, s, 0)
        early = (10, 20, 40, 80)  # before orthogonality is lost: tight parity
        r = K.lyap_std(A, C, tol=1e-6, check=lambda m, lo=lo: m >= lo or m in early, max_iter=int(1.2 * ref))
        assert r.converged and r.m > lo, (s, r.m, lo)
        out["cases"][str(s)] = {"m": r.m, "t": r.t, "window_start": lo,
                                "hist": [[h["m"], h["res"]] for h in r.hist]}
        print(s, r.m, r.t, flush=True)
    json.dump(out, open(os.path.join(HERE, "example1_oracle.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
