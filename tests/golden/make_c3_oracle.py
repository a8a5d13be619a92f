"""Writes c3_oracle.json: the CPU oracle's extended Krylov method (Section 4,
`oracle.extended.lyap_ext`) on the full-size finite-volume configuration --
-div(k grad u) on 100^3 cells (n = 1e6), lognormal k with sigma = 1
(seed_k 3), C = gaussian_C(n, 1, 3), tol 1e-8, the residual of Proposition 1
checked at every step -- with inner solves by the oracle's red-black IC(0)
conjugate gradients in condensed form (`oracle.pcg.schur_rb_cg`, true relative
residual <= 1e-12).  Z itself (n x t) is too large to keep; stored are the
residual history, m, t, beta, the explicit FP64 residual of the oracle's Z,
trace(Z Z^T), ||Z^T Z||_F = ||Z Z^T||_F, 128 seeded rows of Z (so that the
matching principal submatrix of Z Z^T can be compared) and eight seeded
bilinear forms g_k^T (Z Z^T) h_k.  Calls only oracle/ and workloads/; run from
the repository root (about ten minutes on 8 cores):

    python3 tests/golden/make_c3_oracle.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import extended as E  # noqa: E402
from oracle import krylov as K  # noqa: E402
from oracle import pcg as P  # noqa: E402
from workloads import fv3d, gaussian_C  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_ROWS = 128
N_FORMS = 8


def sample_rows(n):
    return np.sort(np.random.default_rng([31, 7]).choice(n, N_ROWS, replace=False))


def form_vectors(n, k):
    return (np.random.default_rng([77, k, 0]).standard_normal(n), np.random.default_rng([77, k, 1]).standard_normal(n))


def main():
    t0 = time.time()
    op = fv3d(100, 1.0, 3)
    A = op.to_scipy()
    C = gaussian_C(op.n, 1, 3)
    grid = (op.nx, op.ny, op.nz)
    iters = []

    def solve(B):
        X = np.empty_like(B)
        for c in range(B.shape[1]):
            r = P.schur_rb_cg(A, B[:, c], grid, eta=1e-12, max_iter=20000)
            assert r.converged, r.relres_true
            X[:, c] = r.x
            iters.append(r.iters)
        return X

    ref = E.lyap_ext(A, C, tol=1e-8, max_iter=80, solve=solve, check_every=1)
    assert ref.converged
    Z = ref.Z
    rows = sample_rows(op.n)
    forms = []
    for k in range(N_FORMS):
        g, h = form_vectors(op.n, k)
        forms.append(float((Z.T @ g) @ (Z.T @ h)))
    out = {
        "source": "oracle/extended.py lyap_ext on fv3d(100, 1.0, 3), C = gaussian_C(n, 1, 3), tol 1e-8, check every "
                  "step, inner solves oracle/pcg.py schur_rb_cg to a true relative residual of 1e-12",
        "n": op.n, "tol": 1e-8, "m": ref.m, "t": ref.t, "beta": ref.beta,
        "hist": [[h["m"], h["res"]] for h in ref.hist],
        "explicit_res": K.explicit_residual(A, Z, C) / ref.beta ** 2,
        "trace": float(np.sum(Z * Z)),
        "fro": float(np.linalg.norm(Z.T @ Z)),
        "rows": rows.tolist(),
        "Z_rows": Z[rows].tolist(),
        "forms": forms,
        "inner_iters": int(sum(iters)), "n_inner": len(iters),
    }
    json.dump(out, open(os.path.join(HERE, "c3_oracle.json"), "w"), indent=0)
    print(f"m={ref.m} t={ref.t} explicit={out['explicit_res']:.3e} inner={out['inner_iters']} "
          f"in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
