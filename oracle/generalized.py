"""Generalized Lyapunov equation A X E + E X A + C C^T = 0 with A symmetric
negative definite and E symmetric positive definite (Section 6, Example 3,
where such an equation is reduced to a standard Lyapunov equation).

Oracle -- test infrastructure only.  Plain float64 NumPy/SciPy, dense E (the
oracle's sizes only).

With the Cholesky factor E = L L^T and X~ = L^T X L the equation becomes the
standard one
    A~ X~ + X~ A~ + C~ C~^T = 0,   A~ = L^{-1} A L^{-T},   C~ = L^{-1} C,
which Algorithm 1 (``krylov.lyap_std``) solves; X = L^{-T} X~ L^{-1}, so the
factor is Z = L^{-T} Z~.  The stopping ratio and the residual history are
those of the transformed equation, ||L^{-1} R L^{-T}||_F / ||L^{-1} C||_F^2
with R = A X E + E X A + C C^T.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import krylov as K


@dataclass
class GenResult:
    Z: np.ndarray
    std: K.LyapResult     # the transformed run (T_m, gamma, history, ...)
    L: np.ndarray


def transform(A, E, C):
    """(A~, C~, L) of the standard equation equivalent to the generalized one."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A, dtype=np.float64)
    Ed = E.toarray() if hasattr(E, "toarray") else np.asarray(E, dtype=np.float64)
    L = sla.cholesky(Ed, lower=True)
    X = sla.solve_triangular(L, Ad, lower=True)             # L^{-1} A
    At = sla.solve_triangular(L, X.T, lower=True).T         # L^{-1} A L^{-T}
    At = 0.5 * (At + At.T)
    Ct = sla.solve_triangular(L, C, lower=True)
    return At, Ct, L


def lyap_gen(A, E, C: np.ndarray, tol: float = 1e-8, max_iter: int = 2000, check=None, check_every: int = 1,
             two_pass: bool = True) -> GenResult:
    """Algorithm 1 on the transformed equation; Z Z^T ~= X."""
    At, Ct, L = transform(A, E, C)
    r = K.lyap_std(At, Ct, tol=tol, max_iter=max_iter, check=check, check_every=check_every, two_pass=two_pass)
    Z = sla.solve_triangular(L.T, r.Z, lower=False)
    return GenResult(Z=Z, std=r, L=L)


def lyap_gen_kron(A: np.ndarray, E: np.ndarray, C: np.ndarray) -> np.ndarray:
    """(E (x) A + A (x) E) vec X = -vec(C C^T), solved densely (n <= ~40);
    independent of the Cholesky transformation."""
    n = A.shape[0]
    Kr = np.kron(E, A) + np.kron(A, E)
    x = np.linalg.solve(Kr, -(C @ C.T).reshape(-1, order="F"))
    return x.reshape(n, n, order="F")


def explicit_residual(A, E, Z: np.ndarray, C: np.ndarray) -> float:
    """||A Z Z^T E + E Z Z^T A + C C^T||_F without n x n matrices:
    R = [AZ, EZ, C] Phi [AZ, EZ, C]^T, Phi = [[0, I, 0], [I, 0, 0], [0, 0, I]]."""
    t = Z.shape[1]
    s = C.shape[1]
    P = np.concatenate([A @ Z, E @ Z, C], axis=1)
    R = np.linalg.qr(P, mode="r")
    Phi = np.zeros((2 * t + s, 2 * t + s))
    Phi[:t, t:2 * t] = np.eye(t)
    Phi[t:2 * t, :t] = np.eye(t)
    Phi[2 * t:, 2 * t:] = np.eye(s)
    return float(np.linalg.norm(R @ Phi @ R.T))
