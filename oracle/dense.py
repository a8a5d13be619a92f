"""Krylov-free reference solutions (oracle; test infrastructure only).

All functions solve  A X + X A^T + C C^T = 0  (Lyapunov, the equation of the
Introduction with B = A, C1 = C2 = C) or  A X + X B + C1 C2^T = 0  (Sylvester)
for symmetric negative definite A, B, in float64.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.fft as sfft


def lyap_kron(A: np.ndarray, C: np.ndarray) -> np.ndarray:
    """(I (x) A + A (x) I) vec X = -vec(C C^T), solved densely.  n <= ~40."""
    n = A.shape[0]
    I = np.eye(n)
    K = np.kron(I, A) + np.kron(A, I)
    rhs = -(C @ C.T).reshape(-1, order="F")
    x = np.linalg.solve(K, rhs)
    return x.reshape(n, n, order="F")


def lyap_eig(A: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Diagonalise A = U diag(a) U^T; in that basis X~_ij = -(U^T C C^T U)_ij /
    (a_i + a_j) (the substitution of eq. (lyap2sol) applied to A itself)."""
    a, U = np.linalg.eigh(A)
    G = U.T @ C
    Xt = -(G @ G.T) / (a[:, None] + a[None, :])
    return U @ Xt @ U.T


def lyap_diag(a: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Closed form for diagonal A = diag(a): X_ij = -(C C^T)_ij / (a_i + a_j)."""
    return -(C @ C.T) / (a[:, None] + a[None, :])


def sylv_eig(A: np.ndarray, B: np.ndarray, C1: np.ndarray, C2: np.ndarray) -> np.ndarray:
    """A X + X B + C1 C2^T = 0 by diagonalising both coefficient matrices."""
    a, U = np.linalg.eigh(A)
    b, P = np.linalg.eigh(B)
    S = (U.T @ C1) @ (P.T @ C2).T
    Xt = -S / (a[:, None] + b[None, :])
    return U @ Xt @ P.T


# ------------------------------------------------------------ 5-point Laplacian
def laplace2d_eigs(N: int, shift: float = 0.0) -> np.ndarray:
    """Eigenvalues of -(1/h^2)(I (x) T + T (x) I) - shift I in DST order:
    lambda_{p,q} = -(4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2)) - shift,
    p (x direction, fastest) and q = 1..N, flattened as p + N q."""
    h = 1.0 / (N + 1)
    k = np.arange(1, N + 1)
    mu = (4.0 / (h * h)) * np.sin(k * np.pi * h / 2.0) ** 2
    lam = -(mu[None, :] + mu[:, None]) - shift    # [q, p]
    return lam.ravel()


def _dst2(Xg: np.ndarray) -> np.ndarray:
    """Orthonormal 2-D DST-I of grid columns: input (N, N, s) indexed [q, p]."""
    return sfft.dst(sfft.dst(Xg, type=1, norm="ortho", axis=0), type=1, norm="ortho", axis=1)


def lyap_laplace2d_dense(N: int, C: np.ndarray, shift: float = 0.0) -> np.ndarray:
    """Exact X for the 5-point Laplacian via its sine-transform eigenvectors
    (the DST-I basis diagonalises the operator exactly).  Dense, n = N^2 <= ~4096."""
    s = C.shape[1]
    lam = laplace2d_eigs(N, shift)
    Ch = _dst2(C.reshape(N, N, s)).reshape(N * N, s)
    Xt = -(Ch @ Ch.T) / (lam[:, None] + lam[None, :])
    # back transform rows and columns: X = S Xt S^T with S symmetric orthogonal
    n = N * N
    Y = _dst2(Xt.reshape(N, N, n)).reshape(n, n)
    X = _dst2(Y.T.reshape(N, N, n)).reshape(n, n)
    return X


def exp_sum_nodes(a: float, b: float, rel: float = 1e-14):
    """Nodes t_k and weights w_k with  1/x ~= sum_k w_k exp(-x t_k)  for x in
    [a, b] to relative accuracy ~rel: the trapezoid rule applied to
    1/x = int_R exp(u - x e^u) du (integrand analytic in |Im u| < pi/2, so the
    rule converges like exp(-pi^2/delta)); both tails are cut where they fall
    below rel."""
    delta = np.pi ** 2 / np.log(1.0 / rel)
    u_lo = np.log(rel / b) - 1.0
    u_hi = np.log(np.log(1.0 / rel) / a) + 1.0
    u = np.arange(u_lo, u_hi + delta, delta)
    return np.exp(u), delta * np.exp(u)


def dst2_columns(Z: np.ndarray, N: int) -> np.ndarray:
    """Orthonormal 2-D DST-I of every column of an N^2 x t block (grid order,
    x fastest): the coordinates of Z in the eigenvector basis of the 5-point
    Laplacian (the transform is symmetric and orthogonal, so applying it twice
    gives Z back)."""
    t = Z.shape[1]
    return _dst2(Z.reshape(N, N, t)).reshape(N * N, t)


def laplace2d_expsum_factor(N: int, C: np.ndarray, shift: float = 0.0, rel: float = 1e-14) -> np.ndarray:
    """Y^ in the sine-transform eigenbasis with X^ ~= Y^ Y^^T, X^ = S X S the
    exact solution in that basis: -1/(l_i + l_j) = int_0^inf exp((l_i + l_j) t) dt
    replaced by the exponential sum of ``exp_sum_nodes``, so that
    Y^ = [sqrt(w_k) exp(Lambda t_k) C^] (n x s*K, uncompressed) with entrywise
    relative error ~rel in X^, hence ||X - S Y^ Y^^T S||_F <= ~rel ||X||_F.
    Krylov-free."""
    n, s = C.shape
    lam = laplace2d_eigs(N, shift)                  # all negative
    a = -2.0 * lam.max()
    b = -2.0 * lam.min()
    t, w = exp_sum_nodes(a, b, rel)
    Ch = dst2_columns(C, N)
    return np.concatenate([np.sqrt(wk) * np.exp(lam * tk)[:, None] * Ch for tk, wk in zip(t, w)], axis=1)


def lyap_laplace2d_lowrank(N: int, C: np.ndarray, shift: float = 0.0,
                           rel: float = 1e-14, compress: float = 1e-15) -> np.ndarray:
    """Low-rank factor Z_ref with X ~= Z_ref Z_ref^T for the 5-point Laplacian,
    Krylov-free: the exponential-sum factor of ``laplace2d_expsum_factor``
    (exp(A t) C applied exactly with the 2-D sine transform), its columns
    compressed by a rank-revealing QR/SVD step at relative level ``compress``
    and transformed back to grid coordinates."""
    n, s = C.shape
    Zh = laplace2d_expsum_factor(N, C, shift, rel)
    # compress: Zh = Q R, SVD of R
    Q, R = np.linalg.qr(Zh)
    U, sv, _ = np.linalg.svd(R)
    keep = sv > compress * sv[0]
    Zh = Q @ (U[:, keep] * sv[keep])
    return dst2_columns(Zh, N)
