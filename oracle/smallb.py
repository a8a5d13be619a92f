"""Large A and small B: A X + X B + C1 C2^T = 0 with a single Krylov space
(Section 5.2, "Large A and small B").

Oracle -- test infrastructure only.  Plain float64 NumPy/SciPy.

Only A is reduced.  V_m is the block Lanczos basis of K_m(A, C1) (Algorithm 2
through ``krylov.block_lanczos_step``), X_m = V_m Y_m, and the one-sided
Galerkin condition V_m^T R_m = 0 (eq. (orthLargeAsmallB)) turns the equation
into the k x n2 Sylvester equation
    T_m Y + Y B + E_1 gamma_1 C2^T = 0                   (eq. (reducedLargeASmallB)).
With T_m = Q Lambda Q^T and B = P Upsilon P^T (B decomposed once, before the
iteration),
    Y_m = Q Y~ P^T,  Y~_ij = -(Q^T E_1 gamma_1 C2^T P)_ij / (lambda_i + upsilon_j)
                                                         (eq. (formulaLargeAsmallB)).
Residual: R_m = V_{m+1} tau_{m+1,m} E_m^T Y_m, so ||R_m||_F = ||tau E_m^T Y_m||_F,
computed without Y_m by Algorithm 5:
    S = (P^T C2 gamma_1^T)(E_1^T Q)   (n2 x k),   W = (Q^T E_m) tau^T   (k x ell),
    res^2 = sum_i || (e_i^T S) (upsilon_i I + Lambda)^{-1} W ||^2.
Truncation: truncated SVD Y~ ~= Y1 Y2^T (tail of the singular values with
Frobenius norm <= eps), Z1 = V_m (Q Y1), Z2 = P Y2, Z1 from the stored basis or
from a second Lanczos pass (Section 3.3).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla

from .krylov import qr_pos, right_solve_upper, block_lanczos_step, assemble_T, two_pass_Z


@dataclass
class Alg5Result:
    res: float
    lam: np.ndarray
    Q: np.ndarray


def small_b_setup(B: np.ndarray, C2: np.ndarray, gamma1: np.ndarray):
    """B = P Upsilon P^T (ascending) and G = P^T C2 gamma_1^T (n2 x ell): the
    inputs of Algorithm 5 that are fixed for the whole iteration."""
    ups, P = sla.eigh(np.asarray(B, dtype=np.float64))
    G = P.T @ C2 @ gamma1.T
    return ups, P, G


def residual_alg5(T: np.ndarray, tau: np.ndarray, G: np.ndarray, ups: np.ndarray) -> Alg5Result:
    """Algorithm 5: ||R_m||_F from T_m, tau_{m+1,m}, G = P^T C2 gamma_1^T and
    the eigenvalues of B, looping over the n2 eigenvalues of B."""
    ell = tau.shape[0]
    lam, Q = sla.eigh(T)                      # step 1
    S = G @ Q[:ell, :]                        # step 2: (P^T C2 gamma1^T)(E_1^T Q)
    W = Q[-ell:, :].T @ tau.T                 # step 3: (Q^T E_m) tau^T
    acc = 0.0                                 # step 4
    for i in range(ups.shape[0]):             # steps 5-8
        D = ups[i] + lam                      # step 6: diagonal of upsilon_i I + Lambda
        row = (S[i, :] / D) @ W               # step 7
        acc += float(row @ row)
    return Alg5Result(float(np.sqrt(acc)), lam, Q)   # step 9


def reduced_solution(T: np.ndarray, B: np.ndarray, gamma1: np.ndarray, C2: np.ndarray) -> np.ndarray:
    """Y_m of eq. (reducedLargeASmallB) by Bartels-Stewart (SciPy)."""
    ell = gamma1.shape[0]
    E1g = np.zeros((T.shape[0], gamma1.shape[1]))
    E1g[:ell] = gamma1
    return sla.solve_sylvester(T, np.asarray(B, dtype=np.float64), -(E1g @ C2.T))


def ytilde(lam, Q, ups, G) -> np.ndarray:
    """Y~ of eq. (formulaLargeAsmallB) (k x n2): Q^T E_1 gamma_1 C2^T P = (G Q[:ell])^T."""
    ell = G.shape[1]
    return -((Q[:ell, :].T @ G.T) / (lam[:, None] + ups[None, :]))


def tsvd_factors(Yt: np.ndarray, eps: float):
    """Y~ = U Sigma W^T; keep the leading t with ||Sigma_tail||_F <= eps;
    returns U_t Sigma_t^{1/2}, W_t Sigma_t^{1/2} and the singular values."""
    U, sv, Wt = np.linalg.svd(Yt, full_matrices=False)
    tail = np.append(np.sqrt(np.cumsum(sv[::-1] ** 2)[::-1]), 0.0)
    t = len(sv)
    while t > 0 and tail[t - 1] <= eps:
        t -= 1
    r = np.sqrt(sv[:t])
    return U[:, :t] * r, Wt[:t].T * r, sv


@dataclass
class SmallBResult:
    Z1: np.ndarray
    Z2: np.ndarray
    m: int
    t: int
    hist: list
    converged: bool
    T: np.ndarray
    gamma1: np.ndarray
    tau: np.ndarray
    ups: np.ndarray
    P: np.ndarray
    beta1: float
    beta2: float
    status: str = "ok"
    extra: dict = field(default_factory=dict)


def sylv_small_b(A, B: np.ndarray, C1: np.ndarray, C2: np.ndarray, tol: float = 1e-8, max_iter: int = 2000,
                 check_every: int = 1, check: Optional[Callable[[int], bool]] = None,
                 two_pass: bool = True) -> SmallBResult:
    """One block Lanczos run on (A, C1), Algorithm 5 at the checked steps,
    stop when ||R||_F / (||C1||_F ||C2||_F) <= tol, truncated Y~, Z1 Z2^T ~= X.
    B is a dense symmetric n2 x n2 matrix."""
    s = C1.shape[1]
    beta1 = float(np.linalg.norm(C1))
    beta2 = float(np.linalg.norm(C2))
    _, gamma1 = qr_pos(C1)
    ups, P, G = small_b_setup(B, C2, gamma1)
    if check is None:
        check = lambda m: (m % check_every) == 0  # noqa: E731
    V1 = right_solve_upper(C1, gamma1)
    prev, cur = np.zeros_like(V1), V1
    basis, recs, hist = [V1], [], []
    converged = False
    a5 = None
    m = 0
    for j in range(1, max_iter + 1):
        Vn, rec, _, _, _ = block_lanczos_step(A, prev, cur)
        recs.append(rec)
        prev, cur = cur, Vn
        basis.append(Vn)
        m = j
        if check(j) or j == max_iter:
            a5 = residual_alg5(assemble_T(recs, j), rec.R, G, ups)
            rr = a5.res / (beta1 * beta2)
            hist.append({"m": j, "res": rr})
            if rr <= tol:
                converged = True
                break
    T = assemble_T(recs, m)
    tau = recs[m - 1].R
    if a5 is None or a5.lam.shape[0] != T.shape[0]:
        a5 = residual_alg5(T, tau, G, ups)
    # ||R(Y) - R(Y + dY)||_F <= (||T_m underline||_2 + ||B||_2) ||dY||_F
    nu = np.max(np.abs(a5.lam)) + np.linalg.norm(tau) + np.max(np.abs(ups))
    eps = min(1e-12, 0.05 * tol / nu) * beta1 * beta2
    Y1, Y2, sv = tsvd_factors(ytilde(a5.lam, a5.Q, ups, G), eps)
    M1 = a5.Q @ Y1
    if two_pass:
        Z1 = two_pass_Z(A, right_solve_upper(C1, gamma1), recs, M1, m)
    else:
        Z1 = np.concatenate(basis[:m], axis=1) @ M1
    Z2 = P @ Y2
    return SmallBResult(Z1=Z1, Z2=Z2, m=m, t=M1.shape[1], hist=hist, converged=converged, T=T, gamma1=gamma1,
                        tau=tau, ups=ups, P=P, beta1=beta1, beta2=beta2,
                        status="ok" if converged else "not_converged", extra={"eps": eps, "sv": sv})
