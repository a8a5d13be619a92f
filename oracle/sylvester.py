"""Two-sided projection for A X + X B + C1 C2^T = 0 (Section 5.1).

Oracle -- test infrastructure only.  Plain float64 NumPy/SciPy.

Two standard block Krylov spaces K_m(A, C1) (basis V, T_m = V^T A V) and
K_m(B, C2) (basis U, J_m = U^T B U) of the same dimension, each built by the
block Lanczos step of Algorithm 2 (``krylov.block_lanczos_step``).  The
reduced equation T_m Y + Y J_m + E_1 gamma_1 gamma_2^T E_1^T = 0 (eq.
(reducedSylv)); Y = Q Y~ P^T with Y~_ij = -S_ij / (lambda_i + upsilon_j),
S = (Q^T E_1 gamma_1)(gamma_2^T E_1^T P).

Residual, eq. (resSylv):
  ||R_m||_F^2 = ||tau_{m+1,m} E_m^T Y_m||_F^2 + ||Y_m E_m iota_{m+1,m}^T||_F^2,
evaluated without Y_m (Algorithm 4).  Reading taken (also in the design
notes): the index of the denominator in eq. (Sylvformula) and the two
diagonal matrices of Algorithm 4 are exchanged in the text; the forms that
agree with eq. (resSylv) are Y~_ij = -S_ij / (lambda_i + upsilon_j) and
  res^2 = sum_i || e_i^T S (lambda_i I + Upsilon)^{-1} G ||^2
        + sum_j || e_j^T S^T (upsilon_j I + Lambda)^{-1} F ||^2,
F = (Q^T E_m) tau^T, G = (P^T E_m) iota^T, with no factor sqrt(2).
``residual_alg4_printed`` keeps the printed pairing for the pin that shows
the difference.

Truncation: truncated SVD of Y~ (Section 5.1), dropping singular values whose
tail has Frobenius norm <= eps; Z1 = V_m Q Y1, Z2 = U_m P Y2, either from the
stored bases or from a second Lanczos pass on each side.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla

from .krylov import (qr_pos, right_solve_upper, block_lanczos_step, assemble_T, two_pass_Z)


@dataclass
class Alg4Result:
    res: float
    lam: np.ndarray
    Q: np.ndarray
    ups: np.ndarray
    P: np.ndarray
    g1: np.ndarray
    g2: np.ndarray


def residual_alg4(T, J, gamma1, gamma2, tau, iota) -> Alg4Result:
    """Algorithm 4 with the shifts of eq. (resSylv)."""
    ell = gamma1.shape[0]
    lam, Q = sla.eigh(T)
    ups, P = sla.eigh(J)
    g1 = Q[:ell, :].T @ gamma1
    g2 = P[:ell, :].T @ gamma2
    S = g1 @ g2.T
    F = Q[-ell:, :].T @ tau.T
    G = P[-ell:, :].T @ iota.T
    acc = 0.0
    for i in range(lam.shape[0]):
        row = (S[i, :] / (lam[i] + ups)) @ G
        acc += float(row @ row)
    for j in range(ups.shape[0]):
        col = (S[:, j] / (ups[j] + lam)) @ F
        acc += float(col @ col)
    return Alg4Result(float(np.sqrt(acc)), lam, Q, ups, P, g1, g2)


def residual_alg4_printed(T, J, gamma1, gamma2, tau, iota) -> float:
    """Algorithm 4 with D'_i = upsilon_i I + Lambda against G and
    D''_i = lambda_i I + Upsilon against F, as printed."""
    ell = gamma1.shape[0]
    lam, Q = sla.eigh(T)
    ups, P = sla.eigh(J)
    S = (Q[:ell, :].T @ gamma1) @ (P[:ell, :].T @ gamma2).T
    F = Q[-ell:, :].T @ tau.T
    G = P[-ell:, :].T @ iota.T
    acc = 0.0
    for i in range(lam.shape[0]):
        a = (S[i, :] / (ups[i] + lam)) @ G
        b = (S[:, i] / (lam[i] + ups)) @ F
        acc += float(a @ a) + float(b @ b)
    return float(np.sqrt(acc))


def reduced_solution(T, J, gamma1, gamma2):
    """Y_m of eq. (reducedSylv) by Bartels-Stewart (SciPy)."""
    ell = gamma1.shape[0]
    k = T.shape[0]
    E1g1 = np.zeros((k, gamma1.shape[1]))
    E1g1[:ell] = gamma1
    E1g2 = np.zeros((k, gamma2.shape[1]))
    E1g2[:ell] = gamma2
    return sla.solve_sylvester(T, J, -(E1g1 @ E1g2.T))


def residual_reduced(T, J, gamma1, gamma2, tau, iota) -> float:
    """Eq. (resSylv) from the dense reduced solution."""
    ell = tau.shape[1]
    Y = reduced_solution(T, J, gamma1, gamma2)
    a = tau @ Y[-ell:, :]
    b = Y[:, -ell:] @ iota.T
    return float(np.sqrt(np.linalg.norm(a) ** 2 + np.linalg.norm(b) ** 2))


def tsvd_factors(lam, Q, ups, P, g1, g2, eps):
    """Y~ = U Sigma W^T; keep the leading t with ||Sigma_tail||_F <= eps;
    returns M1 = Q U_t Sigma_t^{1/2}, M2 = P W_t Sigma_t^{1/2}."""
    Yt = -(g1 @ g2.T) / (lam[:, None] + ups[None, :])
    U, sv, Wt = np.linalg.svd(Yt)
    tail = np.sqrt(np.cumsum(sv[::-1] ** 2)[::-1])
    tail = np.append(tail, 0.0)
    t = len(sv)
    while t > 0 and tail[t - 1] <= eps:
        t -= 1
    r = np.sqrt(sv[:t])
    return Q @ (U[:, :t] * r), P @ (Wt[:t].T * r), sv


@dataclass
class SylvResult:
    Z1: np.ndarray
    Z2: np.ndarray
    m: int
    t: int
    hist: list
    converged: bool
    T: np.ndarray
    J: np.ndarray
    gamma1: np.ndarray
    gamma2: np.ndarray
    tau: np.ndarray
    iota: np.ndarray
    beta1: float
    beta2: float
    status: str = "ok"
    extra: dict = field(default_factory=dict)


def sylv_std(A, B, C1: np.ndarray, C2: np.ndarray, tol: float = 1e-8, max_iter: int = 2000,
             check_every: int = 1, check: Optional[Callable[[int], bool]] = None,
             two_pass: bool = True) -> SylvResult:
    """Two lockstep block Lanczos runs, Algorithm 4 residual (corrected), TSVD,
    Z1 Z2^T ~= X.  Stops when ||R||_F / (||C1||_F ||C2||_F) <= tol."""
    s = C1.shape[1]
    beta1 = float(np.linalg.norm(C1))
    beta2 = float(np.linalg.norm(C2))
    _, gamma1 = qr_pos(C1)
    _, gamma2 = qr_pos(C2)
    if check is None:
        check = lambda m: (m % check_every) == 0  # noqa: E731
    sides = []
    for C, g in ((C1, gamma1), (C2, gamma2)):
        V1 = right_solve_upper(C, g)
        sides.append({"prev": np.zeros_like(V1), "cur": V1, "basis": [V1], "recs": []})
    hist = []
    converged = False
    alg4 = None
    m = 0
    for j in range(1, max_iter + 1):
        for sd, Aop in zip(sides, (A, B)):
            Vn, rec, _, _, _ = block_lanczos_step(Aop, sd["prev"], sd["cur"])
            sd["recs"].append(rec)
            sd["prev"], sd["cur"] = sd["cur"], Vn
            sd["basis"].append(Vn)
        m = j
        if check(j) or j == max_iter:
            T = assemble_T(sides[0]["recs"], j)
            Jm = assemble_T(sides[1]["recs"], j)
            alg4 = residual_alg4(T, Jm, gamma1, gamma2, sides[0]["recs"][-1].R, sides[1]["recs"][-1].R)
            rr = alg4.res / (beta1 * beta2)
            hist.append({"m": j, "res": rr})
            if rr <= tol:
                converged = True
                break
    T = assemble_T(sides[0]["recs"], m)
    Jm = assemble_T(sides[1]["recs"], m)
    tau = sides[0]["recs"][m - 1].R
    iota = sides[1]["recs"][m - 1].R
    if alg4 is None or alg4.lam.shape[0] != T.shape[0]:
        alg4 = residual_alg4(T, Jm, gamma1, gamma2, tau, iota)
    nu = (np.max(np.abs(alg4.lam)) + np.linalg.norm(tau) + np.max(np.abs(alg4.ups)) + np.linalg.norm(iota))
    eps = min(1e-12, 0.05 * tol / nu) * beta1 * beta2
    M1, M2, sv = tsvd_factors(alg4.lam, alg4.Q, alg4.ups, alg4.P, alg4.g1, alg4.g2, eps)
    if two_pass:
        Z1 = two_pass_Z(A, right_solve_upper(C1, gamma1), sides[0]["recs"], M1, m)
        Z2 = two_pass_Z(B, right_solve_upper(C2, gamma2), sides[1]["recs"], M2, m)
    else:
        Z1 = np.concatenate(sides[0]["basis"][:m], axis=1) @ M1
        Z2 = np.concatenate(sides[1]["basis"][:m], axis=1) @ M2
    return SylvResult(Z1=Z1, Z2=Z2, m=m, t=M1.shape[1], hist=hist, converged=converged, T=T, J=Jm,
                      gamma1=gamma1, gamma2=gamma2, tau=tau, iota=iota, beta1=beta1, beta2=beta2,
                      status="ok" if converged else "not_converged", extra={"eps": eps, "sv": sv})


def explicit_residual(A, B, Z1: np.ndarray, Z2: np.ndarray, C1: np.ndarray, C2: np.ndarray) -> float:
    """||A Z1 Z2^T + Z1 Z2^T B + C1 C2^T||_F without n1 x n2 matrices:
    R = [A Z1, Z1, C1] [Z2, B Z2, C2]^T, so ||R||_F = ||R1 R2^T||_F with the
    triangular factors of the two QRs."""
    L = np.concatenate([A @ Z1, Z1, C1], axis=1)
    Rr = np.concatenate([Z2, B @ Z2, C2], axis=1)
    R1 = np.linalg.qr(L, mode="r")
    R2 = np.linalg.qr(Rr, mode="r")
    return float(np.linalg.norm(R1 @ R2.T))


def lowrank_error(Z1, Z2, X) -> float:
    return float(np.linalg.norm(Z1 @ Z2.T - X) / np.linalg.norm(X))


def sylv_ext(A, B, C1: np.ndarray, C2: np.ndarray, tol: float = 1e-8, max_iter: int = 200,
             solveA: Optional[Callable] = None, solveB: Optional[Callable] = None, check_every: int = 1,
             check: Optional[Callable[[int], bool]] = None) -> SylvResult:
    """Section 5.1 with the two extended spaces EK_m(A, C1), EK_m(B, C2) (the
    generalisation the paper calls obvious): T_m and J_m formed as in
    ``extended.lyap_ext`` (ell = 2s), the corrected Algorithm 4 with the first
    s rows of tau_{m+1,m} and iota_{m+1,m} (their lower rows vanish in exact
    arithmetic, Section 4), TSVD, Z1 = V_m Q Y1 and Z2 = U_m P Y2 from the
    stored bases."""
    from .extended import EKSide, band_of
    s = C1.shape[1]
    ell = 2 * s
    sa = EKSide(A, C1, solveA)
    sb = EKSide(B, C2, solveB)
    beta1, beta2 = sa.beta, sb.beta
    if check is None:
        check = lambda m: (m % check_every) == 0  # noqa: E731
    hist = []
    converged = False
    alg4 = None
    m = 0
    for j in range(1, max_iter + 1):
        sa.step()
        sb.step()
        m = j
        if check(j) or j == max_iter:
            alg4 = residual_alg4(band_of(sa.T(), ell), band_of(sb.T(), ell), sa.gamma, sb.gamma,
                                 sa.tau()[:s, :], sb.tau()[:s, :])
            rr = alg4.res / (beta1 * beta2)
            hist.append({"m": j, "res": rr})
            if rr <= tol:
                converged = True
                break
    T, Jm = band_of(sa.T(m), ell), band_of(sb.T(m), ell)
    tau, iota = sa.tau(m), sb.tau(m)
    if alg4 is None or alg4.lam.shape[0] != T.shape[0]:
        alg4 = residual_alg4(T, Jm, sa.gamma, sb.gamma, tau[:s, :], iota[:s, :])
    nu = (np.max(np.abs(alg4.lam)) + np.linalg.norm(tau) + np.max(np.abs(alg4.ups)) + np.linalg.norm(iota))
    eps = min(1e-12, 0.05 * tol / nu) * beta1 * beta2
    M1, M2, sv = tsvd_factors(alg4.lam, alg4.Q, alg4.ups, alg4.P, alg4.g1, alg4.g2, eps)
    Z1 = sa.Vm(m) @ M1
    Z2 = sb.Vm(m) @ M2
    return SylvResult(Z1=Z1, Z2=Z2, m=m, t=M1.shape[1], hist=hist, converged=converged, T=T, J=Jm,
                      gamma1=sa.gamma, gamma2=sb.gamma, tau=tau, iota=iota, beta1=beta1, beta2=beta2,
                      status="ok" if converged else "not_converged", extra={"eps": eps, "sv": sv})
