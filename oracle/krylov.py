"""Standard (block) Krylov Galerkin projection for A X + X A + C C^T = 0.

Oracle — test infrastructure only (see the package docstring).  Plain float64
NumPy/SciPy, written from the paper:

* Algorithm 1 (Galerkin projection method) as the driver;
* Algorithm 2 (one block Lanczos step, block modified Gram-Schmidt applied
  twice, then an economy QR) for the basis, with the index reading
  V_{j+1} tau_{j+1,j} = A V_j - V_j tau_{j,j} - V_{j-1} tau_{j-1,j}
  (eq. (Lanczos) with its indices shifted by one, V_0 = 0);
* the residual norm two ways: from the reduced solution, eq. (reseq1), and
  from Proposition 1 / Algorithm 3 without forming Y_m;
* the rank truncation around eq. (eqn:Y) applied to Y~ (Section 3.2), and the
  factor Z_m = V_m (Q_m Y-check) either from the stored basis (Algorithm 1
  step 9) or from a second Lanczos pass (Section 3.3, eq. (twopasseq)).

Readings of the paper taken here (also listed in the design notes):
* QR factors have a positive diagonal (the unique economy QR); the new block
  is V_{j+1} = W tau_{j+1,j}^{-1} so that a second pass that repeats the same
  operations reproduces every block exactly.
* T_m uses the symmetric part of tau_{j,j} on its diagonal and the QR
  factors tau_{j+1,j} below it (their transposes above).
* Convergence is ||R_m||_F / beta^2 <= tol with beta = ||C||_F (Algorithm 1
  step 6.3).
* Rank-deficient start block (the paper assumes a full-rank basis and leaves
  deflation to the customary practice of block methods): the numerical rank r
  of C is the number of eigenvalues sigma_i^2 of C^T C above 10 n eps sigma_1^2
  (eps = 2^-52; the test a Gram matrix in floating point can make).
  When r < s the method runs on C_r = U_r Sigma_r = C W_r from the SVD
  C = U Sigma W^T, so that C_r C_r^T equals C C^T up to the dropped
  sigma_i^2, with blocks of r columns.  beta stays ||C||_F.  A later block
  that loses rank still ends the run (breakdown).
* The truncation threshold is absolute in the paper with C normalised; here it
  is eps = min(1e-12, 0.05 tol / nu) beta^2 with nu = max|lambda_i(T_m)| +
  ||tau_{m+1,m}||_F >= ||T_m underline||_2, so that dropping Sigma_2 changes
  the residual by at most 2 ||T_m underline||_2 eps <= 0.1 tol beta^2.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------- QR (Alg. 1 step 2, Alg. 2 step 9)
def qr_pos(W: np.ndarray):
    """Economy QR W = Q R with diag(R) > 0 (Householder via LAPACK)."""
    Q, R = np.linalg.qr(W, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :], R * d[:, None]


def right_solve_upper(W: np.ndarray, R: np.ndarray) -> np.ndarray:
    """W R^{-1} for upper triangular R."""
    return sla.solve_triangular(R, W.T, trans="T", lower=False).T


def numerical_rank(C: np.ndarray) -> int:
    """Eigenvalues sigma_i^2 of C^T C above 10 n eps sigma_1^2 (eps = 2^-52,
    machine epsilon), taken from the singular values of C."""
    sv = np.linalg.svd(C, compute_uv=False)
    if sv.shape[0] == 0 or sv[0] == 0.0:
        return 0
    lam = sv ** 2
    return int(np.sum(lam > 10.0 * C.shape[0] * np.finfo(float).eps * lam[0]))


def deflate_columns(C: np.ndarray) -> np.ndarray:
    """C itself at full numerical rank; otherwise C_r = U_r Sigma_r (n x r)
    from the SVD of C, so that C_r C_r^T is C C^T without the dropped
    sigma_i^2.  A zero C raises ValueError (the solution is X = 0)."""
    r = numerical_rank(C)
    if r == 0:
        raise ValueError("C is zero: the solution is X = 0")
    if r == C.shape[1]:
        return C
    U, sv, _ = np.linalg.svd(C, full_matrices=False)
    return U[:, :r] * sv[None, :r]


# ----------------------------------------------------------------- Algorithm 2
@dataclass
class StepRecord:
    alphas: list          # the four applied alpha (s x s), in order
    R: np.ndarray         # tau_{j+1,j}


def block_lanczos_step(A, Vprev: np.ndarray, Vcur: np.ndarray):
    """One block Lanczos step (Algorithm 2): W = A V_j, two sweeps of block
    MGS against V_{j-1} then V_j, accumulating the applied coefficients, then
    W = V_{j+1} tau_{j+1,j}.  Returns (V_{j+1}, StepRecord, tau_{j-1,j},
    tau_{j,j})."""
    W = A @ Vcur
    s = Vcur.shape[1]
    tau_prev = np.zeros((s, s))
    tau_cur = np.zeros((s, s))
    alphas = []
    for _sweep in range(2):
        for which, Vi in (("prev", Vprev), ("cur", Vcur)):
            alpha = Vi.T @ W
            if which == "prev":
                tau_prev = tau_prev + alpha
            else:
                tau_cur = tau_cur + alpha
            W = W - Vi @ alpha
            alphas.append(alpha)
    _, R = qr_pos(W)
    Vnext = right_solve_upper(W, R)
    return Vnext, StepRecord(alphas, R), tau_prev, tau_cur, W


def replay_step(A, Vprev, Vcur, rec: StepRecord):
    """The same operations as ``block_lanczos_step`` with the logged
    coefficients (second pass, Section 3.3)."""
    W = A @ Vcur
    k = 0
    for _sweep in range(2):
        for Vi in (Vprev, Vcur):
            W = W - Vi @ rec.alphas[k]
            k += 1
    return right_solve_upper(W, rec.R)


def assemble_T(records: List[StepRecord], m: int) -> np.ndarray:
    """T_m (sm x sm), symmetric block tridiagonal (Section 2): diagonal blocks
    sym(tau_{j,j}), sub-diagonal blocks tau_{j+1,j}."""
    s = records[0].R.shape[0]
    T = np.zeros((s * m, s * m))
    for j in range(m):
        a = records[j].alphas
        tjj = a[1] + a[3]
        T[j * s:(j + 1) * s, j * s:(j + 1) * s] = 0.5 * (tjj + tjj.T)
        if j + 1 < m:
            R = records[j].R
            T[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = R
            T[j * s:(j + 1) * s, (j + 1) * s:(j + 2) * s] = R.T
    return T


# ----------------------------------------------------------------- residual norms
def reduced_solution(T: np.ndarray, gamma: np.ndarray) -> np.ndarray:
    """Y_m of eq. (reducesLyap) by Bartels-Stewart (SciPy)."""
    ell = gamma.shape[0]
    k = T.shape[0]
    E1g = np.zeros((k, gamma.shape[1]))   # E_1 gamma, k x s (gamma is ell x s)
    E1g[:ell, :] = gamma
    return sla.solve_continuous_lyapunov(T, -(E1g @ E1g.T))


def residual_reduced(T: np.ndarray, gamma: np.ndarray, tau: np.ndarray) -> float:
    """||R_m||_F = sqrt(2) ||Y_m E_m tau_{m+1,m}^T||_F, eq. (reseq1)."""
    ell = tau.shape[1]
    Y = reduced_solution(T, gamma)
    return float(np.sqrt(2.0) * np.linalg.norm(Y[:, -ell:] @ tau.T))


@dataclass
class Alg3Result:
    res: float
    lam: np.ndarray
    Q: np.ndarray
    g: np.ndarray          # Q^T E_1 gamma   (k x ell)
    Wm: np.ndarray         # Q^T E_m tau^T   (k x ell')


def residual_alg3(T: np.ndarray, gamma: np.ndarray, tau: np.ndarray) -> Alg3Result:
    """Proposition 1 evaluated as in Algorithm 3:
    ||R_m||_F^2 = 2 sum_i || e_i^T S_m D_i^{-1} W_m ||^2 with
    S_m = Q^T E_1 gamma gamma^T E_1^T Q, W_m = Q^T E_m tau^T, D_i = lambda_i I + Lambda.
    ``tau`` may be ell x ell or the s x 2s block tau-bar of Section 4."""
    ell = gamma.shape[0]
    lam, Q = sla.eigh(T)
    g = Q[:ell, :].T @ gamma                       # rows E_1^T Q, times gamma
    S = g @ g.T
    Wm = Q[-ell:, :].T @ tau.T if tau.shape[1] == ell else Q[-tau.shape[1]:, :].T @ tau.T
    acc = 0.0
    for i in range(lam.shape[0]):
        Di = lam[i] + lam
        row = (S[i, :] / Di) @ Wm
        acc += float(row @ row)
    return Alg3Result(float(np.sqrt(2.0) * np.sqrt(acc)), lam, Q, g, Wm)


# ----------------------------------------------------------------- truncation
def trunc_eps(lam: np.ndarray, tau: np.ndarray, tol: float, beta: float) -> float:
    nu = float(np.max(np.abs(lam)) + np.linalg.norm(tau))
    return min(1e-12, 0.05 * tol / nu) * beta * beta


def truncated_factor(lam: np.ndarray, Q: np.ndarray, g: np.ndarray, eps: float):
    """Y~_ij = -(g_i . g_j)/(lambda_i + lambda_j) (eq. (lyap2sol) with
    S_m = g g^T).  Eigendecompose Y~ = W Sigma W^T (non-increasing), discard the
    trailing part with ||Sigma_2||_F <= eps (negative rounding eigenvalues are
    always discarded), keep Y-check = W_1 Sigma_1^{1/2} and return
    M = Q Y-check (k x t) and the kept eigenvalues."""
    Yt = -(g @ g.T) / (lam[:, None] + lam[None, :])
    w, U = np.linalg.eigh(Yt)
    w = w[::-1]
    U = U[:, ::-1]
    k = w.shape[0]
    npos = int(np.sum(w > 0))
    # tail[t] = ||w[t:]||_2
    tail = np.sqrt(np.cumsum((w[::-1]) ** 2)[::-1])
    tail = np.append(tail, 0.0)
    t = npos
    while t > 0 and tail[t - 1] <= eps:
        t -= 1
    Ych = U[:, :t] * np.sqrt(w[:t])[None, :]
    return Q @ Ych, w[:t]


# ----------------------------------------------------------------- Algorithm 1
@dataclass
class LyapResult:
    Z: np.ndarray
    m: int
    t: int
    hist: list
    converged: bool
    T: np.ndarray
    gamma: np.ndarray
    tau: np.ndarray
    records: list
    lam: np.ndarray
    beta: float
    M: np.ndarray
    status: str = "ok"
    extra: dict = field(default_factory=dict)


def lyap_std(A, C: np.ndarray, tol: float = 1e-8, max_iter: int = 2000,
             check: Optional[Callable[[int], bool]] = None, check_every: int = 1,
             two_pass: bool = True, compute_dense_residual: bool = False) -> LyapResult:
    """Algorithm 1 with standard block Krylov K_m(A, C).

    ``check(m)`` decides whether the residual is evaluated after m blocks
    (default: every ``check_every`` steps, as the paper's d).  The basis is
    stored only when ``two_pass`` is False (Algorithm 1 step 9); otherwise Z is
    accumulated in a second Lanczos pass from the logged coefficients."""
    beta = float(np.linalg.norm(C))
    Cr = deflate_columns(C)
    n, s = Cr.shape
    _, gamma = qr_pos(Cr)
    V1 = right_solve_upper(Cr, gamma)
    if check is None:
        check = lambda m: (m % check_every) == 0  # noqa: E731
    Vprev = np.zeros_like(V1)
    Vcur = V1
    basis = [V1] if not two_pass else None
    records: List[StepRecord] = []
    hist = []
    converged = False
    status = "not_converged"
    alg3 = None
    m = 0
    for j in range(1, max_iter + 1):
        Vnext, rec, _, _, W = block_lanczos_step(A, Vprev, Vcur)
        records.append(rec)
        m = j
        breakdown = np.min(np.diag(rec.R)) <= n * np.finfo(float).eps * max(np.linalg.norm(W), 1e-300) * 10
        if check(j) or breakdown or j == max_iter:
            T = assemble_T(records, j)
            alg3 = residual_alg3(T, gamma, rec.R)
            rr = alg3.res / beta ** 2
            entry = {"m": j, "res": rr}
            if compute_dense_residual:
                entry["res_reduced"] = residual_reduced(T, gamma, rec.R) / beta ** 2
            hist.append(entry)
            if rr <= tol:
                converged = True
                status = "ok"
                break
            if breakdown:
                status = "breakdown"
                break
        if basis is not None:
            basis.append(Vnext)
        Vprev, Vcur = Vcur, Vnext
    T = assemble_T(records, m)
    if alg3 is None or alg3.lam.shape[0] != T.shape[0]:
        alg3 = residual_alg3(T, gamma, records[m - 1].R)
    eps = trunc_eps(alg3.lam, records[m - 1].R, tol, beta)
    M, _ = truncated_factor(alg3.lam, alg3.Q, alg3.g, eps)
    if two_pass:
        Z = two_pass_Z(A, V1, records, M, m)
    else:
        Z = np.concatenate(basis[:m], axis=1) @ M
    return LyapResult(Z=Z, m=m, t=M.shape[1], hist=hist, converged=converged, T=T,
                      gamma=gamma, tau=records[m - 1].R, records=records, lam=alg3.lam,
                      beta=beta, M=M, status=status, extra={"eps": eps})


def two_pass_Z(A, V1, records, M, m):
    """Second Lanczos pass (Section 3.3): regenerate V_1..V_m from the start
    block and the logged coefficients and accumulate Z = sum_i V_i E_i^T
    (Q Y-check), eq. (twopasseq)."""
    s = V1.shape[1]
    Z = np.zeros((V1.shape[0], M.shape[1]))
    Vprev = np.zeros_like(V1)
    Vcur = V1
    for i in range(1, m + 1):
        Z += Vcur @ M[(i - 1) * s:i * s, :]
        if i < m:
            Vnext = replay_step(A, Vprev, Vcur, records[i - 1])
            Vprev, Vcur = Vcur, Vnext
    return Z


# ----------------------------------------------------------------- comparators
def explicit_residual(A, Z: np.ndarray, C: np.ndarray) -> float:
    """||A Z Z^T + Z Z^T A + C C^T||_F without forming n x n matrices:
    [AZ, Z, C] = Q R, and the residual equals R Phi R^T with
    Phi = [[0, I, 0], [I, 0, 0], [0, 0, I]]."""
    t = Z.shape[1]
    s = C.shape[1]
    P = np.concatenate([A @ Z, Z, C], axis=1)
    R = np.linalg.qr(P, mode="r")
    Phi = np.zeros((2 * t + s, 2 * t + s))
    Phi[:t, t:2 * t] = np.eye(t)
    Phi[t:2 * t, :t] = np.eye(t)
    Phi[2 * t:, 2 * t:] = np.eye(s)
    return float(np.linalg.norm(R @ Phi @ R.T))


def factor_error(Za: np.ndarray, Zb: np.ndarray) -> float:
    """||Za Za^T - Zb Zb^T||_F / ||Zb Zb^T||_F via QR of [Za, Zb]."""
    ta = Za.shape[1]
    R = np.linalg.qr(np.concatenate([Za, Zb], axis=1), mode="r")
    D = np.diag(np.concatenate([np.ones(ta), -np.ones(Zb.shape[1])]))
    num = np.linalg.norm(R @ D @ R.T)
    den = np.linalg.norm(Zb.T @ Zb)
    return float(num / den)


def lowrank_vs_dense_error(Z: np.ndarray, X: np.ndarray) -> float:
    return float(np.linalg.norm(Z @ Z.T - X) / np.linalg.norm(X))
