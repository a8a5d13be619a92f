"""Extended block Krylov projection for A X + X A + C C^T = 0 (Section 4).

Oracle -- test infrastructure only.  Plain float64 NumPy/SciPy.

The space EK_m(A, C) grows in the directions of A and A^{-1} at once: each
block V_j = [V_j^(1), V_j^(2)] has ell = 2s columns, the first s obtained by
multiplication with A, the last s by a solve with A.  Steps, in the paper's
order:

1. start from [C, A^{-1} C] = V_1 R (economy QR, positive diagonal); C is then
   V_1 gamma with gamma = R[:, :s] (2s x s, lower s rows zero);
2. step j: W = [A V_j^(1), A^{-1} V_j^(2)];
3. orthogonalise W against the basis and take the QR W = V_{j+1} theta;
4. the projected matrix T_m = V_m^T A V_m, which is symmetric block
   tridiagonal with 2s x 2s blocks (Section 4);
5. the residual of Proposition 1 / Algorithm 3 with ell = 2s, using
   tau_{m+1,m} = V_{m+1}^T A V_m, or its first s rows tau-bar, since the
   lower s x 2s block of tau_{m+1,m} vanishes (Section 4);
6. Z = V_m Q_m Y-check from the stored basis.

Readings taken where the paper leaves a choice (also in the design notes):
* The paper says the local block Lanczos step (Algorithm 2) can be used for
  step 3.  Here the new block is orthogonalised against *every* stored block,
  twice (block modified Gram-Schmidt, oldest first), which the basis being
  stored anyway allows; with only the two latest blocks, orthogonality is
  lost within a few tens of steps on the heterogeneous 3D operators used
  here.
* T_m is formed directly as V_m^T (A V_m) -- one extra multiplication of
  V_j^(2) by A per step -- instead of the recurrence from H_m that the paper
  cites but does not print.  Diagonal blocks are symmetrised; entries of the
  sub-diagonal blocks below the ell-th subdiagonal, which vanish in exact
  arithmetic, are dropped when T_m is banded.
* Solves with A are exact (sparse LU) unless a solver is passed in.
* A rank-deficient C is deflated to C_r = C W_r (r columns) as in the
  standard method's reading, and the space built on it; a start block
  [C_r, A^{-1} C_r] that still loses rank (span(C_r) meets an invariant
  subspace of A) is a breakdown.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .krylov import (qr_pos, right_solve_upper, residual_alg3, trunc_eps, truncated_factor,
                     deflate_columns)


def lu_solver(A):
    """Exact solves with A (sparse LU), the paper's setting."""
    lu = spla.splu(sp.csc_matrix(A))
    return lambda B: lu.solve(np.asarray(B, dtype=float))


def start_block(A, C: np.ndarray, solve):
    """[C, A^{-1} C] = V_1 R; gamma = R[:, :s]."""
    s = C.shape[1]
    W0 = np.concatenate([C, solve(C)], axis=1)
    _, R = qr_pos(W0)
    V1 = right_solve_upper(W0, R)
    return V1, R[:, :s].copy(), R


def orthogonalise_full(W: np.ndarray, basis: List[np.ndarray], sweeps: int = 2) -> np.ndarray:
    """Block modified Gram-Schmidt against every stored block, oldest first,
    repeated ``sweeps`` times."""
    for _ in range(sweeps):
        for Vi in basis:
            W = W - Vi @ (Vi.T @ W)
    return W


def band_of(T: np.ndarray, ell: int) -> np.ndarray:
    """Keep the lower and upper ell-bands of T (drops the exactly-zero-in-theory
    corners of the sub-diagonal blocks)."""
    k = T.shape[0]
    i, j = np.indices((k, k))
    return np.where(np.abs(i - j) <= ell, T, 0.0)


@dataclass
class ExtResult:
    Z: np.ndarray
    m: int
    t: int
    hist: list
    converged: bool
    T: np.ndarray              # V_m^T A V_m as formed (full)
    gamma: np.ndarray          # 2s x s
    tau: np.ndarray            # tau_{m+1,m} = V_{m+1}^T A V_m (2s x 2s)
    V: np.ndarray              # V_{m+1} (n x 2s(m+1))
    lam: np.ndarray
    beta: float
    M: np.ndarray
    status: str = "ok"
    extra: dict = field(default_factory=dict)


def lyap_ext(A, C: np.ndarray, tol: float = 1e-8, max_iter: int = 200,
             solve: Optional[Callable] = None, check_every: int = 1,
             check: Optional[Callable[[int], bool]] = None) -> ExtResult:
    """Algorithm 1 over EK_m(A, C); a rank-deficient C runs on its deflated
    columns C_r (C_r C_r^T = C C^T up to the dropped sigma_i^2), beta = ||C||_F."""
    beta = float(np.linalg.norm(C))
    C = deflate_columns(C)
    n, s = C.shape
    ell = 2 * s
    if solve is None:
        solve = lu_solver(A)
    if check is None:
        check = lambda m: (m % check_every) == 0  # noqa: E731
    V1, gamma, _ = start_block(A, C, solve)
    basis = [V1]
    AV = []                       # A V_j for the projected matrix
    Tblocks = {}                  # (i, j) -> V_i^T A V_j
    hist = []
    converged = False
    status = "not_converged"
    alg3 = None
    m = 0
    for j in range(1, max_iter + 1):
        Vj = basis[-1]
        AVj = A @ Vj
        AV.append(AVj)
        W = np.concatenate([AVj[:, :s], solve(Vj[:, s:])], axis=1)
        W = orthogonalise_full(W, basis)
        _, R = qr_pos(W)
        Vn = right_solve_upper(W, R)
        basis.append(Vn)
        Tjj = Vj.T @ AVj
        Tblocks[(j, j)] = 0.5 * (Tjj + Tjj.T)
        Tblocks[(j + 1, j)] = Vn.T @ AVj
        m = j
        if check(j) or j == max_iter:
            T = _assemble(Tblocks, j, ell)
            tau = Tblocks[(j + 1, j)]
            alg3 = residual_alg3(band_of(T, ell), gamma, tau[:s, :])
            rr = alg3.res / beta ** 2
            hist.append({"m": j, "res": rr})
            if rr <= tol:
                converged = True
                status = "ok"
                break
    T = _assemble(Tblocks, m, ell)
    tau = Tblocks[(m + 1, m)]
    Tb = band_of(T, ell)
    if alg3 is None or alg3.lam.shape[0] != T.shape[0]:
        alg3 = residual_alg3(Tb, gamma, tau[:s, :])
    eps = trunc_eps(alg3.lam, tau, tol, beta)
    M, _ = truncated_factor(alg3.lam, alg3.Q, alg3.g, eps)
    Vm = np.concatenate(basis[:m], axis=1)
    Z = Vm @ M
    return ExtResult(Z=Z, m=m, t=M.shape[1], hist=hist, converged=converged, T=T, gamma=gamma,
                     tau=tau, V=np.concatenate(basis, axis=1), lam=alg3.lam, beta=beta, M=M,
                     status=status, extra={"eps": eps})


def _assemble(Tblocks, m: int, ell: int) -> np.ndarray:
    T = np.zeros((ell * m, ell * m))
    for j in range(1, m + 1):
        T[(j - 1) * ell:j * ell, (j - 1) * ell:j * ell] = Tblocks[(j, j)]
        if j < m:
            B = Tblocks[(j + 1, j)]
            T[j * ell:(j + 1) * ell, (j - 1) * ell:j * ell] = B
            T[(j - 1) * ell:j * ell, j * ell:(j + 1) * ell] = B.T
    return T


class EKSide:
    """One extended Krylov space EK_m(A, C) advanced one block at a time with
    the same operations as ``lyap_ext`` (steps 1-4 above), for drivers that
    couple two spaces (the Sylvester equation, Section 5.1 with extended
    spaces)."""

    def __init__(self, A, C: np.ndarray, solve: Optional[Callable] = None):
        self.A = A
        self.s = C.shape[1]
        self.ell = 2 * self.s
        self.solve = solve if solve is not None else lu_solver(A)
        self.beta = float(np.linalg.norm(C))
        V1, self.gamma, _ = start_block(A, C, self.solve)
        self.basis = [V1]
        self.Tblocks = {}
        self.m = 0

    def step(self):
        s = self.s
        j = self.m + 1
        Vj = self.basis[-1]
        AVj = self.A @ Vj
        W = np.concatenate([AVj[:, :s], self.solve(Vj[:, s:])], axis=1)
        W = orthogonalise_full(W, self.basis)
        _, R = qr_pos(W)
        Vn = right_solve_upper(W, R)
        self.basis.append(Vn)
        Tjj = Vj.T @ AVj
        self.Tblocks[(j, j)] = 0.5 * (Tjj + Tjj.T)
        self.Tblocks[(j + 1, j)] = Vn.T @ AVj
        self.m = j

    def T(self, m: Optional[int] = None) -> np.ndarray:
        """T_m as formed (full); ``band_of`` gives the banded one."""
        return _assemble(self.Tblocks, self.m if m is None else m, self.ell)

    def tau(self, m: Optional[int] = None) -> np.ndarray:
        m = self.m if m is None else m
        return self.Tblocks[(m + 1, m)]

    def Vm(self, m: Optional[int] = None) -> np.ndarray:
        return np.concatenate(self.basis[:self.m if m is None else m], axis=1)
