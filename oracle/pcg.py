"""Preconditioned conjugate gradients for the inner solves of the extended
Krylov method (Section 4 needs A^{-1} applied to a block at every step).

Oracle -- test infrastructure only.  Plain float64 NumPy/SciPy.

The paper solves with A exactly (sparse LU).  At large n this oracle instead
solves (-A) x = -b (A is symmetric negative definite, so -A is SPD) with
textbook PCG, column by column, and accepts a solve only when the *true*
relative residual ||b - A x|| / ||b|| is at most eta; if the recursively
updated residual reached eta but the true one did not, CG is restarted from
the current iterate with the true residual (at most ``restarts`` times).

Preconditioners:
* ``"none"``;
* ``"jacobi"``: M = diag(-A);
* ``"ic0"``: zero fill-in incomplete Cholesky of -A in the natural (given)
  ordering, M = L L^T, applied by two sparse triangular solves;
* ``"ic0_rb"``: the same factorisation in red-black order (grid cells with
  i + j + l even first, then the odd ones, each group in natural order; needs
  the grid shape), M = P^T L L^T P with P that permutation.

In red-black order the red cells are not coupled to each other, nor the black
ones to each other, so with K = -A = [[D_r, E^T], [E, D_b]] the factor is
L = [[D_r^{1/2}, 0], [E D_r^{-1/2}, S^{1/2}]], S = diag(Sigma) the diagonal of
the black Schur complement Sigma = D_b - E D_r^{-1} E^T (every other entry of
Sigma falls outside the pattern and is dropped).  Hence M^{-1} K is similar to
diag(I, S^{-1} Sigma), and PCG with this M advances like CG on Sigma
preconditioned by S, up to one iteration for the eigenvalue 1 of the red
block.  ``schur_rb_cg`` is that condensed form: CG on the black unknowns,
then x_r = D_r^{-1} (rhs_r - E^T x_b).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class PcgResult:
    x: np.ndarray
    iters: int            # CG iterations summed over restarts
    relres_true: float    # ||b - A x|| / ||b|| at exit
    converged: bool
    restarts: int
    history: list         # recursive ||r_k|| / ||b|| per iteration (first run)


def red_black_order(nx: int, ny: int, nz: int = 1) -> np.ndarray:
    """Row indices of the grid (lexicographic, x fastest) in red-black order:
    cells with i + j + l even, then the odd ones, each in natural order."""
    idx = np.arange(nx * ny * nz)
    i = idx % nx
    j = (idx // nx) % ny
    l = idx // (nx * ny)
    par = (i + j + l) % 2
    return np.concatenate([idx[par == 0], idx[par == 1]])


def ic0(Apos: sp.csr_matrix) -> sp.csr_matrix:
    """Lower triangular L with the sparsity of tril(Apos) and
    (L L^T)_ij = Apos_ij on that pattern (IC(0) in the order of the rows
    given: pass P Apos P^T for another ordering).
    Row-by-row (left-looking) form: for each entry (i, j), j <= i, of the
    pattern, L_ij = (a_ij - sum_{k<j} L_ik L_jk) / L_jj, L_ii = sqrt(a_ii - sum L_ik^2)."""
    A = sp.tril(Apos, format="csr")
    A.sort_indices()
    n = A.shape[0]
    rows = [dict() for _ in range(n)]
    for i in range(n):
        for p in range(A.indptr[i], A.indptr[i + 1]):
            j = A.indices[p]
            v = A.data[p]
            if j < i:
                s = v
                Li, Lj = rows[i], rows[j]
                for k, lik in Li.items():
                    if k < j and k in Lj:
                        s -= lik * Lj[k]
                Li[j] = s / Lj[j]
            elif j == i:
                s = v - sum(l * l for k, l in rows[i].items() if k < i)
                if not s > 0.0:
                    raise np.linalg.LinAlgError("IC(0) pivot is not positive")
                rows[i][i] = np.sqrt(s)
    ri, ci, vv = [], [], []
    for i in range(n):
        for j, v in rows[i].items():
            ri.append(i)
            ci.append(j)
            vv.append(v)
    return sp.csr_matrix((vv, (ri, ci)), shape=(n, n))


def make_preconditioner(A, kind: str, grid=None):
    """Returns z = M^{-1} r for the SPD matrix -A (``grid`` = (nx, ny, nz) for
    the red-black ordering)."""
    Apos = -sp.csr_matrix(A)
    if kind == "ic0_rb":
        perm = red_black_order(*grid)
        L = ic0(Apos[perm][:, perm].tocsr())
        Lt = L.T.tocsr()

        def apply_rb(r):
            y = spla.spsolve_triangular(L, r[perm], lower=True)
            z = np.empty_like(r)
            z[perm] = spla.spsolve_triangular(Lt, y, lower=False)
            return z
        return apply_rb
    if kind == "none":
        return lambda r: r.copy()
    if kind == "jacobi":
        d = Apos.diagonal()
        return lambda r: r / d
    if kind == "ic0":
        L = ic0(Apos)
        Lt = L.T.tocsr()
        def apply(r):
            y = spla.spsolve_triangular(L, r, lower=True)
            return spla.spsolve_triangular(Lt, y, lower=False)
        return apply
    raise ValueError(kind)


def pcg(A, b: np.ndarray, eta: float = 1e-12, max_iter: int = 10000, pc: str = "jacobi",
        restarts: int = 3, precond=None, x0: Optional[np.ndarray] = None, grid=None) -> PcgResult:
    """Solve A x = b (A symmetric negative definite) by PCG on (-A) x = -b."""
    Apos = -sp.csr_matrix(A)
    if precond is None:
        precond = make_preconditioner(A, pc, grid)
    rhs = -b
    bn = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else x0.copy()
    if bn == 0.0:
        return PcgResult(x * 0.0, 0, 0.0, True, 0, [])
    total = 0
    hist = []
    nrest = 0
    while True:
        r = rhs - Apos @ x
        z = precond(r)
        p = z.copy()
        rho = float(r @ z)
        for _ in range(max_iter - total):
            if float(np.linalg.norm(r)) <= eta * bn:
                break
            q = Apos @ p
            sigma = float(p @ q)
            alpha = rho / sigma
            x = x + alpha * p
            r = r - alpha * q
            total += 1
            if nrest == 0:
                hist.append(float(np.linalg.norm(r)) / bn)
            z = precond(r)
            rho_new = float(r @ z)
            beta = rho_new / rho
            rho = rho_new
            p = z + beta * p
        true = float(np.linalg.norm(b - A @ x)) / bn
        if true <= eta:
            return PcgResult(x, total, true, True, nrest, hist)
        if nrest >= restarts or total >= max_iter:
            return PcgResult(x, total, true, False, nrest, hist)
        nrest += 1


def pcg_block(A, B: np.ndarray, **kw):
    """Column-by-column PCG for an n x s block; returns (X, [PcgResult])."""
    X = np.zeros_like(B)
    res = []
    for c in range(B.shape[1]):
        r = pcg(A, B[:, c], **kw)
        X[:, c] = r.x
        res.append(r)
    return X, res


@dataclass
class RbSystem:
    """K = -A split into red and black cells (see the module header).  Black
    vectors are in natural order of the black cells; ``slot`` gives each black
    cell's place in the compact grid array (nz, ny, hxp): compact column
    i // 2 of grid line (j, l), hxp = ceil(nx / 2) rounded up to a multiple of
    ``align`` (the slots past a line's last black cell are padding)."""
    red: np.ndarray        # bool mask over the grid
    blk: np.ndarray
    dr: np.ndarray         # D_r
    Erb: sp.csr_matrix     # red rows, black columns of K (E^T)
    Ebr: sp.csr_matrix     # black rows, red columns of K (E)
    Sigma: sp.csr_matrix   # D_b - E D_r^{-1} E^T
    S: np.ndarray          # diag(Sigma)
    shape: tuple           # compact grid (nz, ny, hxp)
    slot: np.ndarray       # compact slot of each black cell

    def condense(self, res: np.ndarray) -> np.ndarray:
        """rhs~ = res_b - E D_r^{-1} res_r."""
        return res[self.blk] - self.Ebr @ (res[self.red] / self.dr)

    def expand(self, res: np.ndarray, xb: np.ndarray) -> np.ndarray:
        """The whole-grid correction: xb on the black cells and
        D_r^{-1} (res_r - E^T xb) on the red ones."""
        dx = np.empty(self.red.shape[0])
        dx[self.blk] = xb
        dx[self.red] = (res[self.red] - self.Erb @ xb) / self.dr
        return dx

    def embed(self, vb: np.ndarray) -> np.ndarray:
        """Black vector -> compact grid array (zeros at padding), flattened."""
        out = np.zeros(int(np.prod(self.shape)))
        out[self.slot] = vb
        return out

    def extract(self, a: np.ndarray) -> np.ndarray:
        return np.asarray(a).reshape(-1)[self.slot]


def rb_system(A, grid, align: int = 4) -> RbSystem:
    K = -sp.csr_matrix(A)
    n = K.shape[0]
    idx = np.arange(n)
    nx, ny, nz = grid
    i, j, l = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    red = (i + j + l) % 2 == 0
    blk = ~red
    Krr = K[red][:, red]
    Erb = K[red][:, blk].tocsr()
    Ebr = K[blk][:, red].tocsr()
    Kbb = K[blk][:, blk]
    dr = Krr.diagonal()
    if not np.all(dr > 0.0):
        raise np.linalg.LinAlgError("red diagonal is not positive")
    Sigma = (Kbb - Ebr @ sp.diags(1.0 / dr) @ Erb).tocsr()
    S = Sigma.diagonal()
    if not np.all(S > 0.0):
        raise np.linalg.LinAlgError("IC(0) pivot is not positive")
    hx = (nx + 1) // 2
    hxp = (hx + align - 1) // align * align
    slot = ((j + ny * l) * hxp + i // 2)[blk]
    return RbSystem(red, blk, dr, Erb, Ebr, Sigma, S, (nz, ny, hxp), slot)


def schur_rb_cg(A, b: np.ndarray, grid, eta: float = 1e-12, max_iter: int = 10000,
                restarts: int = 3, precond=None, system: Optional[RbSystem] = None) -> PcgResult:
    """Red-black IC(0)-PCG in its condensed form (see the module header):
    with K = -A split into red / black cells, rhs = -b,
      Sigma = D_b - E D_r^{-1} E^T,  rhs~ = rhs_b - E D_r^{-1} rhs_r,
    CG on Sigma x_b = rhs~ with the preconditioner diag(Sigma), stopped when
    ||rhs~ - Sigma x_b|| <= eta ||b||, then x_r = D_r^{-1} (rhs_r - E^T x_b).
    The residual of the whole system is then zero on the red cells and
    rhs~ - Sigma x_b on the black ones.  Accepted on the true relative residual
    ||b - A x|| / ||b|| <= eta; otherwise the condensed CG is run again on the
    residual (x += the correction), at most ``restarts`` times.

    ``precond`` (a function of the black residual) replaces diag(Sigma)^{-1};
    the iteration is then flexible CG (FCG(1): beta = -(z.q) / (p.q)), which
    with a fixed symmetric positive definite preconditioner gives the same
    iterates as PCG."""
    sysm = rb_system(A, grid) if system is None else system
    K = -sp.csr_matrix(A)
    Sigma, S = sysm.Sigma, sysm.S
    bn = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    if bn == 0.0:
        return PcgResult(x, 0, 0.0, True, 0, [])
    total, nrest, hist = 0, 0, []
    res = -b - K @ x
    while True:
        rt = sysm.condense(res)
        xb = np.zeros(int(sysm.blk.sum()))
        r = rt.copy()
        if precond is None:
            z = r / S
            p = z.copy()
            rho = float(r @ z)
            while total < max_iter and float(np.linalg.norm(r)) > eta * bn:
                q = Sigma @ p
                alpha = rho / float(p @ q)
                xb = xb + alpha * p
                r = r - alpha * q
                total += 1
                if nrest == 0:
                    hist.append(float(np.linalg.norm(r)) / bn)
                z = r / S
                rho_new = float(r @ z)
                p = z + (rho_new / rho) * p
                rho = rho_new
        else:
            z = precond(r)
            p = z.copy()
            while total < max_iter and float(np.linalg.norm(r)) > eta * bn:
                q = Sigma @ p
                pq = float(p @ q)
                alpha = float(p @ r) / pq
                xb = xb + alpha * p
                r = r - alpha * q
                total += 1
                if nrest == 0:
                    hist.append(float(np.linalg.norm(r)) / bn)
                z = precond(r)
                beta = -float(z @ q) / pq
                p = z + beta * p
        x = x + sysm.expand(res, xb)
        res = -b - K @ x
        true = float(np.linalg.norm(b - A @ x)) / bn
        if true <= eta:
            return PcgResult(x, total, true, True, nrest, hist)
        if nrest >= restarts or total >= max_iter:
            return PcgResult(x, total, true, False, nrest, hist)
        nrest += 1
