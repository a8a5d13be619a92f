"""Pins of the oracle's red-black IC(0) preconditioner (the plain comparator
of the learned preconditioner in the inner solves of the extended Krylov
method) and of its condensed form.

What fixes it, independently of the code under test:
* the row-by-row IC(0) factor of the red-black-permuted matrix equals the
  closed form [[D_r^{1/2}, 0], [E D_r^{-1/2}, diag(Sigma)^{1/2}]] computed
  densely from its definition (the 7-point graph is bipartite, so the
  diagonal blocks are diagonal);
* L L^T reproduces K = -A on K's pattern (the defining property of IC(0));
* the eigenvalues of M^{-1} K are 1 (once per red cell) and those of
  diag(Sigma)^{-1} Sigma, a planted wrong pivot breaks that;
* PCG with it and the condensed CG both reach the direct solution, in
  iteration counts within one of each other.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import fv3d, laplace2d, gaussian_C
from oracle import pcg as P


def _blocks(op):
    K = (-sp.csr_matrix(op.to_scipy())).toarray()
    grid = (op.nx, op.ny, op.nz if op.kind == "stencil7" else 1)
    perm = P.red_black_order(*grid)
    Kp = K[np.ix_(perm, perm)]
    idx = np.arange(op.n)
    i, j, l = idx % grid[0], (idx // grid[0]) % grid[1], idx // (grid[0] * grid[1])
    nr = int(np.count_nonzero((i + j + l) % 2 == 0))
    return K, Kp, perm, nr, grid


@pytest.mark.parametrize("make", [lambda: fv3d(5, 1.0, 3, Ny=4, Nz=3), lambda: laplace2d(7, shift=0.5)])
def test_rb_factor_closed_form(make):
    op = make()
    K, Kp, perm, nr, _ = _blocks(op)
    Dr = Kp[:nr, :nr]
    Db = Kp[nr:, nr:]
    assert np.count_nonzero(Dr - np.diag(np.diag(Dr))) == 0      # reds uncoupled
    assert np.count_nonzero(Db - np.diag(np.diag(Db))) == 0      # blacks uncoupled
    dr = np.diag(Dr)
    E = Kp[nr:, :nr]
    Sigma = Db - E @ np.diag(1.0 / dr) @ E.T
    Lcf = np.zeros_like(Kp)
    Lcf[:nr, :nr] = np.diag(np.sqrt(dr))
    Lcf[nr:, :nr] = E / np.sqrt(dr)[None, :]
    Lcf[nr:, nr:] = np.diag(np.sqrt(np.diag(Sigma)))
    L = P.ic0(sp.csr_matrix(Kp)).toarray()
    assert np.allclose(L, Lcf, rtol=1e-13, atol=1e-13 * np.abs(Kp).max())


def test_rb_factor_reproduces_pattern():
    op = fv3d(6, 1.0, 4, Ny=5, Nz=4)
    K, Kp, perm, nr, _ = _blocks(op)
    L = P.ic0(sp.csr_matrix(Kp)).toarray()
    LLt = L @ L.T
    mask = Kp != 0.0
    assert np.allclose(LLt[mask], Kp[mask], rtol=1e-12, atol=1e-12 * np.abs(Kp).max())
    # outside the pattern the product differs (dropped fill): it is not exact
    assert np.abs(LLt[~mask]).max() > 1e-3 * np.abs(Kp).max()


def test_rb_spectrum_is_one_and_schur_jacobi():
    op = fv3d(4, 1.0, 5, Ny=4, Nz=3)
    K, Kp, perm, nr, grid = _blocks(op)
    L = P.ic0(sp.csr_matrix(Kp)).toarray()
    M = L @ L.T
    lam = np.sort(sla.eigh(Kp, M, eigvals_only=True))
    dr = np.diag(Kp[:nr, :nr])
    E = Kp[nr:, :nr]
    Sigma = Kp[nr:, nr:] - E @ np.diag(1.0 / dr) @ E.T
    S = np.diag(Sigma)
    mu = sla.eigh(Sigma, np.diag(S), eigvals_only=True)
    want = np.sort(np.concatenate([np.ones(nr), mu]))
    assert np.allclose(lam, want, rtol=1e-10, atol=1e-10)
    # planted mistake: the black pivots taken from K's diagonal (the Schur
    # correction dropped) no longer give this spectrum
    Lbad = L.copy()
    Lbad[nr:, nr:] = np.diag(np.sqrt(np.diag(Kp[nr:, nr:])))
    lam_bad = np.sort(sla.eigh(Kp, Lbad @ Lbad.T, eigvals_only=True))
    assert not np.allclose(lam_bad, want, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("make,seed", [(lambda: fv3d(12, 1.0, 3), 3), (lambda: fv3d(11, 1.0, 7, Ny=10, Nz=9), 4),
                                       (lambda: laplace2d(30), 5)])
def test_rb_pcg_and_condensed_form(make, seed):
    op = make()
    A = op.to_scipy()
    grid = (op.nx, op.ny, op.nz if op.kind == "stencil7" else 1)
    b = gaussian_C(op.n, 1, seed)[:, 0]
    x_ref = spla.spsolve(sp.csc_matrix(A), b)
    rb = P.pcg(A, b, eta=1e-12, pc="ic0_rb", grid=grid)
    cond = P.schur_rb_cg(A, b, grid, eta=1e-12)
    jac = P.pcg(A, b, eta=1e-12, pc="jacobi")
    for r in (rb, cond):
        assert r.converged and r.relres_true <= 1e-12
        assert np.linalg.norm(r.x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    assert abs(rb.iters - cond.iters) <= 1
    assert cond.iters < jac.iters
