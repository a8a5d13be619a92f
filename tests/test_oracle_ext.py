"""Pins of the extended Krylov oracle (Section 4) and of the inner PCG oracle
against facts fixed by the mathematics: dense reference solutions, the block
tridiagonal structure of T_m, the vanishing lower block of tau_{m+1,m}, the
Arnoldi-type relation, span properties of EK_m(A, C), the Krylov optimality
of CG iterates and exact termination cases.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import fv3d, laplace2d, gaussian_C
from oracle import extended as E
from oracle import dense as D
from oracle import krylov as K
from oracle import pcg as P


# ------------------------------------------------------------------ PCG
def _spd_problem(N=8, seed=3):
    op = fv3d(N, 1.0, seed)
    A = op.to_scipy()
    b = gaussian_C(op.n, 1, seed)[:, 0]
    return A, b


def test_pcg_matches_direct_solve():
    A, b = _spd_problem()
    x_ref = spla.spsolve(sp.csc_matrix(A), b)
    for pc in ("none", "jacobi", "ic0"):
        r = P.pcg(A, b, eta=1e-12, pc=pc)
        assert r.converged and r.relres_true <= 1e-12
        assert np.linalg.norm(r.x - x_ref) <= 1e-10 * np.linalg.norm(x_ref), pc


def test_cg_iterates_are_krylov_minimisers():
    """Without preconditioner the k-th CG iterate minimises the (-A)-norm of
    the error over K_k(-A, -b); computed here by a dense Galerkin projection."""
    A, b = _spd_problem(N=6)
    Ap = -A.toarray()
    rhs = -b
    xs = np.linalg.solve(Ap, rhs)
    for k in range(1, 7):
        r = P.pcg(A, b, eta=1e-300, max_iter=k, pc="none", restarts=0)
        Kb = [rhs]
        for _ in range(k - 1):
            Kb.append(Ap @ Kb[-1])
        Q, _ = np.linalg.qr(np.stack(Kb, axis=1))
        xk = Q @ np.linalg.solve(Q.T @ Ap @ Q, Q.T @ rhs)
        assert np.linalg.norm(r.x - xk) <= 1e-9 * np.linalg.norm(xs), k


def test_jacobi_exact_on_diagonal_and_ic0_exact_on_tridiagonal():
    d = -np.linspace(1.0, 50.0, 40)
    A = sp.diags(d).tocsr()
    b = np.random.default_rng(0).standard_normal(40)
    r = P.pcg(A, b, eta=1e-14, pc="jacobi")
    assert r.iters == 1 and np.allclose(r.x, b / d, rtol=1e-14)
    # IC(0) of a tridiagonal SPD matrix has no fill: it is the exact Cholesky factor
    n = 30
    T = sp.diags([np.full(n - 1, 1.0), np.full(n, -3.0), np.full(n - 1, 1.0)], [-1, 0, 1]).tocsr()
    L = P.ic0(-T)
    assert np.allclose((L @ L.T).toarray(), (-T).toarray(), atol=1e-13)
    r = P.pcg(T, b[:n], eta=1e-13, pc="ic0")
    assert r.iters == 1


def test_ic0_matches_pattern():
    A, _ = _spd_problem(N=5)
    Ap = -sp.csr_matrix(A)
    L = P.ic0(Ap)
    LLt = (L @ L.T).toarray()
    mask = Ap.toarray() != 0
    assert np.allclose(LLt[mask], Ap.toarray()[mask], rtol=1e-12, atol=1e-9)
    assert np.all(np.triu(L.toarray(), 1) == 0)


# ------------------------------------------------------------------ extended Krylov
@pytest.fixture(scope="module")
def ek_small():
    op = fv3d(10, 1.0, 3)
    A = op.to_scipy()
    C = gaussian_C(op.n, 1, 3)
    r = E.lyap_ext(A, C, tol=1e-8)
    return op, A, C, r


def test_ek_against_dense_solution(ek_small):
    op, A, C, r = ek_small
    assert r.converged
    X = D.lyap_eig(A.toarray(), C)
    assert K.lowrank_vs_dense_error(r.Z, X) <= 1e-7
    # the cheap residual equals the explicit one (FP64, exact solves)
    ex = K.explicit_residual(A, r.Z, C) / r.beta ** 2
    assert ex <= 1.5e-8
    assert abs(ex - r.hist[-1]["res"]) <= 0.05 * ex + 1e-12


def test_ek_structure(ek_small):
    """T_m = V^T A V is block tridiagonal with 2s x 2s blocks, the lower s rows
    of tau_{m+1,m} vanish, A V_m = V_{m+1} T_m-underline, V orthonormal."""
    op, A, C, r = ek_small
    s = C.shape[1]
    ell = 2 * s
    T = r.T
    k = T.shape[0]
    i, j = np.indices((k, k))
    scale = np.abs(T).max()
    assert np.abs(np.where(np.abs(i - j) > ell, T, 0.0)).max() <= 1e-10 * scale
    assert np.abs(r.tau[s:, :]).max() <= 1e-9 * np.abs(r.tau).max()
    V = r.V
    Vm = V[:, :k]
    Tu = np.zeros((k + ell, k))
    Tu[:k] = T
    Tu[k:, k - ell:] = r.tau
    assert np.linalg.norm(A @ Vm - V @ Tu) <= 1e-10 * np.linalg.norm(A.toarray(), 2)
    assert np.linalg.norm(V.T @ V - np.eye(V.shape[1])) <= 1e-12


def test_ek_span_contains_both_directions(ek_small):
    """EK_m(A, C) contains A^{-j} C and A^{j} C for j < m: the start block and
    the W assembly put A^{-1} and A in the right halves."""
    op, A, C, r = ek_small
    k = 2 * C.shape[1] * r.m
    Vm = r.V[:, :k]
    lu = spla.splu(sp.csc_matrix(A))
    for v in (lu.solve(C), lu.solve(lu.solve(C)), A @ C, A @ (A @ C)):
        res = v - Vm @ (Vm.T @ v)
        assert np.linalg.norm(res) <= 1e-9 * np.linalg.norm(v)
    # planted mistake: a basis built with A in both halves misses A^{-1} C
    V1, _, _ = E.start_block(A, C, lambda B: A @ B)
    v = lu.solve(C)
    assert np.linalg.norm(v - V1 @ (V1.T @ v)) > 1e-3 * np.linalg.norm(v)


def test_ek_residual_three_ways(ek_small):
    """Proposition 1 with tau-bar (the paper's shortcut) = with the whole tau =
    the reduced-solution formula sqrt(2) ||Y E_m tau^T|| (eq. (reseq1))."""
    op, A, C, r = ek_small
    s = C.shape[1]
    ell = 2 * s
    Tb = E.band_of(r.T, ell)
    a = K.residual_alg3(Tb, r.gamma, r.tau[:s, :]).res
    b = K.residual_alg3(Tb, r.gamma, r.tau).res
    c = K.residual_reduced(r.T, r.gamma, r.tau)
    assert abs(a - b) <= 1e-8 * b
    assert abs(a - c) <= 1e-6 * c


def test_ek_diagonal_operator():
    """Diagonal A: X_ij = -(C C^T)_ij / (a_i + a_j) in closed form."""
    rng = np.random.default_rng(7)
    a = -np.sort(rng.uniform(1.0, 100.0, 300))
    A = sp.diags(a).tocsr()
    C = rng.standard_normal((300, 2))
    r = E.lyap_ext(A, C, tol=1e-10)
    assert r.converged
    X = D.lyap_diag(a, C)
    assert K.lowrank_vs_dense_error(r.Z, X) <= 1e-9


def test_ek_with_pcg_solves_matches_lu():
    """Inexact (certified 1e-12) PCG solves give the same iteration count and
    factor as exact solves."""
    op = fv3d(8, 1.0, 5)
    A = op.to_scipy()
    C = gaussian_C(op.n, 2, 5)
    r_lu = E.lyap_ext(A, C, tol=1e-8)
    solve = lambda B: P.pcg_block(A, B, eta=1e-12, pc="jacobi")[0]  # noqa: E731
    r_cg = E.lyap_ext(A, C, tol=1e-8, solve=solve)
    assert r_lu.m == r_cg.m
    assert K.factor_error(r_cg.Z, r_lu.Z) <= 1e-8


def test_ek_converges_faster_than_standard_on_laplacian():
    """On an ill-conditioned operator EK needs far fewer blocks (Section 4)."""
    op = laplace2d(40)
    A = op.to_scipy()
    C = gaussian_C(op.n, 1, 1)
    r_ek = E.lyap_ext(A, C, tol=1e-8)
    r_std = K.lyap_std(A, C, tol=1e-8)
    assert r_ek.converged and r_std.converged
    assert 2 * r_ek.m < r_std.m
