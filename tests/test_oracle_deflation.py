"""Pins of the oracle's deflation of a rank-deficient start block (standard
and extended Krylov).  The paper assumes C has full column rank and leaves
deflation to the customary practice of block methods; the reading taken is
C -> C_r = C W_r with r the number of eigenvalues of C^T C above
10 n eps lambda_max (eps = 2^-52).  What pins it, independently of the
oracle's own code:

* the dense solution of A X + X A + C C^T = 0 (sine-transform eigenbasis or
  eigendecomposition), which depends on C only through C C^T;
* a rank-one C with s = 4 gives the run of s = 1 on the one direction;
* the undeflated route (a QR of the dependent block) does not give an
  orthonormal start block, and the planted misreadings (U_r without Sigma_r,
  a threshold on sigma instead of sigma^2) change the answer or the rank.
"""
import numpy as np
import pytest

from workloads import laplace2d, gaussian_C
from oracle import dense as D
from oracle import krylov as K
from oracle import extended as E


def _dependent_C(n, seed=5):
    c = gaussian_C(n, 2, seed)
    return np.stack([c[:, 0], c[:, 1], c[:, 0] + 2.0 * c[:, 1]], axis=1)


def test_numerical_rank_reading():
    n = 576
    C = _dependent_C(n)
    assert K.numerical_rank(C) == 2
    assert K.numerical_rank(1e-150 * C) == 2 and K.numerical_rank(1e150 * C) == 2
    assert K.numerical_rank(np.zeros((n, 3))) == 0
    g = gaussian_C(n, 3, 6)
    assert K.numerical_rank(g) == 3
    # sigma_3 / sigma_1 = 1e-8: a Gram matrix cannot resolve it
    # (lambda_3 / lambda_1 = 1e-16 < 10 n eps), a threshold on sigma would keep it
    U, _ = np.linalg.qr(g)
    Ct = U * np.array([1.0, 0.5, 1e-8])[None, :]
    assert K.numerical_rank(Ct) == 2
    assert np.sum(np.linalg.svd(Ct, compute_uv=False) > 10 * n * np.finfo(float).eps) == 3
    # 1e-4 is kept
    assert K.numerical_rank(U * np.array([1.0, 0.5, 1e-4])[None, :]) == 3


def test_deflated_columns_keep_CCt():
    C = _dependent_C(400)
    Cr = K.deflate_columns(C)
    assert Cr.shape == (400, 2)
    P, Q = C @ C.T, Cr @ Cr.T
    assert np.abs(P - Q).max() <= 1e-13 * np.abs(P).max()
    # full rank: returned as is
    g = gaussian_C(400, 3, 1)
    assert K.deflate_columns(g) is g
    with pytest.raises(ValueError):
        K.deflate_columns(np.zeros((400, 2)))


def test_undeflated_start_block_is_not_orthonormal():
    """The QR route on a dependent block: the third column of V_1 is rounding
    noise divided by a tiny R_33, not a unit vector orthogonal to the rest."""
    C = _dependent_C(400)
    _, R = K.qr_pos(C)
    assert R[2, 2] <= 1e-12 * R[0, 0]
    V = K.right_solve_upper(C, R)
    Cr = K.deflate_columns(C)
    _, Rr = K.qr_pos(Cr)
    Vr = K.right_solve_upper(Cr, Rr)
    assert np.abs(Vr.T @ Vr - np.eye(2)).max() <= 1e-13
    # the deflated start spans the columns of C
    assert np.linalg.norm(C - Vr @ (Vr.T @ C)) <= 1e-13 * np.linalg.norm(C)
    del V  # its orthogonality is not guaranteed: nothing built on it is used


@pytest.mark.parametrize("dep", ["linear", "repeated"])
def test_std_dependent_columns_against_dense(dep):
    """24 x 24 Laplacian; C with dependent columns, s = 3 (r = 2) or s = 4
    (one column repeated twice, r = 2)."""
    N = 24
    op = laplace2d(N)
    A = op.to_scipy()
    if dep == "linear":
        C = _dependent_C(op.n)
    else:
        c = gaussian_C(op.n, 2, 8)
        C = np.stack([c[:, 0], c[:, 1], c[:, 0], -c[:, 1]], axis=1)
    r = K.lyap_std(A, C, tol=1e-10, check_every=1, compute_dense_residual=True)
    assert r.converged and r.gamma.shape == (2, 2)
    assert abs(r.beta - np.linalg.norm(C)) <= 1e-15 * r.beta
    X = D.lyap_laplace2d_dense(N, C)
    assert K.lowrank_vs_dense_error(r.Z, X) <= 1e-8
    assert K.explicit_residual(A, r.Z, C) / r.beta ** 2 <= 1.1e-10
    last = r.hist[-1]
    # Proposition 1 and the reduced residual agree to rounding (relative to beta^2)
    assert abs(last["res"] - last["res_reduced"]) <= 1e-14


def test_rank_one_block_equals_single_column_run():
    """C = c a^T with a in R^4: C C^T = |a|^2 c c^T, so the run is the s = 1
    run on |a| c (same m, residual history and Z Z^T)."""
    N = 20
    op = laplace2d(N)
    A = op.to_scipy()
    c = gaussian_C(op.n, 1, 4)
    a = np.array([1.0, -2.0, 0.5, 3.0])
    C = c @ a[None, :]
    r4 = K.lyap_std(A, C, tol=1e-9, check_every=1)
    r1 = K.lyap_std(A, np.linalg.norm(a) * c, tol=1e-9, check_every=1)
    assert r4.gamma.shape == (1, 1)
    assert r4.m == r1.m
    for h4, h1 in zip(r4.hist, r1.hist):
        assert abs(h4["res"] - h1["res"]) <= 1e-14  # rounding, relative to beta^2
    assert K.factor_error(r4.Z, r1.Z) <= 1e-12


@pytest.mark.parametrize("mistake", ["no_sigma", "sigma_threshold"])
def test_deflation_pins_catch_planted_mistakes(mistake):
    N = 16
    op = laplace2d(N)
    C = _dependent_C(op.n)
    X = D.lyap_laplace2d_dense(N, C)
    U, sv, Wt = np.linalg.svd(C, full_matrices=False)
    if mistake == "no_sigma":
        # C_r = U_r: the right subspace but the wrong weights
        Cr = U[:, :2]
        Z = K.lyap_std(op.to_scipy(), Cr, tol=1e-10, check_every=1).Z
        assert K.lowrank_vs_dense_error(Z, X) > 1e-2
    else:
        g = gaussian_C(op.n, 3, 6)
        Q, _ = np.linalg.qr(g)
        Ct = Q * np.array([1.0, 0.5, 1e-8])[None, :]
        lam = np.linalg.svd(Ct, compute_uv=False)
        r_sigma = int(np.sum(lam > 10 * op.n * np.finfo(float).eps * lam[0]))
        assert r_sigma != K.numerical_rank(Ct)


def test_zero_C_raises():
    op = laplace2d(8)
    with pytest.raises(ValueError):
        K.lyap_std(op.to_scipy(), np.zeros((op.n, 2)))
    with pytest.raises(ValueError):
        E.lyap_ext(op.to_scipy(), np.zeros((op.n, 2)))


def test_ext_dependent_columns_against_dense():
    """Extended Krylov, s = 4 with r = 2 (ell = 4 after deflation), 20 x 20
    Laplacian with a shift, against the dense solution."""
    N = 20
    op = laplace2d(N, shift=3.0)
    A = op.to_scipy()
    c = gaussian_C(op.n, 2, 12)
    C = np.stack([c[:, 0], c[:, 1], c[:, 0] - c[:, 1], 3.0 * c[:, 1]], axis=1)
    r = E.lyap_ext(A, C, tol=1e-10, check_every=1)
    assert r.converged and r.gamma.shape == (4, 2)
    X = D.lyap_eig(A.toarray(), C)
    assert K.lowrank_vs_dense_error(r.Z, X) <= 1e-8
    # equals the run on the two independent directions it spans
    r2 = E.lyap_ext(A, K.deflate_columns(C), tol=1e-10, check_every=1)
    assert r2.m == r.m and K.factor_error(r.Z, r2.Z) <= 1e-12
