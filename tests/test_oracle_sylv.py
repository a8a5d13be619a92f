"""Pins of the Sylvester oracle (Section 5.1): the corrected Algorithm 4
against the reduced-solution formula (eq. (resSylv)) and the explicit
residual, the printed pairing of shifts shown to disagree, the Lyapunov
special case, the dense reference solution and the two-pass factors.  CPU."""
import numpy as np
import pytest

from workloads import fv3d, laplace2d, gaussian_C
from oracle import sylvester as Y
from oracle import dense as D
from oracle import krylov as K


@pytest.fixture(scope="module")
def case():
    A = laplace2d(14).to_scipy()
    B = fv3d(6, 0.5, 4).to_scipy()
    C1 = gaussian_C(A.shape[0], 2, 4)
    C2 = gaussian_C(B.shape[0], 2, 5)
    r = Y.sylv_std(A, B, C1, C2, tol=1e-9)
    return A, B, C1, C2, r


def test_sylv_against_dense(case):
    A, B, C1, C2, r = case
    assert r.converged
    X = D.sylv_eig(A.toarray(), B.toarray(), C1, C2)
    assert Y.lowrank_error(r.Z1, r.Z2, X) <= 1e-8
    ex = Y.explicit_residual(A, B, r.Z1, r.Z2, C1, C2) / (r.beta1 * r.beta2)
    assert abs(ex - r.hist[-1]["res"]) <= 0.02 * ex


def test_alg4_equals_reduced_formula_and_printed_differs(case):
    A, B, C1, C2, r = case
    # at an intermediate m, where the residual is far from zero
    m = 8
    s = C1.shape[1]
    rr = Y.sylv_std(A, B, C1, C2, tol=1e-30, max_iter=m + 1, check=lambda j: False)
    T = rr.T[:s * m, :s * m]
    J = rr.J[:s * m, :s * m]
    tau = rr.T[s * m:s * (m + 1), s * (m - 1):s * m] if rr.T.shape[0] > s * m else None
    assert tau is not None
    iota = rr.J[s * m:s * (m + 1), s * (m - 1):s * m]
    a = Y.residual_alg4(T, J, rr.gamma1, rr.gamma2, tau, iota).res
    b = Y.residual_reduced(T, J, rr.gamma1, rr.gamma2, tau, iota)
    p = Y.residual_alg4_printed(T, J, rr.gamma1, rr.gamma2, tau, iota)
    assert abs(a - b) <= 1e-9 * b
    assert abs(p - b) > 1e-3 * b


def test_explicit_residual_identity():
    """The factored residual norm equals the dense one."""
    rng = np.random.default_rng(3)
    A = laplace2d(6).to_scipy()
    B = fv3d(3, 0.5, 2).to_scipy()
    Z1 = rng.standard_normal((A.shape[0], 3))
    Z2 = rng.standard_normal((B.shape[0], 3))
    C1 = rng.standard_normal((A.shape[0], 2))
    C2 = rng.standard_normal((B.shape[0], 2))
    X = Z1 @ Z2.T
    dense = np.linalg.norm(A.toarray() @ X + X @ B.toarray() + C1 @ C2.T)
    assert abs(Y.explicit_residual(A, B, Z1, Z2, C1, C2) - dense) <= 1e-12 * dense


def test_lyapunov_special_case():
    """B = A, C2 = C1: the Sylvester iteration is the Lyapunov one, and both
    residual formulas coincide (two equal terms = sqrt(2) ||.||)."""
    A = laplace2d(12).to_scipy()
    C = gaussian_C(A.shape[0], 2, 1)
    rs = Y.sylv_std(A, A, C, C, tol=1e-8)
    rl = K.lyap_std(A, C, tol=1e-8)
    assert rs.m == rl.m
    for a, b in zip(rs.hist, rl.hist):
        assert abs(a["res"] - b["res"]) <= 1e-10 * b["res"]


def test_two_pass_equals_stored(case):
    A, B, C1, C2, r = case
    r2 = Y.sylv_std(A, B, C1, C2, tol=1e-9, two_pass=False)
    assert np.allclose(r.Z1 @ r.Z2.T, r2.Z1 @ r2.Z2.T, atol=1e-12 * np.abs(r2.Z1 @ r2.Z2.T).max())


def test_tsvd_error_bound(case):
    A, B, C1, C2, r = case
    from oracle import sylvester as S
    al = S.residual_alg4(r.T, r.J, r.gamma1, r.gamma2, r.tau, r.iota)
    Yt = -(al.g1 @ al.g2.T) / (al.lam[:, None] + al.ups[None, :])
    for eps in (1e-6, 1e-9, 1e-12):
        M1, M2, _ = S.tsvd_factors(al.lam, al.Q, al.ups, al.P, al.g1, al.g2, eps)
        approx = al.Q.T @ M1 @ (al.P.T @ M2).T
        assert np.linalg.norm(Yt - approx) <= eps * (1 + 1e-8)


# ------------------------------------------------------------------ extended spaces (Section 5.1 with Section 4)
@pytest.fixture(scope="module")
def ext_case():
    A = laplace2d(12).to_scipy()
    B = fv3d(5, 0.5, 4).to_scipy()
    C1 = gaussian_C(A.shape[0], 2, 14)
    C2 = gaussian_C(B.shape[0], 2, 15)
    return A, B, C1, C2


def test_sylv_ext_against_dense(ext_case):
    A, B, C1, C2 = ext_case
    r = Y.sylv_ext(A, B, C1, C2, tol=1e-9)
    assert r.converged
    X = D.sylv_eig(A.toarray(), B.toarray(), C1, C2)
    assert Y.lowrank_error(r.Z1, r.Z2, X) <= 1e-8
    ex = Y.explicit_residual(A, B, r.Z1, r.Z2, C1, C2) / (r.beta1 * r.beta2)
    assert ex <= 1.2e-9
    # extended spaces need fewer blocks than the standard ones on this pair
    assert r.m < Y.sylv_std(A, B, C1, C2, tol=1e-9).m


def test_sylv_ext_alg4_with_tau_bar_equals_reduced_and_explicit(ext_case):
    from oracle.extended import EKSide, band_of
    A, B, C1, C2 = ext_case
    s, m = 2, 4
    sa, sb = EKSide(A, C1), EKSide(B, C2)
    for _ in range(m):
        sa.step()
        sb.step()
    T, J = band_of(sa.T(), 2 * s), band_of(sb.T(), 2 * s)
    a4 = Y.residual_alg4(T, J, sa.gamma, sb.gamma, sa.tau()[:s, :], sb.tau()[:s, :])
    rr = Y.residual_reduced(T, J, sa.gamma, sb.gamma, sa.tau(), sb.tau())
    assert abs(a4.res - rr) <= 1e-8 * rr
    Yr = Y.reduced_solution(T, J, sa.gamma, sb.gamma)
    X = sa.Vm() @ Yr @ sb.Vm().T
    R = A @ X + X @ B + C1 @ C2.T
    assert abs(np.linalg.norm(R) - a4.res) <= 1e-7 * a4.res


def test_sylv_ext_lyapunov_special_case():
    from oracle.extended import lyap_ext
    A = laplace2d(12).to_scipy()
    C = gaussian_C(A.shape[0], 2, 16)
    r = Y.sylv_ext(A, A, C, C, tol=1e-9)
    q = lyap_ext(A, C, tol=1e-9)
    assert r.m == q.m
    Xq = q.Z @ q.Z.T
    assert np.linalg.norm(r.Z1 @ r.Z2.T - Xq) <= 1e-9 * np.linalg.norm(Xq)


def test_ek_side_matches_lyap_ext():
    from oracle.extended import EKSide, lyap_ext
    A = laplace2d(10).to_scipy()
    C = gaussian_C(A.shape[0], 1, 17)
    q = lyap_ext(A, C, tol=1e-30, max_iter=5, check=lambda j: False)
    e = EKSide(A, C)
    for _ in range(5):
        e.step()
    assert np.array_equal(e.T(), q.T) and np.array_equal(e.tau(), q.tau) and np.array_equal(e.gamma, q.gamma)
