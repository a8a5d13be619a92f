"""Pins of the large-A / small-B oracle (Section 5.2): Algorithm 5 against the
reduced equation solved by SciPy's Bartels-Stewart and against the explicit
residual of X_m = V_m Y_m, the one-sided Galerkin condition, eq.
(formulaLargeAsmallB) against the same Bartels-Stewart Y_m, four planted
mistakes caught, convergence to the dense Sylvester solution, the scalar-B
case (a shifted linear system), two-pass = stored basis and the truncation
bound.  CPU."""
import numpy as np
import pytest
import scipy.linalg as sla

from workloads import fd1d_dense, fd2d_variable, laplace2d, gaussian_C, uniform_C
from oracle import krylov as K
from oracle import smallb as SB


def _spd_dense(n, seed, lo=1.0, hi=50.0):
    """-(Q diag(d) Q^T): a dense symmetric negative definite test matrix."""
    rng = np.random.default_rng([seed])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = lo + (hi - lo) * rng.random(n)
    return -(Q * d) @ Q.T


def _basis(A, C1, m):
    _, gamma1 = K.qr_pos(C1)
    V1 = K.right_solve_upper(C1, gamma1)
    prev, cur = np.zeros_like(V1), V1
    Vs, recs = [V1], []
    for _ in range(m):
        Vn, rec, _, _, _ = K.block_lanczos_step(A, prev, cur)
        recs.append(rec)
        prev, cur = cur, Vn
        Vs.append(Vn)
    return gamma1, Vs, recs


@pytest.fixture(scope="module")
def case():
    op = fd2d_variable(12, lambda x, y: np.exp(-x * y), lambda x, y: np.exp(x * y))
    A = op.to_scipy()
    B = fd1d_dense(7, 10.0)
    C1 = uniform_C(op.n, 2, 1)
    C2 = uniform_C(7, 2, 2)
    return A, B, C1, C2


def test_alg5_equals_reduced_and_explicit_residual(case):
    A, B, C1, C2 = case
    m = 6
    gamma1, Vs, recs = _basis(A, C1, m)
    T = K.assemble_T(recs, m)
    tau = recs[m - 1].R
    ups, P, G = SB.small_b_setup(B, C2, gamma1)
    a5 = SB.residual_alg5(T, tau, G, ups)
    Y = SB.reduced_solution(T, B, gamma1, C2)
    # eq. (reducedLargeASmallB) really is solved
    E1g = np.zeros((T.shape[0], C1.shape[1]))
    E1g[:2] = gamma1
    assert np.linalg.norm(T @ Y + Y @ B + E1g @ C2.T) <= 1e-12 * np.linalg.norm(Y) * np.linalg.norm(T)
    # ||R_m||_F = ||tau E_m^T Y_m||_F
    r_red = np.linalg.norm(tau @ Y[-2:, :])
    assert abs(a5.res - r_red) <= 1e-10 * r_red
    # explicit residual of X_m = V_m Y_m (n1 x n2 is small here)
    V = np.concatenate(Vs[:m], axis=1)
    X = V @ Y
    R = A @ X + X @ B + C1 @ C2.T
    r_ex = np.linalg.norm(R)
    assert abs(a5.res - r_ex) <= 1e-8 * r_ex
    # one-sided Galerkin condition V_m^T R_m = 0 (eq. (orthLargeAsmallB))
    assert np.linalg.norm(V.T @ R) <= 1e-10 * r_ex
    # eq. (formulaLargeAsmallB): Y_m = Q Y~ P^T
    Yf = a5.Q @ SB.ytilde(a5.lam, a5.Q, ups, G) @ P.T
    assert np.linalg.norm(Yf - Y) <= 1e-10 * np.linalg.norm(Y)


def _alg5_variant(T, tau, G, ups, mistake):
    ell = tau.shape[0]
    lam, Q = sla.eigh(T)
    S = G @ (Q[-ell:, :] if mistake == "E1_vs_Em" else Q[:ell, :])
    W = Q[-ell:, :].T @ (tau if mistake == "tau_not_transposed" else tau.T)
    acc = 0.0
    for i in range(ups.shape[0]):
        D = ups[i] - lam if mistake == "sign" else ups[i] + lam
        row = (S[i, :] / D) @ W
        acc += row @ row
    return np.sqrt(acc)


@pytest.mark.parametrize("mistake", ["E1_vs_Em", "tau_not_transposed", "sign", "no_gamma"])
def test_pins_catch_planted_mistakes(case, mistake):
    A, B, C1, C2 = case
    m = 6
    gamma1, _, recs = _basis(A, C1, m)
    T = K.assemble_T(recs, m)
    tau = recs[m - 1].R
    ups, P, G = SB.small_b_setup(B, C2, gamma1)
    r_red = np.linalg.norm(tau @ SB.reduced_solution(T, B, gamma1, C2)[-2:, :])
    assert abs(_alg5_variant(T, tau, G, ups, "none") - r_red) <= 1e-10 * r_red
    if mistake == "no_gamma":
        bad = _alg5_variant(T, tau, P.T @ C2, ups, "none")
    else:
        bad = _alg5_variant(T, tau, G, ups, mistake)
    assert abs(bad - r_red) > 1e-3 * r_red


def test_converges_to_dense_solution():
    op = laplace2d(10)
    A = op.to_scipy()
    B = _spd_dense(9, 3, 5.0, 400.0)
    C1 = gaussian_C(op.n, 3, 7)
    C2 = gaussian_C(9, 3, 8)
    r = SB.sylv_small_b(A, B, C1, C2, tol=1e-10)
    assert r.converged
    X = sla.solve_sylvester(A.toarray(), B, -(C1 @ C2.T))
    err = np.linalg.norm(r.Z1 @ r.Z2.T - X) / np.linalg.norm(X)
    assert err <= 1e-8
    R = A @ (r.Z1 @ r.Z2.T) + (r.Z1 @ r.Z2.T) @ B + C1 @ C2.T
    ex = np.linalg.norm(R) / (r.beta1 * r.beta2)
    assert ex <= 1.2e-10
    # the history decreases to the stop and the stop is the first passing check
    assert r.hist[-1]["res"] <= 1e-10 and all(h["res"] > 1e-10 for h in r.hist[:-1])


def test_scalar_b_is_a_shifted_linear_system():
    """n2 = 1: (A + b I) x = -C1 c2^T, the Galerkin solution of a single
    shifted system; at convergence the factor equals the direct solve."""
    op = laplace2d(12)
    A = op.to_scipy()
    b = -37.0
    C1 = gaussian_C(op.n, 1, 11)
    C2 = np.array([[0.5]])
    r = SB.sylv_small_b(A, np.array([[b]]), C1, C2, tol=1e-12)
    assert r.converged and r.t == 1
    x = -sla.solve(A.toarray() + b * np.eye(op.n), C1[:, 0] * 0.5)
    assert np.linalg.norm((r.Z1 @ r.Z2.T)[:, 0] - x) <= 1e-10 * np.linalg.norm(x)


def test_two_pass_equals_stored_and_truncation_bound(case):
    A, B, C1, C2 = case
    r1 = SB.sylv_small_b(A, B, C1, C2, tol=1e-9, two_pass=True)
    r2 = SB.sylv_small_b(A, B, C1, C2, tol=1e-9, two_pass=False)
    assert r1.m == r2.m and r1.t == r2.t
    X1 = r1.Z1 @ r1.Z2.T
    assert np.linalg.norm(X1 - r2.Z1 @ r2.Z2.T) <= 1e-12 * np.linalg.norm(X1)
    # the dropped singular values of Y~ have tail norm <= eps
    sv = r1.extra["sv"]
    assert np.sqrt(np.sum(sv[r1.t:] ** 2)) <= r1.extra["eps"]
    assert r1.t == len(sv) or np.sqrt(np.sum(sv[r1.t - 1:] ** 2)) > r1.extra["eps"]

