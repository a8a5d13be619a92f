"""Pins of the generalized-Lyapunov oracle (A X E + E X A + C C^T = 0, E
symmetric positive definite; Section 6, Example 3): against a dense Kronecker
solve that does not use the Cholesky transformation, the factored explicit
residual against the dense one, E = I reducing to the standard run, the
E-inner-product block Lanczos recurrence (the form the GPU runs: basis W with
W^T E W = I, P = E W, one solve with E per step) giving the same T_m and
gamma as the transformed run, and planted mistakes caught.  CPU."""
import numpy as np
import pytest
import scipy.linalg as sla

from workloads import fe_p1_2d, gaussian_C
from oracle import generalized as G
from oracle import krylov as K


@pytest.fixture(scope="module")
def small():
    A, E = fe_p1_2d(6)            # n = 36
    return A.to_scipy(), E.to_scipy(), gaussian_C(A.n, 2, 3)


def test_against_kronecker_solution(small):
    A, E, C = small
    r = G.lyap_gen(A, E, C, tol=1e-12)
    assert r.std.converged
    X = G.lyap_gen_kron(A.toarray(), E.toarray(), C)
    assert np.linalg.norm(r.Z @ r.Z.T - X) <= 1e-9 * np.linalg.norm(X)


def test_explicit_residual_and_transformed_history():
    Ao, Eo = fe_p1_2d(12)          # n = 144: stops well before the space is complete
    A, E, C = Ao.to_scipy(), Eo.to_scipy(), gaussian_C(Ao.n, 2, 4)
    r = G.lyap_gen(A, E, C, tol=1e-7, check_every=1)
    assert r.std.converged and 2 * r.std.m < A.shape[0]
    Ad, Ed = A.toarray(), E.toarray()
    X = r.Z @ r.Z.T
    Rd = Ad @ X @ Ed + Ed @ X @ Ad + C @ C.T
    # both evaluations cancel O(||C||^2) terms down to the residual
    assert abs(G.explicit_residual(A, E, r.Z, C) - np.linalg.norm(Rd)) <= 1e-13 * np.linalg.norm(C) ** 2
    # the history is the residual of the transformed equation
    Li = sla.solve_triangular(r.L, np.eye(A.shape[0]), lower=True)
    Rt = Li @ Rd @ Li.T
    bt2 = np.linalg.norm(Li @ C) ** 2
    # (truncation moves it by at most 0.1 tol)
    assert abs(np.linalg.norm(Rt) / bt2 - r.std.hist[-1]["res"]) <= 0.02 * r.std.hist[-1]["res"] + 1e-8


def test_identity_mass_is_the_standard_run(small):
    A, E, C = small
    n = A.shape[0]
    r = G.lyap_gen(A, np.eye(n), C, tol=1e-9)
    s = K.lyap_std(A.toarray(), C, tol=1e-9)
    assert r.std.m == s.m
    assert np.linalg.norm(r.Z @ r.Z.T - s.Z @ s.Z.T) <= 1e-12 * np.linalg.norm(s.Z @ s.Z.T)


def _e_lanczos(A, E, C, m):
    """Block Lanczos for E^{-1} A in the E inner product (the GPU's form):
    U = E^{-1} A W_j, two sweeps of block MGS against W_{j-1}, W_j with
    alpha = P_i^T U (P_i = E W_i) and G = E U kept alongside, then the E-norm
    Cholesky QR twice.  Returns T_m (assembled like the standard run), gamma
    and the basis."""
    Ad, Ed = A.toarray(), E.toarray()
    U0 = np.linalg.solve(Ed, C)
    G0 = Ed @ U0
    g = np.linalg.cholesky(U0.T @ G0).T                  # upper, positive diagonal
    W = [sla.solve_triangular(g, U0.T, trans="T").T]
    P = [sla.solve_triangular(g, G0.T, trans="T").T]
    s = C.shape[1]
    Wp, Pp = np.zeros_like(W[0]), np.zeros_like(P[0])
    recs = []
    for j in range(m):
        U = np.linalg.solve(Ed, Ad @ W[j])
        Gm = Ed @ U
        alphas = []
        for _ in range(2):
            for Wi, Pi in ((Wp, Pp), (W[j], P[j])):
                a = Pi.T @ U
                U = U - Wi @ a
                Gm = Gm - Pi @ a
                alphas.append(a)
        R = np.eye(s)
        for _ in range(2):
            Gr = U.T @ Gm
            Rk = np.linalg.cholesky(0.5 * (Gr + Gr.T)).T
            U = sla.solve_triangular(Rk, U.T, trans="T").T
            Gm = sla.solve_triangular(Rk, Gm.T, trans="T").T
            R = Rk @ R
        recs.append(K.StepRecord(alphas, R))
        Wp, Pp = W[j], P[j]
        W.append(U)
        P.append(Gm)
    return K.assemble_T(recs, m), g, W


def test_e_inner_product_lanczos_equals_transformed(small):
    A, E, C = small
    m = 6
    T, g, W = _e_lanczos(A, E, C, m)
    At, Ct, L = G.transform(A, E, C)
    r = K.lyap_std(At, Ct, tol=1e-30, max_iter=m, check=lambda j: False, two_pass=False)
    assert np.linalg.norm(T - r.T) <= 1e-10 * np.linalg.norm(r.T)
    assert np.linalg.norm(g - r.gamma) <= 1e-12 * np.linalg.norm(r.gamma)
    Wm = np.concatenate(W[:m], axis=1)
    assert np.linalg.norm(Wm.T @ E.toarray() @ Wm - np.eye(Wm.shape[1])) <= 1e-10


@pytest.mark.parametrize("mistake", ["L_not_transposed", "C_untransformed", "mass_ignored"])
def test_planted_mistakes_caught(small, mistake):
    A, E, C = small
    X = G.lyap_gen_kron(A.toarray(), E.toarray(), C)
    At, Ct, L = G.transform(A, E, C)
    if mistake == "L_not_transposed":
        r = K.lyap_std(At, Ct, tol=1e-12)
        Z = sla.solve_triangular(L, r.Z, lower=True)
    elif mistake == "C_untransformed":
        r = K.lyap_std(At, C, tol=1e-12)
        Z = sla.solve_triangular(L.T, r.Z, lower=False)
    else:
        r = K.lyap_std(A.toarray(), C, tol=1e-12)
        Z = r.Z
    assert np.linalg.norm(Z @ Z.T - X) > 1e-3 * np.linalg.norm(X)
