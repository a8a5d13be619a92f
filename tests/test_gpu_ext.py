"""GPU parity of the extended Krylov path and its inner PCG (through the C
ABI) against the CPU FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

from workloads import laplace2d, fv3d, gaussian_C
from oracle import extended as E
from oracle import krylov as K
from oracle import dense as D
from oracle import pcg as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _b():
    from paper_1602_05033_amd import binding
    return binding


def _dev(C):
    return torch.from_numpy(np.ascontiguousarray(C)).cuda()


# ------------------------------------------------------------------ inner PCG
@pytest.mark.parametrize("N,s,pc", [(9, 1, "jacobi"), (12, 2, "jacobi"), (10, 4, "jacobi"), (9, 1, "none"),
                                    (17, 1, "jacobi")])
def test_inner_pcg_parity(lib, N, s, pc):
    b = _b()
    op = fv3d(N, 1.0, 3)
    A = op.to_scipy()
    B = gaussian_C(op.n, s, 9)
    dop = b.device_op(op)
    pcc = b.PC_JACOBI if pc == "jacobi" else b.PC_NONE
    X, iters, rel, st = b.inner_solve(dop, _dev(B), inner_pc=pcc, inner_tol=1e-12)
    assert st == b.OK and rel <= 1e-12
    Xh = X.cpu().numpy()
    ref, res = P.pcg_block(A, B, eta=1e-12, pc=pc)
    for c in range(s):
        assert np.linalg.norm(A @ Xh[:, c] - B[:, c]) <= 1e-12 * np.linalg.norm(B[:, c])
        assert np.linalg.norm(Xh[:, c] - ref[:, c]) <= 1e-9 * np.linalg.norm(ref[:, c])
    # columns advance together: the GPU count is the slowest column's, within
    # one iteration of the oracle's (recursive target eta/2 vs eta)
    assert abs(iters - max(r.iters for r in res)) <= max(3, 0.05 * iters), (iters, [r.iters for r in res])


def test_inner_pcg_ragged_and_stencil5(lib):
    """n not a multiple of any tile, 5-point operator, CSR copy of the same."""
    b = _b()
    op = laplace2d(53, shift=2.0)
    A = op.to_scipy()
    B = gaussian_C(op.n, 2, 4)
    for csr in (False, True):
        dop = b.device_op(op, as_csr=csr)
        X, iters, rel, st = b.inner_solve(dop, _dev(B), inner_pc=b.PC_JACOBI)
        Xh = X.cpu().numpy()
        for c in range(2):
            assert np.linalg.norm(A @ Xh[:, c] - B[:, c]) <= 1e-12 * np.linalg.norm(B[:, c])


def test_inner_pcg_not_converged_reports(lib):
    b = _b()
    op = fv3d(12, 1.0, 3)
    B = gaussian_C(op.n, 1, 9)
    dop = b.device_op(op)
    X, iters, rel, st = b.inner_solve(dop, _dev(B), raise_on_error=False, inner_pc=b.PC_JACOBI, inner_max_iter=5)
    assert st == b.E_INNER and rel > 1e-12 and iters == 5


def test_inner_pcg_zero_rhs(lib):
    b = _b()
    op = fv3d(6, 1.0, 3)
    dop = b.device_op(op)
    B = np.zeros((op.n, 2))
    B[:, 1] = gaussian_C(op.n, 1, 2)[:, 0]
    X, iters, rel, st = b.inner_solve(dop, _dev(B))
    assert st == b.OK
    Xh = X.cpu().numpy()
    assert np.all(Xh[:, 0] == 0.0)
    A = op.to_scipy()
    assert np.linalg.norm(A @ Xh[:, 1] - B[:, 1]) <= 1e-12 * np.linalg.norm(B[:, 1])


def test_inner_pcg_unsupported_pc(lib):
    b = _b()
    op = fv3d(5, 1.0, 3)
    dop = b.device_op(op)
    B = gaussian_C(op.n, 1, 2)
    with pytest.raises(b.LyapError):
        b.inner_solve(dop, _dev(B), inner_pc=7)          # no such preconditioner
    with pytest.raises(b.LyapError):
        b.inner_solve(dop, _dev(B), inner_pc=b.PC_LEARNED)  # trained only inside an EK solve


# ------------------------------------------------------------------ extended Krylov
def _ek_case(op, s, seed, tol=1e-8):
    b = _b()
    A = op.to_scipy()
    C = gaussian_C(op.n, s, seed)
    dop = b.device_op(op)
    sol = b.lyap_solve(dop, _dev(C), method=b.METHOD_EXT, tol=tol, check_every=1, want_T=True)
    ref = E.lyap_ext(A, C, tol=tol)
    return A, C, sol, ref


@pytest.mark.parametrize("N,s", [(10, 1), (12, 2), (9, 4), (16, 1)])
def test_ek_parity_fv3d(lib, N, s):
    op = fv3d(N, 1.0, 3)
    A, C, sol, ref = _ek_case(op, s, 3)
    assert sol.status == 0 and ref.converged
    assert sol.m == ref.m, (sol.m, ref.m)
    # residual histories (same check points)
    assert sol.hist_m == [h["m"] for h in ref.hist]
    for g, r in zip(sol.hist_res, ref.hist):
        assert abs(g - r["res"]) <= 1e-5 * r["res"] + 1e-13
    Z = sol.Z.cpu().numpy()
    X = D.lyap_eig(A.toarray(), C)
    assert K.lowrank_vs_dense_error(Z, X) <= 1e-7
    assert K.factor_error(Z, ref.Z) <= 1e-7
    assert K.explicit_residual(A, Z, C) / sol.beta ** 2 <= 1.2e-8
    # T_m: early blocks entrywise (band storage), tau-bar, gamma
    ell = 2 * s
    k = ell * sol.m
    Tb = sol.T_band
    Tref = E.band_of(ref.T, ell)
    for c in range(min(k, 3 * ell)):
        for d in range(ell + 1):
            if c + d < k:
                assert abs(Tb[c, d] - Tref[c + d, c]) <= 1e-9 * np.abs(ref.T).max()
    assert np.allclose(sol.gamma[:, :s], ref.gamma, rtol=0, atol=1e-12 * np.abs(ref.gamma).max())
    assert np.all(sol.gamma[:, s:] == 0.0)
    assert sol.n_inner == sol.m + 1 and sol.inner_iters > 0


def test_ek_parity_laplace_csr(lib):
    """2D Laplacian through the CSR path and through the stencil path."""
    b = _b()
    op = laplace2d(30)
    A = op.to_scipy()
    C = gaussian_C(op.n, 2, 1)
    ref = E.lyap_ext(A, C, tol=1e-9)
    X = D.lyap_eig(A.toarray(), C)
    for csr in (False, True):
        dop = b.device_op(op, as_csr=csr)
        sol = b.lyap_solve(dop, _dev(C), method=b.METHOD_EXT, tol=1e-9, check_every=1)
        assert sol.status == 0 and sol.m == ref.m
        Z = sol.Z.cpu().numpy()
        assert K.lowrank_vs_dense_error(Z, X) <= 1e-7
        assert K.factor_error(Z, ref.Z) <= 1e-7


def test_ek_adaptive_schedule(lib):
    b = _b()
    op = fv3d(14, 1.0, 3)
    A = op.to_scipy()
    C = gaussian_C(op.n, 1, 3)
    dop = b.device_op(op)
    sol = b.lyap_solve(dop, _dev(C), method=b.METHOD_EXT, tol=1e-8, check_every=0)
    ref = E.lyap_ext(A, C, tol=1e-8)
    assert sol.status == 0
    assert ref.m <= sol.m <= ref.m + 5
    Z = sol.Z.cpu().numpy()
    assert K.explicit_residual(A, Z, C) / sol.beta ** 2 <= 1.2e-8


def test_ek_errors(lib):
    b = _b()
    op = fv3d(6, 1.0, 3)
    dop = b.device_op(op)
    C = _dev(gaussian_C(op.n, 3, 3))
    with pytest.raises(b.LyapError):
        b.lyap_solve(dop, C, method=b.METHOD_EXT)          # s = 3 not built
    C1 = _dev(gaussian_C(op.n, 1, 3))
    with pytest.raises(b.LyapError):
        b.lyap_solve(dop, C1, method=b.METHOD_EXT, storage=b.STORE_F32)
    Cz = torch.zeros((op.n, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(b.LyapError):
        b.lyap_solve(dop, Cz, method=b.METHOD_EXT)
    # max_iter reached: NOT_CONVERGED with a history
    sol = b.lyap_solve(dop, C1, method=b.METHOD_EXT, tol=1e-14, max_iter=3, raise_on_error=False)
    assert sol.status == b.NOT_CONVERGED and sol.m == 3 and sol.Z is not None


def test_ek_lucky_breakdown_eigenvector(lib):
    """C an eigenvector of A: [C, A^{-1} C] is rank one, reported as breakdown."""
    b = _b()
    op = laplace2d(12)
    N = 12
    x = np.arange(1, N + 1) / (N + 1)
    v = np.outer(np.sin(np.pi * x), np.sin(np.pi * x)).reshape(-1)[:, None]
    dop = b.device_op(op)
    sol = b.lyap_solve(dop, _dev(v), method=b.METHOD_EXT, raise_on_error=False)
    assert sol.status == b.E_BREAKDOWN


def _explicit_residual_gpu(b, dop, Z, C):
    """||A Z Z^T + Z Z^T A + C C^T||_F from a QR of [AZ, Z, C] (FP64, torch on the device)."""
    n, t = Z.shape
    AZ = torch.empty_like(Z)
    for c0 in range(0, t, 8):
        AZ[:, c0:c0 + 8] = b.op_apply(dop, Z[:, c0:c0 + 8].contiguous(), b.STORE_F64)
    P = torch.cat([AZ, Z, C], dim=1)
    R = torch.linalg.qr(P, mode="r")[1]
    s = C.shape[1]
    Phi = torch.zeros(2 * t + s, 2 * t + s, dtype=torch.float64, device=Z.device)
    Phi[:t, t:2 * t] = torch.eye(t, dtype=torch.float64, device=Z.device)
    Phi[t:2 * t, :t] = torch.eye(t, dtype=torch.float64, device=Z.device)
    Phi[2 * t:, 2 * t:] = torch.eye(s, dtype=torch.float64, device=Z.device)
    return float(torch.linalg.norm(R @ Phi @ R.T))


def test_ek_full_size_100cubed(lib):
    """The full-size extended Krylov configuration: 100^3 cells, lognormal k
    (sigma 1), s = 1, n = 1e6, the launch configuration bench.py times.  The
    oracle cannot run here, so: convergence by Proposition 1, the explicit
    FP64 residual of the returned Z agrees with it, T_m is banded symmetric
    negative definite (Ritz values < 0) and every inner solve was certified."""
    b = _b()
    op = fv3d(100, 1.0, 3)
    C = gaussian_C(op.n, 1, 3)
    dop = b.device_op(op)
    Cd = _dev(C)
    sol = b.lyap_solve(dop, Cd, method=b.METHOD_EXT, tol=1e-8, check_every=0, inner_pc=b.PC_JACOBI,
                       inner_tol=1e-12, want_T=True)
    assert sol.status == b.OK and sol.res <= 1e-8
    assert 30 <= sol.m <= 70 and sol.n_inner == sol.m + 1
    ex = _explicit_residual_gpu(b, dop, sol.Z, Cd) / sol.beta ** 2
    assert ex <= 1.2e-8, ex
    # T_m symmetric negative definite: dense from the band
    k = sol.T_band.shape[0]
    ell = sol.T_band.shape[1] - 1
    T = np.zeros((k, k))
    for c in range(k):
        for d in range(ell + 1):
            if c + d < k:
                T[c + d, c] = T[c, c + d] = sol.T_band[c, d]
    assert np.linalg.eigvalsh(T).max() < 0.0


def test_ek_full_size_learned_preconditioner(lib):
    """The full-size extended Krylov configuration with the learned inner
    preconditioner (a correction of red-black IC(0) trained in the run): same
    acceptance as with IC(0), every inner solve certified, fewer inner
    iterations than IC(0) itself and than Jacobi."""
    b = _b()
    op = fv3d(100, 1.0, 3)
    C = gaussian_C(op.n, 1, 3)
    dop = b.device_op(op)
    Cd = _dev(C)
    sol = b.lyap_solve(dop, Cd, method=b.METHOD_EXT, tol=1e-8, check_every=0, inner_pc=b.PC_LEARNED,
                       inner_tol=1e-12)
    assert sol.status == b.OK and sol.res <= 1e-8
    ex = _explicit_residual_gpu(b, dop, sol.Z, Cd) / sol.beta ** 2
    assert ex <= 1.2e-8, ex
    ic0 = b.lyap_solve(dop, Cd, method=b.METHOD_EXT, tol=1e-8, check_every=0, inner_pc=b.PC_IC0, inner_tol=1e-12)
    jac = b.lyap_solve(dop, Cd, method=b.METHOD_EXT, tol=1e-8, check_every=0, inner_pc=b.PC_JACOBI, inner_tol=1e-12)
    assert abs(sol.m - ic0.m) <= 2 and abs(sol.m - jac.m) <= 2
    print(f"inner iterations: learned {sol.inner_iters}, IC(0) {ic0.inner_iters}, Jacobi {jac.inner_iters}")
    assert sol.inner_iters < 0.5 * ic0.inner_iters and ic0.inner_iters < jac.inner_iters
