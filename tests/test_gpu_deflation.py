"""GPU parity of the deflated start block (a C with dependent columns) through
the C ABI, against the CPU FP64 oracle on the same seeded inputs.

The rank is the number of eigenvalues of C^T C above 10 n eps lambda_max
(eps = 2^-52); the solve runs on C W_r (r columns).  The oracle deflates with
the SVD (U_r Sigma_r = C W_r), so the two start blocks differ by an
orthogonal r x r factor: m, the residual history and Z Z^T agree, V_1 and
T_m need not."""
import numpy as np
import pytest

from workloads import laplace2d, fv3d, gaussian_C
from oracle import krylov as K
from oracle import extended as E
from oracle import dense as D

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _b():
    from paper_1602_05033_amd import binding
    return binding


def _dev(C):
    return torch.from_numpy(np.ascontiguousarray(C)).cuda()


def _dependent(n, kind, seed):
    c = gaussian_C(n, 2, seed)
    if kind == "linear":          # s = 3, r = 2
        return np.stack([c[:, 0], c[:, 1], c[:, 0] + 2.0 * c[:, 1]], axis=1)
    if kind == "repeated":        # s = 4, r = 2
        return np.stack([c[:, 0], c[:, 1], c[:, 0], -c[:, 1]], axis=1)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["linear", "repeated"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_std_dependent_columns_parity(lib, kind, storage):
    b = _b()
    N = 24
    op = laplace2d(N)
    A = op.to_scipy()
    C = _dependent(op.n, kind, 5)
    tol = 1e-10 if storage == "f64" else 1e-7
    print(f"std deflation {kind} {storage}", flush=True)
    sol = b.lyap_solve(b.device_op(op), _dev(C), tol=tol, check_every=1,
                       storage=b.STORE_F64 if storage == "f64" else b.STORE_F32)
    ref = K.lyap_std(A, C, tol=tol, check_every=1)
    assert sol.status == b.OK and sol.s == 2 and sol.ell == 2
    assert abs(sol.beta - ref.beta) <= 1e-13 * ref.beta
    Z = sol.Z.cpu().numpy()
    X = D.lyap_laplace2d_dense(N, C)
    if storage == "f64":
        assert sol.m == ref.m
        gh, oh = np.array(sol.hist_res), np.array([h["res"] for h in ref.hist])
        # relative 1e-6, and rounding at the 1e-14 beta^2 level
        assert len(gh) == len(oh)
        assert np.all(np.abs(gh - oh) <= 1e-6 * oh + 1e-14), np.max(np.abs(gh - oh) / oh)
        assert K.factor_error(Z, ref.Z) <= 1e-9
        assert K.lowrank_vs_dense_error(Z, X) <= 1e-8
        assert K.explicit_residual(A, Z, C) / sol.beta ** 2 <= 1.2e-10
    else:
        assert abs(sol.m - ref.m) <= 1
        assert K.lowrank_vs_dense_error(Z, X) <= 1e-5
        assert K.explicit_residual(A, Z, C) / sol.beta ** 2 <= 1e-6


def test_rank_one_block_equals_single_column_run(lib):
    """C = c a^T (s = 4, rank one) runs as s = 1 on |a| c."""
    b = _b()
    op = laplace2d(40)
    c = gaussian_C(op.n, 1, 4)
    a = np.array([1.0, -2.0, 0.5, 3.0])
    dop = b.device_op(op)
    s4 = b.lyap_solve(dop, _dev(c @ a[None, :]), tol=1e-9, check_every=1)
    s1 = b.lyap_solve(dop, _dev(np.linalg.norm(a) * c), tol=1e-9, check_every=1)
    assert s4.status == b.OK and s4.s == 1
    assert s4.m == s1.m
    h4, h1 = np.array(s4.hist_res), np.array(s1.hist_res)
    assert np.all(np.abs(h4 - h1) <= 1e-8 * h1 + 1e-14), np.max(np.abs(h4 - h1) / h1)
    assert K.factor_error(s4.Z.cpu().numpy(), s1.Z.cpu().numpy()) <= 1e-10


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_std_deflation_wide_block_large_grid(lib, storage):
    """300 x 300 Laplacian (n = 90000, several tiles and a ragged tail), s = 8
    with three dependent columns (r = 5, the 256-thread kernels): the same run
    as the full-rank s = 5 solve on the oracle's deflated columns, and the
    explicit residual against the original C."""
    b = _b()
    op = laplace2d(300)
    g = gaussian_C(op.n, 5, 7)
    C = np.concatenate([g, g[:, :3] @ np.array([[1.0, 0.0, -1.0], [2.0, 1.0, 0.0], [0.0, 3.0, 1.0]])], axis=1)
    Cr = K.deflate_columns(C)
    assert Cr.shape[1] == 5
    dop = b.device_op(op)
    st = b.STORE_F64 if storage == "f64" else b.STORE_F32
    tol = 1e-8 if storage == "f64" else 1e-6
    print(f"std deflation s=8 r=5 {storage}", flush=True)
    sol = b.lyap_solve(dop, _dev(C), tol=tol, check_every=5, storage=st)
    ref = b.lyap_solve(dop, _dev(Cr), tol=tol, check_every=5, storage=st)
    assert sol.status == b.OK and ref.status == b.OK and sol.s == 5
    assert sol.m == ref.m
    gh, rh = np.array(sol.hist_res), np.array(ref.hist_res)
    rel = 1e-6 if storage == "f64" else 1e-3
    assert np.all(np.abs(gh - rh) <= rel * rh + 1e-14), np.max(np.abs(gh - rh) / rh)
    Z, Zr = sol.Z.cpu().numpy(), ref.Z.cpu().numpy()
    assert K.factor_error(Z, Zr) <= (1e-8 if storage == "f64" else 1e-4)
    expl = K.explicit_residual(op.to_scipy(), Z, C) / sol.beta ** 2
    assert expl <= (1.2 * tol if storage == "f64" else 1e-5)


@pytest.mark.parametrize("scale,r", [(1e-8, 2), (1e-4, 3)])
def test_rank_threshold_on_gram_eigenvalues(lib, scale, r):
    """sigma_3 / sigma_1 = 1e-8 is below what the Gram matrix resolves
    (dropped); 1e-4 is kept."""
    b = _b()
    op = laplace2d(24)
    U, _ = np.linalg.qr(gaussian_C(op.n, 3, 6))
    C = U * np.array([1.0, 0.5, scale])[None, :]
    assert K.numerical_rank(C) == r
    sol = b.lyap_solve(b.device_op(op), _dev(C), tol=1e-9, check_every=1)
    assert sol.status == b.OK and sol.s == r
    X = D.lyap_laplace2d_dense(24, C)
    assert K.lowrank_vs_dense_error(sol.Z.cpu().numpy(), X) <= 1e-8


def test_ext_dependent_columns_parity(lib):
    """Extended Krylov, s = 4 with r = 2 (ell = 4), finite-volume 3D operator,
    against the oracle's run (exact solves) and the dense solution."""
    b = _b()
    op = fv3d(10, 1.0, 3)
    A = op.to_scipy()
    c = gaussian_C(op.n, 2, 12)
    C = np.stack([c[:, 0], c[:, 1], c[:, 0] - c[:, 1], 3.0 * c[:, 1]], axis=1)
    print("ext deflation s=4 r=2", flush=True)
    sol = b.lyap_solve(b.device_op(op), _dev(C), method=b.METHOD_EXT, tol=1e-9, check_every=1)
    ref = E.lyap_ext(A, C, tol=1e-9)
    assert sol.status == b.OK and sol.s == 2 and sol.ell == 4
    assert sol.m == ref.m
    for g, h in zip(sol.hist_res, ref.hist):
        assert abs(g - h["res"]) <= 1e-5 * h["res"] + 1e-13
    Z = sol.Z.cpu().numpy()
    assert K.factor_error(Z, ref.Z) <= 1e-7
    assert K.lowrank_vs_dense_error(Z, D.lyap_eig(A.toarray(), C)) <= 1e-7


def test_ext_deflated_rank_not_built(lib):
    """Rank 3 out of 4 columns: the extended kernels take 1, 2 or 4 columns."""
    b = _b()
    op = fv3d(6, 1.0, 3)
    g = gaussian_C(op.n, 3, 2)
    C = np.concatenate([g, g[:, :1] - g[:, 2:3]], axis=1)
    sol = b.lyap_solve(b.device_op(op), _dev(C), method=b.METHOD_EXT, raise_on_error=False)
    assert sol.status == b.E_UNSUPPORTED


def test_zero_C_is_an_argument_error(lib):
    b = _b()
    op = laplace2d(16)
    sol = b.lyap_solve(b.device_op(op), torch.zeros((op.n, 3), dtype=torch.float64, device="cuda"),
                       raise_on_error=False)
    assert sol.status == b.E_ARG
