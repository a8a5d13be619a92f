"""GPU parity of the inner solver with red-black IC(0) (run on the GPU in its
condensed form: CG on the black Schur complement preconditioned by its
diagonal) against the CPU FP64 oracle on the same seeded inputs, and of the
extended Krylov method driven by it.

The oracle's condensed form (``oracle.pcg.schur_rb_cg``) is the same
iteration as the GPU's; its red-black IC(0)-PCG on the whole grid
(``pc="ic0_rb"``) reaches the same solution within one iteration of it
(pinned in tests/test_oracle_ic0.py).  The GPU stops its recursion at half
the requested tolerance (so that the true residual passes), so the oracle is
run with eta / 2."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import laplace2d, fv3d, fd2d_variable, gaussian_C
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


def _grid(op):
    return (op.nx, op.ny, op.nz if op.kind == "stencil7" else 1)


CASES = {
    "fv3d_12": (lambda: fv3d(12, 1.0, 3), 1),
    "fv3d_11x10x9_odd": (lambda: fv3d(11, 1.0, 7, Ny=10, Nz=9), 2),
    "fv3d_10_s4": (lambda: fv3d(10, 1.0, 3), 4),
    "laplace2d_30": (lambda: laplace2d(30), 1),
    "laplace2d_31_shift": (lambda: laplace2d(31, shift=0.5), 2),
    "fd2d_variable_25": (lambda: fd2d_variable(25, lambda x, y: np.exp(-x * y), lambda x, y: np.exp(x * y)), 1),
    "fv3d_7x5x1_plane": (lambda: fv3d(7, 1.0, 2, Ny=5, Nz=1), 4),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_ic0_parity(lib, case):
    make, s = CASES[case]
    b = _b()
    op = make()
    A = op.to_scipy()
    B = gaussian_C(op.n, s, 9)
    print(f"case {case} n={op.n} s={s}", flush=True)
    X, iters, rel, st = b.inner_solve(b.device_op(op), _dev(B), inner_pc=b.PC_IC0, inner_tol=1e-12)
    assert st == b.OK and rel <= 1e-12
    Xh = X.cpu().numpy()
    lu = spla.splu(sp.csc_matrix(A))
    cond_its, full_its = [], []
    for c in range(s):
        x_ref = lu.solve(B[:, c])
        assert np.linalg.norm(A @ Xh[:, c] - B[:, c]) <= 1e-12 * np.linalg.norm(B[:, c])
        assert np.linalg.norm(Xh[:, c] - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
        cond = P.schur_rb_cg(A, B[:, c], _grid(op), eta=0.5e-12)
        full = P.pcg(A, B[:, c], eta=0.5e-12, pc="ic0_rb", grid=_grid(op))
        assert cond.converged and full.converged
        cond_its.append(cond.iters)
        full_its.append(full.iters)
    # the columns advance together: the GPU count is the slowest column's
    assert abs(iters - max(cond_its)) <= 1, (iters, cond_its)
    assert abs(iters - max(full_its)) <= 2, (iters, full_its)


def test_ic0_fewer_iterations_than_jacobi(lib):
    b = _b()
    op = fv3d(16, 1.0, 3)
    B = _dev(gaussian_C(op.n, 1, 4))
    dop = b.device_op(op)
    _, it_ic0, rel0, _ = b.inner_solve(dop, B, inner_pc=b.PC_IC0)
    _, it_jac, rel1, _ = b.inner_solve(dop, B, inner_pc=b.PC_JACOBI)
    assert rel0 <= 1e-12 and rel1 <= 1e-12
    assert it_ic0 < 0.7 * it_jac, (it_ic0, it_jac)


def test_ic0_zero_rhs_and_errors(lib):
    b = _b()
    op = fv3d(6, 1.0, 3)
    dop = b.device_op(op)
    B = np.zeros((op.n, 2))
    B[:, 1] = gaussian_C(op.n, 1, 2)[:, 0]
    X, iters, rel, st = b.inner_solve(dop, _dev(B), inner_pc=b.PC_IC0)
    assert st == b.OK
    Xh = X.cpu().numpy()
    assert np.all(Xh[:, 0] == 0.0)
    A = op.to_scipy()
    assert np.linalg.norm(A @ Xh[:, 1] - B[:, 1]) <= 1e-12 * np.linalg.norm(B[:, 1])
    # too few iterations: reported, not raised
    X, iters, rel, st = b.inner_solve(b.device_op(fv3d(12, 1.0, 3)), _dev(gaussian_C(1728, 1, 9)),
                                      raise_on_error=False, inner_pc=b.PC_IC0, inner_max_iter=5)
    assert st == b.E_INNER and rel > 1e-12 and iters == 5
    # a CSR operator has no grid to colour
    lop = laplace2d(9)
    with pytest.raises(b.LyapError) as e:
        b.inner_solve(b.device_op(lop, as_csr=True), _dev(gaussian_C(lop.n, 1, 1)), inner_pc=b.PC_IC0)
    assert e.value.status == b.E_UNSUPPORTED


@pytest.mark.parametrize("N,s", [(10, 1), (12, 2)])
def test_ek_with_ic0_parity(lib, N, s):
    """Extended Krylov with IC(0) inner solves against the oracle's EK with
    exact (LU) solves: same m, residual histories, Z Z^T."""
    b = _b()
    op = fv3d(N, 1.0, 3)
    A = op.to_scipy()
    C = gaussian_C(op.n, s, 3)
    sol = b.lyap_solve(b.device_op(op), _dev(C), method=b.METHOD_EXT, tol=1e-8, check_every=1,
                       inner_pc=b.PC_IC0, inner_tol=1e-12)
    ref = E.lyap_ext(A, C, tol=1e-8)
    assert sol.status == b.OK and sol.m == ref.m
    for g, r in zip(sol.hist_res, ref.hist):
        assert abs(g - r["res"]) <= 1e-5 * r["res"] + 1e-13
    Z = sol.Z.cpu().numpy()
    assert K.factor_error(Z, ref.Z) <= 1e-7
    assert K.lowrank_vs_dense_error(Z, D.lyap_eig(A.toarray(), C)) <= 1e-7
    assert K.explicit_residual(A, Z, C) / sol.beta ** 2 <= 1.2e-8


@pytest.mark.parametrize("pc", ["ic0", "jacobi"])
def test_inner_cg_full_launch_shape(lib, pc):
    """Inner CG at 81^3 = 531441 rows (at least 2^19: the launch shape of the
    n = 1e6 runs, two 1024-thread workgroups per CU for Jacobi) against the
    oracle's PCG on the same operator and right-hand side."""
    b = _b()
    op = fv3d(81, 1.0, 3)
    A = op.to_scipy()
    B = gaussian_C(op.n, 1, 5)
    print(f"pc {pc} n={op.n}", flush=True)
    X, iters, rel, st = b.inner_solve(b.device_op(op), _dev(B), inner_pc=b.PC_IC0 if pc == "ic0" else b.PC_JACOBI,
                                      inner_tol=1e-12, inner_max_iter=20000)
    assert st == b.OK and rel <= 1e-12
    if pc == "ic0":
        ref = P.schur_rb_cg(A, B[:, 0], _grid(op), eta=0.5e-12, max_iter=20000)
    else:
        ref = P.pcg(A, B[:, 0], eta=0.5e-12, pc="jacobi", max_iter=20000)
    assert ref.converged
    Xh = X.cpu().numpy()[:, 0]
    assert np.linalg.norm(Xh - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    assert abs(iters - ref.iters) <= 3, (iters, ref.iters)
