"""The allocation-free apply of the learned preconditioner
(lyap_pcnet_apply_noalloc): the same result as lyap_pcnet_apply, call after
call, with every intermediate buffer taken from the library's static
per-device workspace, and a clear error past its size limit."""
import numpy as np
import pytest

from workloads import fv3d, laplace2d
from oracle import cnn as N

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _b():
    from paper_1602_05033_amd import binding
    return binding


def _case(op, C, seed):
    b = _b()
    W = b.pcnet_init(C, 100 + seed, 0.3)
    r = torch.from_numpy(np.random.default_rng(seed).standard_normal(op.n)).cuda()
    dop = b.device_op(op)
    ref = b.pcnet_apply(dop, C, W, r)
    z = torch.full_like(r, float("nan"))
    b.pcnet_apply_noalloc(dop, C, W, r, z)
    torch.cuda.synchronize()
    return W, r.cpu().numpy(), ref.cpu().numpy(), z.cpu().numpy()


def _oracle_ok(op, C, W, r, z):
    nz = op.nz if op.kind == "stencil7" else 1
    A = op.to_scipy()
    g = N.grid_of(A, op.nx, op.ny, nz)
    ref = N.apply(N.PcNet.from_flat(np.asarray(W, dtype=np.float64), C), g, r)
    corr = ref - g.dinv * r
    return np.linalg.norm(z - ref) <= 2e-6 * np.linalg.norm(corr) + 1e-14 * np.linalg.norm(ref)


def test_noalloc_matches_apply_two_calls(lib):
    # first call: a 7-point operator on 40 x 36 x 32 cells (vector path, nx % 4 == 0)
    big = fv3d(40, 1.0, 3, Ny=36, Nz=32)
    W, r, ref, z = _case(big, 4, 1)
    assert np.array_equal(z, ref)
    assert _oracle_ok(big, 4, W, r, z)
    # second call, smaller and on the scalar path (nx % 4 != 0): the workspace
    # still holds the first call's data
    small = fv3d(9, 1.0, 5, Ny=7, Nz=6)
    W, r, ref, z = _case(small, 2, 2)
    assert np.array_equal(z, ref)
    assert _oracle_ok(small, 2, W, r, z)
    # a 5-point operator (no coefficient copies)
    lap = laplace2d(24, shift=1.0)
    W, r, ref, z = _case(lap, 8, 3)
    assert np.array_equal(z, ref)


def test_noalloc_largest_input(lib):
    # n = 64^3 = 262144 with C = 4 is the documented limit; it fits
    op = fv3d(64, 1.0, 7)
    W, r, ref, z = _case(op, 4, 4)
    assert np.array_equal(z, ref)


def test_noalloc_rejects_too_large(lib):
    b = _b()
    op = fv3d(80, 1.0, 3, Ny=80, Nz=48)  # n = 307200: over the 32 MiB workspace at C = 4
    dop = b.device_op(op)
    W = b.pcnet_init(4, 1, 0.1)
    r = torch.ones(op.n, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(r)
    with pytest.raises(b.LyapError) as ei:
        b.pcnet_apply_noalloc(dop, 4, W, r, z)
    assert ei.value.status == b.E_ARG
    assert "workspace" in str(ei.value)
    assert float(z.abs().max()) == 0.0  # nothing written
    # the entry point still works after the rejection
    small = fv3d(8, 1.0, 3)
    W, r, ref, z2 = _case(small, 4, 6)
    assert np.array_equal(z2, ref)
