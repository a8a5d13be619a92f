"""Pins of the learned-preconditioner oracle: the convolution against a brute
force, the transposed convolution as its adjoint, symmetry and definiteness
of M, zero weights = Jacobi, gradients against central finite differences,
the Adam update in closed form, FCG with the Jacobi preconditioner = PCG, and
training that lowers the FCG iteration count.  CPU."""
import numpy as np
import pytest

from workloads import fv3d, gaussian_C
from oracle import cnn as N
from oracle import pcg as P


def _brute_conv(x, W):
    Ci, nz, ny, nx = x.shape
    out = np.zeros((W.shape[0], nz, ny, nx))
    for o in range(W.shape[0]):
        for z in range(nz):
            for y in range(ny):
                for xx in range(nx):
                    acc = 0.0
                    for t, (dz, dy, dx) in enumerate(N.OFFSETS):
                        zz, yy, x2 = z + dz, y + dy, xx + dx
                        if 0 <= zz < nz and 0 <= yy < ny and 0 <= x2 < nx:
                            acc += W[o, :, t] @ x[:, zz, yy, x2]
                    out[o, z, y, xx] = acc
    return out


def test_conv_brute_force_and_adjoint():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4, 3, 5))
    W = rng.standard_normal((3, 2, 27))
    assert np.allclose(N.conv(x, W), _brute_conv(x, W), atol=1e-12)
    y = rng.standard_normal((3, 4, 3, 5))
    assert abs(np.sum(N.conv(x, W) * y) - np.sum(x * N.convT(y, W))) <= 1e-10 * np.abs(np.sum(x * N.convT(y, W)))
    # weight gradient = d/dW <y, conv(x, W)>
    dW = N.conv_wgrad(x, y)
    E = np.zeros_like(W)
    E[1, 0, 13] = 1.0
    assert abs(dW[1, 0, 13] - np.sum(y * N.conv(x, E))) <= 1e-12


@pytest.fixture(scope="module")
def small():
    op = fv3d(6, 1.0, 3)
    A = op.to_scipy()
    g = N.grid_of(A, op.nx, op.ny, op.nz)
    return op, A, g


def test_M_spd_and_jacobi_limit(small):
    op, A, g = small
    net = N.init_net(3, 1, scale=0.3)
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal(op.n), rng.standard_normal(op.n)
    Ma, Mb = N.apply(net, g, a), N.apply(net, g, b)
    assert abs(a @ Mb - b @ Ma) <= 1e-12 * abs(a @ Mb)
    assert a @ Ma > 0 and b @ Mb > 0
    zero = N.PcNet(3, np.zeros((3, 2, 27)), np.zeros((3, 3, 27)))
    assert np.allclose(N.apply(zero, g, a), g.dinv * a, rtol=0, atol=0)


def test_gradient_central_differences(small):
    op, A, g = small
    net = N.init_net(2, 4, scale=0.2)
    rng = np.random.default_rng(5)
    e = rng.standard_normal(op.n)
    r = -(A @ e)                      # (-A) e = r
    L, dW1, dW2 = N.loss_and_grad(net, g, A, r, e)
    grad = np.concatenate([dW1.ravel(), dW2.ravel()])
    v0 = net.flat()
    h = 1e-6
    for idx in list(range(0, 108, 13)) + list(range(108, 216, 17)):
        vp, vm = v0.copy(), v0.copy()
        vp[idx] += h
        vm[idx] -= h
        Lp = N.loss_and_grad(N.PcNet.from_flat(vp, 2), g, A, r, e)[0]
        Lm = N.loss_and_grad(N.PcNet.from_flat(vm, 2), g, A, r, e)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(grad[idx])) + 1e-8, (idx, fd, grad[idx])


def test_adam_closed_form():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 0.0])
    opt = N.Adam(lr=0.1)
    opt.step([p], [g])
    # first step: m_hat = g, v_hat = g^2 -> p -= lr * g / (|g| + eps)
    assert np.allclose(p, [1.0 - 0.1 * 0.5 / (0.5 + 1e-8), -2.0 + 0.1 * 4.0 / (4.0 + 1e-8), 3.0])


def test_fcg_with_jacobi_is_pcg():
    op = fv3d(7, 1.0, 3)
    A = op.to_scipy()
    b = gaussian_C(op.n, 1, 3)[:, 0]
    dinv = 1.0 / (-A.diagonal())
    x, it, rel = N.fcg(A, b, lambda r: r * dinv, eta=1e-12)
    ref = P.pcg(A, b, eta=1e-12, pc="jacobi", restarts=0)
    assert rel <= 1e-12 and abs(it - ref.iters) <= 1


def test_training_lowers_iterations():
    op = fv3d(12, 1.0, 3)
    A = op.to_scipy()
    g = N.grid_of(A, op.nx, op.ny, op.nz)
    b = gaussian_C(op.n, 1, 3)[:, 0]
    pairs, _, it_j = N.harvest_pairs(A, b, every=4, keep=16)
    net = N.init_net(4, 7)
    losses = N.train(net, g, A, pairs, steps=120, lr=2e-3)
    assert np.mean(losses[-16:]) < np.mean(losses[:16])
    b2 = gaussian_C(op.n, 1, 11)[:, 0]          # a different right-hand side
    _, it_l, rel = N.fcg(A, b2, lambda r: N.apply(net, g, r), eta=1e-12)
    _, it_0, _ = N.fcg(A, b2, lambda r: r * g.dinv, eta=1e-12)
    assert rel <= 1e-12 and it_l < it_0


def test_splitmix64_reference_vector():
    """The generator's published test vector (seed 1234567)."""
    assert list(N.splitmix64(1234567, 5)) == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                              4593380528125082431, 16408922859458223821]


# ------------------------------------------------------------------ on the black Schur complement
@pytest.fixture(scope="module")
def condensed():
    op = fv3d(7, 1.0, 3, Ny=6, Nz=5)           # odd nx: padding slots in the compact grid
    A = op.to_scipy()
    sysm = P.rb_system(A, (op.nx, op.ny, op.nz))
    return op, A, sysm, N.condensed_grid(sysm), N.condensed_operator(sysm)


def test_condensed_grid_layout(condensed):
    op, A, sysm, g, Ap = condensed
    nz, ny, hxp = g.shape
    assert (nz, ny) == (op.nz, op.ny) and hxp % 4 == 0 and hxp >= (op.nx + 1) // 2
    # every black cell (i, j, l) sits at compact column i // 2 of its line
    idx = np.arange(op.n)[sysm.blk]
    i, j, l = idx % op.nx, (idx // op.nx) % op.ny, idx // (op.nx * op.ny)
    assert np.array_equal(sysm.slot, (j + op.ny * l) * hxp + i // 2)
    assert len(set(sysm.slot.tolist())) == sysm.slot.shape[0]
    rng = np.random.default_rng(1)
    v = rng.standard_normal(sysm.slot.shape[0])
    assert np.array_equal(sysm.extract(sysm.embed(v)), v)
    pad = np.ones(int(np.prod(g.shape)), bool)
    pad[sysm.slot] = False
    assert pad.any() and np.all(g.dinv[pad] == 0.0) and np.all(g.s.reshape(-1)[pad] == 0.0)
    assert np.allclose(g.dinv[sysm.slot], 1.0 / sysm.Sigma.diagonal(), rtol=1e-15)
    # -Ap is Sigma on the slots, zero at the padding
    assert abs(Ap[np.ix_(sysm.slot, sysm.slot)] + sysm.Sigma).max() == 0.0
    assert Ap[pad].nnz == 0


def test_condensed_M_spd_and_ic0_limit(condensed):
    op, A, sysm, g, Ap = condensed
    nb = sysm.slot.shape[0]
    net = N.init_net(2, 3, scale=0.3)
    M = np.column_stack([N.condensed_precond(net, sysm, g)(e) for e in np.eye(nb)])
    assert np.allclose(M, M.T, rtol=0, atol=1e-13 * np.abs(M).max())
    assert np.linalg.eigvalsh(M).min() > 0.0
    zero = N.PcNet(2, np.zeros((2, 2, 27)), np.zeros((2, 2, 27)))
    b = gaussian_C(op.n, 1, 5)[:, 0]
    grid = (op.nx, op.ny, op.nz)
    ic0 = P.schur_rb_cg(A, b, grid, eta=1e-12, system=sysm)
    fz = P.schur_rb_cg(A, b, grid, eta=1e-12, system=sysm, precond=N.condensed_precond(zero, sysm, g))
    # zero weights: diag(Sigma)^{-1}, and FCG with a fixed SPD preconditioner is PCG
    assert fz.iters == ic0.iters and np.linalg.norm(fz.x - ic0.x) <= 1e-10 * np.linalg.norm(ic0.x)


def test_condensed_gradient_central_differences(condensed):
    op, A, sysm, g, Ap = condensed
    net = N.init_net(2, 8, scale=0.2)
    rng = np.random.default_rng(6)
    e = sysm.embed(rng.standard_normal(sysm.slot.shape[0]))
    r = -(Ap @ e)                              # Sigma e = r on the slots
    L, dW1, dW2 = N.loss_and_grad(net, g, Ap, r, e)
    grad = np.concatenate([dW1.ravel(), dW2.ravel()])
    v0 = net.flat()
    h = 1e-6
    for idx in list(range(0, 108, 11)) + list(range(108, 216, 19)):
        vp, vm = v0.copy(), v0.copy()
        vp[idx] += h
        vm[idx] -= h
        Lp = N.loss_and_grad(N.PcNet.from_flat(vp, 2), g, Ap, r, e)[0]
        Lm = N.loss_and_grad(N.PcNet.from_flat(vm, 2), g, Ap, r, e)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(grad[idx])) + 1e-8, (idx, fd, grad[idx])


def test_condensed_training_beats_ic0():
    """Harvest from the condensed IC(0) CG, train, and the learned correction
    needs fewer iterations than IC(0) itself on another right-hand side."""
    op = fv3d(16, 1.0, 3)
    A = op.to_scipy()
    grid = (op.nx, op.ny, op.nz)
    sysm = P.rb_system(A, grid)
    g, Ap = N.condensed_grid(sysm), N.condensed_operator(sysm)
    pairs, it_h = N.harvest_condensed(sysm, gaussian_C(op.n, 1, 3)[:, 0], every=4, keep=16)
    pairs = [p for p in pairs if np.linalg.norm(p[1]) > 0]
    net = N.init_net(2, 0x5eed)
    N.train(net, g, Ap, pairs, steps=200, lr=2e-3)
    b2 = gaussian_C(op.n, 1, 11)[:, 0]
    ic0 = P.schur_rb_cg(A, b2, grid, eta=1e-12, system=sysm)
    lrn = P.schur_rb_cg(A, b2, grid, eta=1e-12, system=sysm, precond=N.condensed_precond(net, sysm, g))
    assert lrn.converged and lrn.relres_true <= 1e-12
    assert lrn.iters < 0.8 * ic0.iters, (lrn.iters, ic0.iters)
