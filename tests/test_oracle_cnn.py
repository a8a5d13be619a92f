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
