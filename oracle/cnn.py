"""Learned preconditioner for the inner solves of the extended Krylov method:
a small linear 3-D convolutional network K that forms a symmetric positive
definite correction of the Jacobi preconditioner, its training on error /
residual pairs harvested from the run's own solves, and flexible CG driven by
it.

Oracle -- test infrastructure only.  Plain float64 NumPy.  Not from the paper
(which solves exactly).

Preconditioner (grid nx x ny x nz, lexicographic x fastest, zero padding):
  D^{-1} = diag(-A)^{-1},  s = sqrt(D^{-1}),  f = log(-diag A) - mean(log(-diag A))
  K(u)   = conv2(conv1([u, f u]))          2 -> C -> C channels, 3x3x3, no bias
  M r    = D^{-1} r + s * K^T(K(s * r))
K^T is the adjoint of K (transposed convolutions, then [v0 + f v1]); hence M is
symmetric positive definite for any weights, so CG/FCG stay well posed and the
zero weights give plain Jacobi.  conv(x, W)[o, p] = sum_i sum_t W[o, i, t]
x[i, p + t] over the 27 offsets t in {-1,0,1}^3; convT(y, W)[i, q] = sum_o sum_t
W[o, i, t] y[o, q - t].

Training on pairs (r, e) with (-A) e = r (e = x* - x_i of a harvested CG
iterate): energy-norm loss  L = (M r - e)^T (-A) (M r - e) / e^T (-A) e, Adam.

Flexible CG (FCG(1)): q = (-A) p; alpha = p.r / p.q; x += alpha p;
r -= alpha q; z = M(r); beta = -(z.q) / (p.q); p = z + beta p.

The same network also corrects the red-black IC(0) preconditioner: the
inner solve is then run on the black Schur complement Sigma (oracle.pcg), and
M = diag(Sigma)^{-1} + s K^T K s acts on the compact array of the black cells
(``condensed_grid``: nz x ny x hxp, compact column i // 2 of each grid line,
padding slots held at zero), so that zero weights give IC(0) itself; pairs
are harvested from the condensed IC(0) CG (``harvest_condensed``) and the
loss uses Sigma in place of -A.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np
import scipy.sparse as sp

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shift(x: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """y[p] = x[p + t] with zero padding; x has shape (..., nz, ny, nx)."""
    y = np.zeros_like(x)
    nz, ny, nx = x.shape[-3:]
    zs = slice(max(0, -dz), nz - max(0, dz))
    zd = slice(max(0, dz), nz - max(0, -dz))
    ys = slice(max(0, -dy), ny - max(0, dy))
    yd = slice(max(0, dy), ny - max(0, -dy))
    xs = slice(max(0, -dx), nx - max(0, dx))
    xd = slice(max(0, dx), nx - max(0, -dx))
    y[..., zs, ys, xs] = x[..., zd, yd, xd]
    return y


def conv(x: np.ndarray, W: np.ndarray) -> np.ndarray:
    """x (Ci, nz, ny, nx), W (Co, Ci, 27) -> (Co, nz, ny, nx)."""
    out = np.zeros((W.shape[0],) + x.shape[1:])
    for t, (dz, dy, dx) in enumerate(OFFSETS):
        out += np.einsum("oi,izyx->ozyx", W[:, :, t], shift(x, dz, dy, dx))
    return out


def convT(y: np.ndarray, W: np.ndarray) -> np.ndarray:
    """The adjoint of conv: y (Co, ...) -> (Ci, ...)."""
    out = np.zeros((W.shape[1],) + y.shape[1:])
    for t, (dz, dy, dx) in enumerate(OFFSETS):
        out += np.einsum("oi,ozyx->izyx", W[:, :, t], shift(y, -dz, -dy, -dx))
    return out


def conv_wgrad(x: np.ndarray, g: np.ndarray) -> np.ndarray:
    """d/dW of <g, conv(x, W)>: dW[o, i, t] = sum_p g[o, p] x[i, p + t]."""
    dW = np.zeros((g.shape[0], x.shape[0], 27))
    for t, (dz, dy, dx) in enumerate(OFFSETS):
        dW[:, :, t] = np.einsum("ozyx,izyx->oi", g, shift(x, dz, dy, dx))
    return dW


@dataclass
class PcNet:
    C: int
    W1: np.ndarray   # (C, 2, 27)
    W2: np.ndarray   # (C, C, 27)

    def flat(self) -> np.ndarray:
        return np.concatenate([self.W1.ravel(), self.W2.ravel()])

    @staticmethod
    def from_flat(v: np.ndarray, C: int) -> "PcNet":
        k1 = C * 2 * 27
        return PcNet(C, np.array(v[:k1], dtype=np.float64).reshape(C, 2, 27),
                     np.array(v[k1:k1 + C * C * 27], dtype=np.float64).reshape(C, C, 27))


def param_count(C: int) -> int:
    return C * 2 * 27 + C * C * 27


def splitmix64(seed: int, count: int) -> np.ndarray:
    """SplitMix64 (Steele, Lea and Flood, 2014): state += 0x9E3779B97F4A7C15;
    z = state; z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9; z = (z ^ (z >> 27)) *
    0x94D049BB133111EB; out = z ^ (z >> 31), all mod 2^64."""
    M = (1 << 64) - 1
    state = seed & M
    out = np.empty(count, dtype=np.uint64)
    for i in range(count):
        state = (state + 0x9E3779B97F4A7C15) & M
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        out[i] = z ^ (z >> 31)
    return out


def init_net(C: int, seed: int, scale: float = 0.05) -> PcNet:
    """Weights uniform in [-scale, scale): u = (top 53 bits of SplitMix64) / 2^53,
    w = scale (2u - 1), W1 then W2 in row-major order (the same generator is
    implemented on the device side)."""
    raw = splitmix64(seed, param_count(C))
    u = (raw >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    return PcNet.from_flat(scale * (2.0 * u - 1.0), C)


@dataclass
class Grid:
    shape: tuple          # (nz, ny, nx)
    dinv: np.ndarray      # (n,)
    s: np.ndarray         # (nz, ny, nx)
    f: np.ndarray         # (nz, ny, nx)


def grid_of(A, nx: int, ny: int, nz: int) -> Grid:
    d = -np.asarray(sp.csr_matrix(A).diagonal())
    ld = np.log(d)
    shape = (nz, ny, nx)
    return Grid(shape, 1.0 / d, np.sqrt(1.0 / d).reshape(shape), (ld - ld.mean()).reshape(shape))


def K_apply(net: PcNet, g: Grid, u: np.ndarray):
    x0 = np.stack([u, g.f * u])
    a1 = conv(x0, net.W1)
    return conv(a1, net.W2), x0, a1


def KT_apply(net: PcNet, g: Grid, k: np.ndarray) -> np.ndarray:
    d = convT(convT(k, net.W2), net.W1)
    return d[0] + g.f * d[1]


def apply(net: PcNet, g: Grid, r: np.ndarray) -> np.ndarray:
    """z = M r."""
    u = g.s * r.reshape(g.shape)
    k, _, _ = K_apply(net, g, u)
    return g.dinv * r + (g.s * KT_apply(net, g, k)).reshape(-1)


def loss_and_grad(net: PcNet, g: Grid, A, r: np.ndarray, e: np.ndarray):
    """Energy-norm loss and (dW1, dW2).  With w = K^T K u:
    dL = gw . (dK^T K u + K^T dK u) = (K gw) . (dK u) + (K u) . (dK gw),
    gw = s * dL/dz, dL/dz = 2 (-A)(z - e) / e^T (-A) e."""
    Ap = -sp.csr_matrix(A)
    u = g.s * r.reshape(g.shape)
    k, x0, a1 = K_apply(net, g, u)
    z = g.dinv * r + (g.s * KT_apply(net, g, k)).reshape(-1)
    d = z - e
    Ad = Ap @ d
    eAe = float(e @ (Ap @ e))
    L = float(d @ Ad) / eAe
    gz = 2.0 * Ad / eAe
    gw = g.s * gz.reshape(g.shape)
    kg, x0g, a1g = K_apply(net, g, gw)
    # dK u = W2 (dW1 x0) + dW2 a1: back-propagate each output gradient
    dW2 = conv_wgrad(a1, kg) + conv_wgrad(a1g, k)
    dW1 = conv_wgrad(x0, convT(kg, net.W2)) + conv_wgrad(x0g, convT(k, net.W2))
    return L, dW1, dW2


@dataclass
class Adam:
    lr: float = 2e-3
    b1: float = 0.9
    b2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: list = field(default_factory=list)
    v: list = field(default_factory=list)

    def step(self, params: List[np.ndarray], grads: List[np.ndarray]):
        """In place: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
        p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""
        if not self.m:
            self.m = [np.zeros_like(p) for p in params]
            self.v = [np.zeros_like(p) for p in params]
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, gr, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * gr
            v *= self.b2
            v += (1.0 - self.b2) * gr * gr
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


def harvest_pairs(A, b: np.ndarray, every: int = 32, keep: int = 16, eta: float = 1e-12):
    """Jacobi-PCG on (-A) x = -b; snapshots (r_i, x_i) every `every`
    iterations, then e_i = x* - x_i with the converged x*."""
    Ap = -sp.csr_matrix(A)
    dinv = 1.0 / Ap.diagonal()
    x = np.zeros_like(b)
    r = -b.copy()
    z = r * dinv
    p = z.copy()
    rho = float(r @ z)
    snaps = []
    bn = float(np.linalg.norm(b))
    it = 0
    while float(np.linalg.norm(r)) > eta * bn and it < 100000:
        if it % every == 0 and len(snaps) < keep:
            snaps.append((r.copy(), x.copy()))
        q = Ap @ p
        alpha = rho / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = r * dinv
        rn = float(r @ z)
        p = z + (rn / rho) * p
        rho = rn
        it += 1
    return [(ri, x - xi) for ri, xi in snaps], x, it


def train(net: PcNet, g: Grid, A, pairs, steps: int, lr: float = 2e-3):
    """Adam over the pairs in order (pair (t mod P) at step t); returns the losses."""
    opt = Adam(lr=lr)
    losses = []
    for t in range(steps):
        r, e = pairs[t % len(pairs)]
        L, dW1, dW2 = loss_and_grad(net, g, A, r, e)
        opt.step([net.W1, net.W2], [dW1, dW2])
        losses.append(L)
    return losses


def fcg(A, b: np.ndarray, precond, eta: float = 1e-12, max_iter: int = 10000):
    """Flexible CG on (-A) x = -b; returns (x, iterations, true relative residual)."""
    Ap = -sp.csr_matrix(A)
    x = np.zeros_like(b)
    r = -b.copy()
    bn = float(np.linalg.norm(b))
    z = precond(r)
    p = z.copy()
    it = 0
    while it < max_iter and float(np.linalg.norm(r)) > eta * bn:
        q = Ap @ p
        pq = float(p @ q)
        alpha = float(p @ r) / pq
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        z = precond(r)
        beta = -float(z @ q) / pq
        p = z + beta * p
    return x, it, float(np.linalg.norm(b - A @ x)) / bn


# ------------------------------------------------------------ on the Schur complement
def condensed_grid(sysm) -> Grid:
    """The network's grid for the black Schur complement of a red-black split
    (``oracle.pcg.rb_system``): the compact array of the black cells, with
    D = diag(Sigma) at the cells and dinv = s = f = 0 at the padding slots."""
    nsl = int(np.prod(sysm.shape))
    dinv = np.zeros(nsl)
    dinv[sysm.slot] = 1.0 / sysm.S
    f = np.zeros(nsl)
    ld = np.log(sysm.S)
    f[sysm.slot] = ld - ld.mean()
    return Grid(sysm.shape, dinv, np.sqrt(dinv).reshape(sysm.shape), f.reshape(sysm.shape))


def condensed_operator(sysm):
    """-Sigma on the compact slots (zero rows and columns at the padding), the
    "A" that ``loss_and_grad`` takes for the condensed system."""
    nsl = int(np.prod(sysm.shape))
    nb = sysm.slot.shape[0]
    P = sp.csr_matrix((np.ones(nb), (sysm.slot, np.arange(nb))), shape=(nsl, nb))
    return (-(P @ sysm.Sigma @ P.T)).tocsr()


def condensed_precond(net: PcNet, sysm, g: Grid):
    """z = M r for a black-cell residual r."""
    return lambda rb: sysm.extract(apply(net, g, sysm.embed(rb)))


def harvest_condensed(sysm, b: np.ndarray, every: int, keep: int, eta: float = 1e-12):
    """Pairs (r_i, e_i) in compact-slot layout from the condensed IC(0) CG of
    A x = b: CG on Sigma x_b = rhs~ (rhs~ = the condensed -b) preconditioned by
    diag(Sigma), snapshots every `every` iterations (``harvest_pairs`` on
    -Sigma)."""
    rt = sysm.condense(-b)
    pairs, xb, it = harvest_pairs(-sysm.Sigma, -rt, every=every, keep=keep, eta=eta)
    return [(sysm.embed(r), sysm.embed(e)) for r, e in pairs], it

