"""Problem generators: symmetric negative definite sparse operators and seeded
right-hand sides.

Grid ordering is lexicographic with x fastest: cell (i, j, l) has row index
``i + Nx*(j + Ny*l)``.

Operators
---------
``stencil5``  constant-coefficient 5-point operator on an N x N interior grid:
              ``A[r,r] = cc``, ``A[r,nbr] = co`` for the four grid neighbours.
              ``laplace2d`` gives A = -(1/h^2)(I (x) T + T (x) I) - shift*I with
              T = tridiag(-1, 2, -1), h = 1/(N+1), zero Dirichlet boundary.
``csr``       a general sparse matrix given by its CSR arrays (``fe_p1_2d``).
``stencil7``  variable-coefficient 7-point operator on Nx x Ny x Nz cells
              (Nz = 1 for 2D), given by per-cell arrays ``diag`` (the diagonal),
              ``tx``, ``ty``, ``tz`` (the coupling to the +x, +y, +z neighbour;
              zero on the last cell of a line).  Symmetric by construction.

Every operator can also be emitted as CSR (int64 row pointers, int32 column
indices sorted within a row, float64 values).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Operator:
    kind: str                      # "stencil5" | "stencil7"
    n: int
    nx: int
    ny: int
    nz: int = 1
    h: float = 1.0
    cc: float = 0.0                # stencil5 centre coefficient
    co: float = 0.0                # stencil5 neighbour coefficient
    diag: Optional[np.ndarray] = None
    tx: Optional[np.ndarray] = None
    ty: Optional[np.ndarray] = None
    tz: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)
    csr: Optional[tuple] = None    # kind "csr": (rowptr, col, val)

    # ------------------------------------------------------------------ CSR
    def to_csr(self):
        """Return (rowptr int64[n+1], col int32[nnz], val float64[nnz])."""
        if self.kind == "csr":
            return self.csr
        if self.kind == "stencil5":
            N = self.nx
            n = self.n
            idx = np.arange(n, dtype=np.int64)
            i = idx % N
            j = idx // N
            cols = []
            vals = []
            masks = []
            # order: -y, -x, centre, +x, +y  (ascending column index)
            for (di, dj, v) in ((0, -1, self.co), (-1, 0, self.co), (0, 0, self.cc),
                                (1, 0, self.co), (0, 1, self.co)):
                ok = (i + di >= 0) & (i + di < N) & (j + dj >= 0) & (j + dj < N)
                cols.append(idx + di + dj * N)
                vals.append(np.full(n, v))
                masks.append(ok)
            return _pack_csr(n, cols, vals, masks)
        if self.kind == "stencil7":
            nx, ny, nz = self.nx, self.ny, self.nz
            n = self.n
            idx = np.arange(n, dtype=np.int64)
            i = idx % nx
            j = (idx // nx) % ny
            l = idx // (nx * ny)
            sxy = nx * ny
            zero = np.zeros(n)
            tzm = np.concatenate([zero[:sxy], self.tz[:-sxy]]) if nz > 1 else zero
            tym = np.concatenate([zero[:nx], self.ty[:-nx]]) if ny > 1 else zero
            txm = np.concatenate([zero[:1], self.tx[:-1]])
            entries = [
                (-sxy, tzm, l > 0),
                (-nx, tym, j > 0),
                (-1, txm, i > 0),
                (0, self.diag, np.ones(n, bool)),
                (1, self.tx, i < nx - 1),
                (nx, self.ty, j < ny - 1),
                (sxy, self.tz, l < nz - 1),
            ]
            cols = [idx + off for off, _, _ in entries]
            vals = [np.asarray(v, dtype=np.float64) for _, v, _ in entries]
            masks = [m for _, _, m in entries]
            return _pack_csr(n, cols, vals, masks)
        raise ValueError(self.kind)

    def to_scipy(self):
        import scipy.sparse as sp
        rp, ci, va = self.to_csr()
        return sp.csr_matrix((va, ci.astype(np.int64), rp), shape=(self.n, self.n))


def _pack_csr(n, cols, vals, masks):
    M = np.stack(masks, axis=1)                  # n x K
    C = np.stack(cols, axis=1)
    V = np.stack(vals, axis=1)
    counts = M.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = C[M].astype(np.int32)                  # row-major traversal keeps order
    val = V[M].astype(np.float64)
    return rowptr, col, val


# ---------------------------------------------------------------- operators
def laplace2d(N: int, shift: float = 0.0) -> Operator:
    """A = -(1/h^2)(I (x) T + T (x) I) - shift*I on an N x N interior grid,
    h = 1/(N+1), zero Dirichlet boundary (the 5-point finite-difference
    Laplacian, negated so that A is symmetric negative definite)."""
    h = 1.0 / (N + 1)
    inv = 1.0 / (h * h)
    return Operator(kind="stencil5", n=N * N, nx=N, ny=N, nz=1, h=h,
                    cc=-4.0 * inv - shift, co=inv,
                    meta={"name": "laplace2d", "N": N, "shift": shift})


def _harm(a, b):
    return 2.0 * a * b / (a + b)


def fv3d(N: int, sigma: float, seed_k: int, Ny: Optional[int] = None,
         Nz: Optional[int] = None) -> Operator:
    """A = -div(k grad u), cell-centred finite volumes on the unit cube split
    into N x Ny x Nz cells of size h = 1/N, zero Dirichlet boundary.

    k is lognormal per cell: k = exp(sigma * xi), xi ~ N(0,1) drawn from
    ``numpy.random.default_rng([seed_k])`` in cell order.  An interior face
    between cells a and b has transmissibility 2 k_a k_b / (k_a + k_b) / h^2
    (harmonic mean); a boundary face of cell c has 2 k_c / h^2 (the boundary
    value sits half a cell away).  A[r,r] = -(sum of r's six face values),
    A[r, nbr] = +face value.
    """
    Ny = N if Ny is None else Ny
    Nz = N if Nz is None else Nz
    nx, ny, nz = N, Ny, Nz
    n = nx * ny * nz
    h = 1.0 / N
    inv = 1.0 / (h * h)
    xi = np.random.default_rng([seed_k]).standard_normal(n)
    k = np.exp(sigma * xi).reshape(nz, ny, nx)
    tx = np.zeros((nz, ny, nx))
    ty = np.zeros((nz, ny, nx))
    tz = np.zeros((nz, ny, nx))
    tx[:, :, :-1] = _harm(k[:, :, :-1], k[:, :, 1:]) * inv
    ty[:, :-1, :] = _harm(k[:, :-1, :], k[:, 1:, :]) * inv
    tz[:-1, :, :] = _harm(k[:-1, :, :], k[1:, :, :]) * inv
    s = np.zeros((nz, ny, nx))
    s += tx
    s[:, :, 1:] += tx[:, :, :-1]
    s += ty
    s[:, 1:, :] += ty[:, :-1, :]
    s += tz
    s[1:, :, :] += tz[:-1, :, :]
    # boundary faces
    bnd = 2.0 * k * inv
    s[:, :, 0] += bnd[:, :, 0]
    s[:, :, -1] += bnd[:, :, -1]
    s[:, 0, :] += bnd[:, 0, :]
    s[:, -1, :] += bnd[:, -1, :]
    if nz > 1:
        s[0, :, :] += bnd[0, :, :]
        s[-1, :, :] += bnd[-1, :, :]
    return Operator(kind="stencil7", n=n, nx=nx, ny=ny, nz=nz, h=h,
                    diag=(-s).ravel(), tx=tx.ravel(), ty=ty.ravel(), tz=tz.ravel(),
                    meta={"name": "fv3d", "N": N, "sigma": sigma, "seed_k": seed_k,
                          "k": k.ravel()})


def fd2d_variable(N: int, ax, ay, name: str = "fd2d") -> Operator:
    """Centred, conservative finite differences for (a_x u_x)_x + (a_y u_y)_y on
    the unit square, N x N interior points, h = 1/(N+1), zero Dirichlet
    boundary; a_x and a_y are evaluated at the half-grid faces.  The result is
    negated twice, i.e. A itself is the (negative definite) discrete operator."""
    h = 1.0 / (N + 1)
    inv = 1.0 / (h * h)
    x = (np.arange(N) + 1) * h
    X, Y = np.meshgrid(x, x, indexing="xy")          # X[j,i] = x_i, Y[j,i] = y_j
    axp = ax(X + 0.5 * h, Y) * inv                    # face (i+1/2, j)
    axm = ax(X - 0.5 * h, Y) * inv
    ayp = ay(X, Y + 0.5 * h) * inv
    aym = ay(X, Y - 0.5 * h) * inv
    diag = -(axp + axm + ayp + aym)
    tx = axp.copy()
    tx[:, -1] = 0.0
    ty = ayp.copy()
    ty[-1, :] = 0.0
    n = N * N
    return Operator(kind="stencil7", n=n, nx=N, ny=N, nz=1, h=h,
                    diag=diag.ravel(), tx=tx.ravel(), ty=ty.ravel(), tz=np.zeros(n),
                    meta={"name": name, "N": N})


def fd1d_dense(N: int, a: float = 1.0) -> np.ndarray:
    """Dense N x N matrix of a u_zz by centred second differences on (0, 1),
    N interior points, h = 1/(N+1), zero Dirichlet boundary:
    (a/h^2) tridiag(1, -2, 1), symmetric negative definite (the small B of a
    separable 3-D operator split as A X + X B)."""
    h = 1.0 / (N + 1)
    B = np.zeros((N, N))
    i = np.arange(N)
    B[i, i] = -2.0 * a / (h * h)
    B[i[:-1], i[:-1] + 1] = a / (h * h)
    B[i[:-1] + 1, i[:-1]] = a / (h * h)
    return B


def fe_p1_2d(N: int):
    """Linear (P1) finite elements on the unit square, N x N interior nodes,
    h = 1/(N+1), every mesh square cut by its (i, j)-(i+1, j+1) diagonal, zero
    Dirichlet boundary.  Returns (A, E) as CSR operators: A = -K (K the
    stiffness matrix, so A is symmetric negative definite) and E = M (the
    consistent mass matrix, symmetric positive definite), both assembled from
    the element matrices; the pair of a semi-discrete heat equation
    M x' = -K x + C u and of its generalized Lyapunov equation."""
    import scipy.sparse as sp
    h = 1.0 / (N + 1)
    n = N * N
    P = N + 2                                         # nodes per line, boundary included
    gi, gj = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="xy")
    gi, gj = gi.ravel(), gj.ravel()
    node = lambda i, j: i + P * j                     # noqa: E731
    tris = np.concatenate([
        np.stack([node(gi, gj), node(gi + 1, gj), node(gi + 1, gj + 1)], axis=1),
        np.stack([node(gi, gj), node(gi + 1, gj + 1), node(gi, gj + 1)], axis=1)])
    # reference element: right triangle with legs h
    Ke = np.array([[1.0, -1.0, 0.0], [-1.0, 2.0, -1.0], [0.0, -1.0, 1.0]])
    Ke2 = np.array([[1.0, 0.0, -1.0], [0.0, 1.0, -1.0], [-1.0, -1.0, 2.0]])
    Me = (h * h / 24.0) * np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]])
    nt = tris.shape[0] // 2
    rows, cols, kv, mv = [], [], [], []
    for t_rng, Kloc in ((slice(0, nt), Ke), (slice(nt, 2 * nt), Ke2)):
        T = tris[t_rng]
        for a in range(3):
            for b in range(3):
                rows.append(T[:, a])
                cols.append(T[:, b])
                kv.append(np.full(T.shape[0], 0.5 * Kloc[a, b]))
                mv.append(np.full(T.shape[0], Me[a, b]))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    ii, jj = r % P, r // P
    ic, jc = c % P, c // P
    inner = (ii >= 1) & (ii <= N) & (jj >= 1) & (jj <= N) & (ic >= 1) & (ic <= N) & (jc >= 1) & (jc <= N)
    ri = (ii - 1) + N * (jj - 1)
    ci = (ic - 1) + N * (jc - 1)
    K = sp.csr_matrix((np.concatenate(kv)[inner], (ri[inner], ci[inner])), shape=(n, n))
    M = sp.csr_matrix((np.concatenate(mv)[inner], (ri[inner], ci[inner])), shape=(n, n))
    out = []
    for mat in (-K, M):
        mat = mat.tocsr()
        mat.sum_duplicates()
        mat.sort_indices()
        mat.eliminate_zeros()
        out.append(Operator(kind="csr", n=n, nx=N, ny=N, nz=1, h=h,
                            csr=(mat.indptr.astype(np.int64), mat.indices.astype(np.int32),
                                 mat.data.astype(np.float64)),
                            meta={"name": "fe_p1_2d", "N": N}))
    return out[0], out[1]


# ----------------------------------------------------------- right-hand sides
def random_band_T(k: int, ell: int, seed: int, delta: float = 1e-4):
    """A symmetric negative definite banded matrix of the shape of the
    projected matrix T_m (bandwidth ell, order k), for exercising the residual
    formula at sizes a short Krylov run does not reach: every band entry off
    the diagonal is 1 and the diagonal is -(2 ell + delta (1 + u)), u uniform
    in (0, 1) -- a Toeplitz symbol in [-(4 ell + delta), -delta] (so the
    eigenvalues range over [-(4 ell + 2 delta), -delta] like a stiff
    operator's Ritz values, and the eigenvectors spread over all rows) with
    the diagonal jitter keeping the eigenvalues distinct.  Returns
    (band, gamma, tau): band[c, d] = T[c + d, c] (k x (ell+1)), gamma ell x ell
    upper triangular with diagonal in (1, 2), tau ell x ell, drawn from
    ``numpy.random.default_rng([seed])`` and ``default_rng([seed, 1])``."""
    rng = np.random.default_rng([seed])
    band = np.zeros((k, ell + 1))
    band[:, 0] = -(2.0 * ell + delta) - delta * rng.random(k)
    for d in range(1, ell + 1):
        band[:k - d, d] = 1.0
    r2 = np.random.default_rng([seed, 1])
    gamma = np.triu(r2.uniform(-1.0, 1.0, (ell, ell)), 1) + np.diag(1.0 + r2.random(ell))
    tau = r2.uniform(-1.0, 1.0, (ell, ell))
    return band, gamma, tau


def gaussian_C(n: int, s: int, seed: int) -> np.ndarray:
    """n x s standard Gaussian, column c from ``default_rng([seed, c])`` so that
    the s=1 matrix is a prefix of any wider one.  Fortran (column-major) order."""
    C = np.empty((n, s), dtype=np.float64, order="F")
    for c in range(s):
        C[:, c] = np.random.default_rng([seed, c]).standard_normal(n)
    return C


def uniform_C(n: int, s: int, seed: int) -> np.ndarray:
    """n x s uniform on (0,1), then scaled to unit Frobenius norm (the
    right-hand sides of the paper's experiments).  Column-major."""
    C = np.empty((n, s), dtype=np.float64, order="F")
    for c in range(s):
        C[:, c] = np.random.default_rng([seed, c]).random(n)
    C /= np.linalg.norm(C)
    return C


def batch_c5(count: int = 64, master_seed: int = 6):
    """The batched workload: ``count`` independent equations with
    A_i = -(L_{N_i}/h_i^2 + c_i I), N_i ~ U{64..512}, c_i ~ U[0,10),
    s_i ~ U{1,2,4}, C_i Gaussian with seed 1000*master_seed + i."""
    rng = np.random.default_rng([master_seed])
    Ns = rng.integers(64, 513, size=count)
    cs = rng.random(count) * 10.0
    ss = rng.choice(np.array([1, 2, 4]), size=count)
    out = []
    for i in range(count):
        op = laplace2d(int(Ns[i]), shift=float(cs[i]))
        C = gaussian_C(op.n, int(ss[i]), 1000 * master_seed + i)
        out.append((op, C))
    return out
