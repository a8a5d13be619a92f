// Incomplete Cholesky IC(0) preconditioned CG in red-black order, run in its
// condensed form, for the inner solves A x = b of the extended Krylov method
// (Section 4 applies A^{-1} to a block at every step) on 5- and 7-point
// stencil operators.
//
// Colour the grid cells red (i + j + l even) and black (odd).  A stencil
// couples only cells of different colours, so with K = -A (SPD) in red-black
// order, K = [[D_r, E^T], [E, D_b]] with D_r, D_b diagonal.  IC(0) of that
// matrix is L = [[D_r^{1/2}, 0], [E D_r^{-1/2}, diag(Sigma)^{1/2}]] where
// Sigma = D_b - E D_r^{-1} E^T is the black Schur complement (every other
// entry of Sigma falls outside K's pattern and is dropped).  Hence M^{-1} K
// has the eigenvalue 1 on the red cells and the spectrum of
// diag(Sigma)^{-1} Sigma elsewhere, and PCG with M = L L^T advances like CG on
// Sigma x_b = rhs_b - E D_r^{-1} rhs_r preconditioned by diag(Sigma).  This
// file runs that condensed iteration: half the unknowns, no triangular solve
// (both triangular factors are explicit), then x_r = D_r^{-1}(rhs_r - E^T x_b).
//
// Layout: the black cells of grid line (j, l) sit at compact slots
// (j + ny l) hx + i / 2, hx = ceil(nx / 2) rounded up to a multiple of 4 (the
// slots past a line's last cell are padding: zero from allocation on, never
// written by the iteration).  The red cells use the same formula.  Vectors of the condensed iteration are
// row-interleaved (slot q holds its S right-hand-side entries contiguously).
//
// The iteration is the single-reduction (Chronopoulos-Gear) form of the
// Jacobi kernel in pcg.hip, two kernels per iteration: the update with
// v = D_r^{-1} E^T u at the red cells, then Sigma u = D_b u - E v with the
// next iteration's inner products.  (One kernel that took Sigma u at each black
// cell from u at the 19 black cells within two stencil steps, recomputed
// there, issued about 170 loads per black cell and ran 2.7 times slower.)
#include <cmath>

#include "pcg.hpp"
#include "pcnet.hpp"

namespace lyap {

namespace {

struct RbGeom {
  int nx, ny, nz, hx;
  int nb;  // compact slots: hx * ny * nz
};

// Natural coordinates of the cell of colour `odd` (0 red, 1 black) at slot q;
// false for a padding slot.
__device__ __forceinline__ bool rb_cell(const RbGeom& g, int q, int odd, int& i, int& j, int& l) {
  const int line = q / g.hx;
  const int h = q - line * g.hx;
  l = line / g.ny;
  j = line - l * g.ny;
  i = 2 * h + ((j + l + odd) & 1);
  return i < g.nx;
}

__device__ __forceinline__ int rb_slot(const RbGeom& g, int i, int j, int l) {
  return (j + g.ny * l) * g.hx + (i >> 1);
}

// K = -A: diagonal and the face transmissibilities (A's off-diagonal entries,
// K's are their negatives).  fx(r) couples r and r + 1, fy(r) r and r + nx,
// fz(r) r and r + nx ny.
template <bool K7>
__device__ __forceinline__ double kdiag(const OpDev<double>& op, int r) {
  if constexpr (K7) return -op.diag[r];
  else return -op.cc;
}
template <bool K7>
__device__ __forceinline__ double fx(const OpDev<double>& op, int r) {
  if constexpr (K7) return op.tx[r];
  else return op.co;
}
template <bool K7>
__device__ __forceinline__ double fy(const OpDev<double>& op, int r) {
  if constexpr (K7) return op.ty[r];
  else return op.co;
}
template <bool K7>
__device__ __forceinline__ double fz(const OpDev<double>& op, int r) {
  if constexpr (K7) return op.tz[r];
  else return op.co;
}

// Calls f(ni, nj, nl, nat, t, d) for each grid neighbour of cell (i, j, l)
// (natural index r) in the fixed order -z, -y, -x, +x, +y, +z (d = 0..5), t
// the transmissibility of the shared face.
template <bool K7, typename F>
__device__ __forceinline__ void for_neighbours(const OpDev<double>& op, const RbGeom& g, int i, int j, int l, int r,
                                               F&& f) {
  const int nx = g.nx, nxy = g.nx * g.ny;
  if (l > 0) f(i, j, l - 1, r - nxy, fz<K7>(op, r - nxy), 0);
  if (j > 0) f(i, j - 1, l, r - nx, fy<K7>(op, r - nx), 1);
  if (i > 0) f(i - 1, j, l, r - 1, fx<K7>(op, r - 1), 2);
  if (i < nx - 1) f(i + 1, j, l, r + 1, fx<K7>(op, r), 3);
  if (j < g.ny - 1) f(i, j + 1, l, r + nx, fy<K7>(op, r), 4);
  if (l < g.nz - 1) f(i, j, l + 1, r + nxy, fz<K7>(op, r), 5);
}

// Once per operator: rinv = 1 / D_r at the red slots; at the black slots
// db = D_b and sinv = 1 / Sigma_bb, Sigma_bb = D_b - sum_r t_br^2 / D_r.
// flag[0] = 1 when a pivot is not positive.
template <bool K7>
__global__ void k_rb_setup(OpDev<double> op, RbGeom g, double* __restrict__ rinv, double* __restrict__ db,
                           double* __restrict__ sinv, int* flag) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < g.nb; q += gridDim.x * blockDim.x) {
    int i, j, l;
    if (rb_cell(g, q, 0, i, j, l)) {
      const double d = kdiag<K7>(op, i + g.nx * (j + g.ny * l));
      if (!(d > 0.0)) flag[0] = 1;
      rinv[q] = 1.0 / d;
    }
    if (rb_cell(g, q, 1, i, j, l)) {
      const int r = i + g.nx * (j + g.ny * l);
      const double d = kdiag<K7>(op, r);
      double sig = d;
      for_neighbours<K7>(op, g, i, j, l, r, [&](int, int, int, int rr, double t, int) {
        sig -= t * t / kdiag<K7>(op, rr);
      });
      if (!(d > 0.0) || !(sig > 0.0)) flag[0] = 1;
      db[q] = d;
      sinv[q] = 1.0 / sig;
    }
  }
}

// Condensed right-hand side of a (re)start: with res the residual of
// K x = -B on the whole grid (mode 0: x = 0, res = -B; mode 1: res = R, the
// natural-order residual A x - B), rt_b = res_b - E D_r^{-1} res_r
// = res_b + sum_r t_br res_r / D_r at the black slots, and xb = 0.  Partials:
// B^T B over all cells (each slot covers one red and one black cell).
template <bool K7, int S, int NT>
__global__ __launch_bounds__(NT) void k_rb_rhs(OpDev<double> op, RbGeom g, const double* __restrict__ B,
                                               const double* __restrict__ R, int mode,
                                               const double* __restrict__ rinv, double* __restrict__ rt,
                                               double* __restrict__ xb, double* pout) {
  __shared__ double red[pow2_at_least(S) * (NT / 64)];
  double acc[S];
#pragma unroll
  for (int c = 0; c < S; ++c) acc[c] = 0.0;
  auto res = [&](int r, double (&v)[S]) {
    if (mode == 0) {
      load_row<double, S>(B + (size_t)r * S, v);
#pragma unroll
      for (int c = 0; c < S; ++c) v[c] = -v[c];
    } else {
      load_row<double, S>(R + (size_t)r * S, v);
    }
  };
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, g.nb, lo, hi);
  for (int q = lo + threadIdx.x; q < hi; q += NT) {
    int i, j, l;
    if (rb_cell(g, q, 0, i, j, l)) {
      double bv[S];
      load_row<double, S>(B + (size_t)(i + g.nx * (j + g.ny * l)) * S, bv);
#pragma unroll
      for (int c = 0; c < S; ++c) acc[c] = fma(bv[c], bv[c], acc[c]);
    }
    if (rb_cell(g, q, 1, i, j, l)) {
      const int r = i + g.nx * (j + g.ny * l);
      double bv[S], v[S];
      load_row<double, S>(B + (size_t)r * S, bv);
#pragma unroll
      for (int c = 0; c < S; ++c) acc[c] = fma(bv[c], bv[c], acc[c]);
      res(r, v);
      for_neighbours<K7>(op, g, i, j, l, r, [&](int ri, int rj, int rl, int rr, double t, int) {
        double w[S];
        res(rr, w);
        const double f = t * rinv[rb_slot(g, ri, rj, rl)];
#pragma unroll
        for (int c = 0; c < S; ++c) v[c] = fma(f, w[c], v[c]);
      });
      store_row<double, S>(rt + (size_t)q * S, v);
      double z[S];
#pragma unroll
      for (int c = 0; c < S; ++c) z[c] = 0.0;
      store_row<double, S>(xb + (size_t)q * S, z);
    }
  }
  write_partial<S, NT>(acc, red, pout);
}

// state[c] = eta2 * (B^T B)_c: the recursive threshold of every iteration
// (||r_b|| <= eta_rec ||b|| per column).
template <int S>
__global__ __launch_bounds__(256) void k_rb_thr(const double* pin, int nparts, double eta2, double* state) {
  __shared__ double red[pow2_at_least(S) * 4];
  reduce_partials<S, 256>(pin, nparts, red);
  if (threadIdx.x < S) state[threadIdx.x] = eta2 * red[threadIdx.x];
}

// The product Sigma u = D_b u - E D_r^{-1} E^T u is taken in two sweeps, each
// one kernel over the compact slots: v = D_r^{-1} (T^T u) at the red cells
// (T = -E, the transmissibilities), then D_b u - T v at the black cells.
//
// Sweep 1 of an iteration (it counted from the start of this (re)start),
// the single-reduction CG update at the black slot and v at the red slot:
//   beta = gamma_i / gamma_{i-1},  alpha = gamma_i / (delta_i - beta gamma_i / alpha_{i-1}),
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//   u = diag(Sigma)^{-1} r  (stored),
// and at the red cell v = D_r^{-1} sum_b t_rb u_b with u at its black
// neighbours recomputed from their previous r, w, s (the same operations as
// their own update, so the same bits).  START: no update (u = diag(Sigma)^{-1} r
// of the given r).  A column whose r.r is at most state[c] is frozen
// (alpha = beta = 0).
template <bool K7, int S, int NT, bool START>
__global__ __launch_bounds__(NT) void k_rb_upd(OpDev<double> op, RbGeom g, const double* __restrict__ rinv,
                                               const double* __restrict__ sinv, double* __restrict__ x,
                                               const double* __restrict__ rin, double* __restrict__ rout,
                                               const double* __restrict__ win, double* __restrict__ p,
                                               const double* __restrict__ sin, double* __restrict__ sout,
                                               double* __restrict__ u, double* __restrict__ v, CgIter* log, int it,
                                               const double* state, const double* pin, int nparts, int* flag) {
  double alpha[S], beta[S];
#pragma unroll
  for (int c = 0; c < S; ++c) alpha[c] = beta[c] = 0.0;
  if constexpr (!START) {
    __shared__ double red[pow2_at_least(3 * S) * (NT / 64)];
    reduce_partials<3 * S, NT>(pin, nparts, red);
#pragma unroll
    for (int c = 0; c < S; ++c) {
      const double gm = uniform_d(red[c]);
      const double dl = uniform_d(red[S + c]);
      const double rr = uniform_d(red[2 * S + c]);
      const bool active = rr > uniform_d(state[c]);
      double a = 0.0, b = 0.0;
      bool bad = false;
      if (active) {
        if (it == 0) {
          bad = !(dl > 0.0);
          a = bad ? 0.0 : gm / dl;
        } else {
          const double gp = uniform_d(log[it - 1].rho[c]);
          const double ap = uniform_d(log[it - 1].alpha[c]);
          b = gm / gp;
          const double den = dl - b * gm / ap;
          bad = !(den > 0.0) || !(gp > 0.0) || !(ap > 0.0);
          a = bad ? 0.0 : gm / den;
          if (bad) b = 0.0;
        }
      }
      alpha[c] = a;
      beta[c] = b;
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        log[it].rho[c] = gm;
        log[it].rr[c] = rr;
        log[it].sigma[c] = dl;
        log[it].alpha[c] = a;
        if (bad) flag[1] = it + 1;
      }
    }
  }
  const double* so = (!START && it > 0) ? sin : nullptr;
  // u of the new iterate at black slot q from the previous r, w, s there
  auto ueval = [&](int q, double (&uv)[S]) {
    double rv[S];
    load_row<double, S>(rin + (size_t)q * S, rv);
    const double m = sinv[q];
    if constexpr (START) {
#pragma unroll
      for (int c = 0; c < S; ++c) uv[c] = m * rv[c];
    } else {
      double wv[S];
      load_row<double, S>(win + (size_t)q * S, wv);
      if (so) {
        double sv[S];
        load_row<double, S>(so + (size_t)q * S, sv);
#pragma unroll
        for (int c = 0; c < S; ++c) wv[c] = fma(beta[c], sv[c], wv[c]);
      }
#pragma unroll
      for (int c = 0; c < S; ++c) uv[c] = m * fma(-alpha[c], wv[c], rv[c]);
    }
  };
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, g.nb, lo, hi);
  for (int q = lo + threadIdx.x; q < hi; q += NT) {
    int i, j, l;
    if (rb_cell(g, q, 1, i, j, l)) {
      double rv[S], uv[S];
      load_row<double, S>(rin + (size_t)q * S, rv);
      const double m = sinv[q];
      if constexpr (START) {
#pragma unroll
        for (int c = 0; c < S; ++c) uv[c] = m * rv[c];
      } else {
        double wv[S], pv[S], sv[S], xv[S];
        load_row<double, S>(win + (size_t)q * S, wv);
        load_row<double, S>(x + (size_t)q * S, xv);
        if (so) {
          load_row<double, S>(p + (size_t)q * S, pv);
          load_row<double, S>(so + (size_t)q * S, sv);
        } else {
#pragma unroll
          for (int c = 0; c < S; ++c) pv[c] = sv[c] = 0.0;
        }
#pragma unroll
        for (int c = 0; c < S; ++c) {
          pv[c] = fma(beta[c], pv[c], m * rv[c]);
          sv[c] = fma(beta[c], sv[c], wv[c]);
          xv[c] = fma(alpha[c], pv[c], xv[c]);
          rv[c] = fma(-alpha[c], sv[c], rv[c]);
          uv[c] = m * rv[c];
        }
        store_row<double, S>(p + (size_t)q * S, pv);
        store_row<double, S>(sout + (size_t)q * S, sv);
        store_row<double, S>(x + (size_t)q * S, xv);
        store_row<double, S>(rout + (size_t)q * S, rv);
      }
      store_row<double, S>(u + (size_t)q * S, uv);
    }
    if (rb_cell(g, q, 0, i, j, l)) {
      double acc[S];
#pragma unroll
      for (int c = 0; c < S; ++c) acc[c] = 0.0;
      for_neighbours<K7>(op, g, i, j, l, i + g.nx * (j + g.ny * l), [&](int bi, int bj, int bl, int, double t, int) {
        double uv[S];
        ueval(rb_slot(g, bi, bj, bl), uv);
#pragma unroll
        for (int c = 0; c < S; ++c) acc[c] = fma(t, uv[c], acc[c]);
      });
      const double ri = rinv[q];
#pragma unroll
      for (int c = 0; c < S; ++c) acc[c] *= ri;
      store_row<double, S>(v + (size_t)q * S, acc);
    }
  }
}

// Sweep 2: w = Sigma u = D_b u - sum_r t_br v_r at the black slots, and the
// partials gamma = r.u, delta = w.u, r.r of the next iteration.
template <bool K7, int S, int NT>
__global__ __launch_bounds__(NT) void k_rb_w(OpDev<double> op, RbGeom g, const double* __restrict__ db,
                                             const double* __restrict__ r, const double* __restrict__ u,
                                             const double* __restrict__ v, double* __restrict__ w, double* pout) {
  __shared__ double red[pow2_at_least(3 * S) * (NT / 64)];
  double acc[3 * S];
#pragma unroll
  for (int c = 0; c < 3 * S; ++c) acc[c] = 0.0;
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, g.nb, lo, hi);
  for (int q = lo + threadIdx.x; q < hi; q += NT) {
    int i, j, l;
    if (!rb_cell(g, q, 1, i, j, l)) continue;
    double rv[S], uv[S], wv[S];
    load_row<double, S>(r + (size_t)q * S, rv);
    load_row<double, S>(u + (size_t)q * S, uv);
    const double d = db[q];
#pragma unroll
    for (int c = 0; c < S; ++c) wv[c] = d * uv[c];
    for_neighbours<K7>(op, g, i, j, l, i + g.nx * (j + g.ny * l), [&](int ri, int rj, int rl, int, double t, int) {
      double vv[S];
      load_row<double, S>(v + (size_t)rb_slot(g, ri, rj, rl) * S, vv);
#pragma unroll
      for (int c = 0; c < S; ++c) wv[c] = fma(-t, vv[c], wv[c]);
    });
#pragma unroll
    for (int c = 0; c < S; ++c) {
      acc[c] = fma(rv[c], uv[c], acc[c]);
      acc[S + c] = fma(wv[c], uv[c], acc[S + c]);
      acc[2 * S + c] = fma(rv[c], rv[c], acc[2 * S + c]);
    }
    store_row<double, S>(w + (size_t)q * S, wv);
  }
  write_partial<3 * S, NT>(acc, red, pout);
}

// Back to the whole grid: X_b (+)= xb, X_r (+)= D_r^{-1} (res_r + sum_b t_rb xb_b)
// with res as in k_rb_rhs (mode 0 overwrites X, mode 1 adds the correction).
template <bool K7, int S>
__global__ void k_rb_finish(OpDev<double> op, RbGeom g, const double* __restrict__ B, const double* __restrict__ R,
                            int mode, const double* __restrict__ rinv, const double* __restrict__ xb,
                            double* __restrict__ X) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < g.nb; q += gridDim.x * blockDim.x) {
    int i, j, l;
    if (rb_cell(g, q, 1, i, j, l)) {
      const int r = i + g.nx * (j + g.ny * l);
      double v[S];
      load_row<double, S>(xb + (size_t)q * S, v);
      if (mode == 1) {
        double xv[S];
        load_row<double, S>(X + (size_t)r * S, xv);
#pragma unroll
        for (int c = 0; c < S; ++c) v[c] += xv[c];
      }
      store_row<double, S>(X + (size_t)r * S, v);
    }
    if (rb_cell(g, q, 0, i, j, l)) {
      const int r = i + g.nx * (j + g.ny * l);
      double v[S];
      if (mode == 0) {
        load_row<double, S>(B + (size_t)r * S, v);
#pragma unroll
        for (int c = 0; c < S; ++c) v[c] = -v[c];
      } else {
        load_row<double, S>(R + (size_t)r * S, v);
      }
      for_neighbours<K7>(op, g, i, j, l, r, [&](int bi, int bj, int bl, int, double t, int) {
        double w[S];
        load_row<double, S>(xb + (size_t)rb_slot(g, bi, bj, bl) * S, w);
#pragma unroll
        for (int c = 0; c < S; ++c) v[c] = fma(t, w[c], v[c]);
      });
      const double ri = rinv[q];
#pragma unroll
      for (int c = 0; c < S; ++c) v[c] *= ri;
      if (mode == 1) {
        double xv[S];
        load_row<double, S>(X + (size_t)r * S, xv);
#pragma unroll
        for (int c = 0; c < S; ++c) v[c] += xv[c];
      }
      store_row<double, S>(X + (size_t)r * S, v);
    }
  }
}

// ------------------------------------------------------------------ Sigma x for a given x
// (one right-hand side, compact black slots; the network's training applies it)
// v = D_r^{-1} T^T x at the red slots
template <bool K7>
__global__ void k_rb_vx(OpDev<double> op, RbGeom g, const double* __restrict__ rinv, const double* __restrict__ x,
                        double* __restrict__ v) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < g.nb; q += gridDim.x * blockDim.x) {
    int i, j, l;
    if (!rb_cell(g, q, 0, i, j, l)) continue;
    double acc = 0.0;
    for_neighbours<K7>(op, g, i, j, l, i + g.nx * (j + g.ny * l),
                       [&](int bi, int bj, int bl, int, double t, int) { acc = fma(t, x[rb_slot(g, bi, bj, bl)], acc); });
    v[q] = acc * rinv[q];
  }
}

// y = D_b x - T v at the black slots, 0 at the padding slots
template <bool K7>
__global__ void k_rb_yx(OpDev<double> op, RbGeom g, const double* __restrict__ db, const double* __restrict__ x,
                        const double* __restrict__ v, double* __restrict__ y) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < g.nb; q += gridDim.x * blockDim.x) {
    int i, j, l;
    if (!rb_cell(g, q, 1, i, j, l)) {
      y[q] = 0.0;
      continue;
    }
    double acc = db[q] * x[q];
    for_neighbours<K7>(op, g, i, j, l, i + g.nx * (j + g.ny * l),
                       [&](int ri, int rj, int rl, int, double t, int) { acc = fma(-t, v[rb_slot(g, ri, rj, rl)], acc); });
    y[q] = acc;
  }
}

// e_i = x* - x_i in place over the compact slots
__global__ void k_rb_err(const double* __restrict__ xs, double* __restrict__ xi, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) xi[p] = xs[p] - xi[p];
}

// ------------------------------------------------------------------ flexible CG on Sigma
// with the network z = M(r) (one right-hand side).  Per iteration: sweep A
// (direction at the black slots, v = D_r^{-1} T^T p at the red slots), sweep B
// (q = Sigma p, partials p.q and p.r), the update (x, r, partial r.r), then
// the network.

// partial r.r over the black slots
template <int NT>
__global__ __launch_bounds__(NT) void k_rbf_rr(RbGeom g, const double* __restrict__ r, double* pout) {
  __shared__ double red[NT / 64];
  double acc[1] = {0.0};
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, g.nb, lo, hi);
  for (int q = lo + threadIdx.x; q < hi; q += NT) acc[0] = fma(r[q], r[q], acc[0]);
  write_partial<1, NT>(acc, red, pout);
}

// Sweep A: beta = -(z.q_old) / (p_old.q_old) (0 at it = 0), p = z + beta p_old
// (0 once r.r <= state); v = D_r^{-1} T^T p at the red slots, by linearity from
// z at the black neighbours and the previous iteration's v.
template <bool K7, int NT>
__global__ __launch_bounds__(NT) void k_rbf_dira(OpDev<double> op, RbGeom g, const double* __restrict__ rinv,
                                                 const double* __restrict__ z, const double* __restrict__ pold,
                                                 double* __restrict__ pnew, double* __restrict__ v, CgIter* log, int it,
                                                 const double* state, const double* partR, int nparts,
                                                 const double* partZ, int nzparts) {
  __shared__ double red[2 * (NT / 64) + 2];
  // r.r of the updated residual and (after the first iteration) z.q_old
  reduce_partials_pair<NT>(partR, nparts, partZ, it > 0 ? nzparts : 0, red);
  const double rr = uniform_d(red[0]);
  const double zq = uniform_d(red[1]);
  const bool active = rr > uniform_d(state[0]);
  const double pq_old = it > 0 ? uniform_d(log[it - 1].sigma[0]) : 1.0;
  const double beta = (active && it > 0 && pq_old > 0.0) ? -zq / pq_old : 0.0;
  const double mask = active ? 1.0 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) log[it].rr[0] = rr;
  const double* po = it > 0 ? pold : nullptr;
  auto prow = [&](int q) -> double { return mask * (po ? fma(beta, po[q], z[q]) : z[q]); };
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, g.nb, lo, hi);
  for (int q = lo + threadIdx.x; q < hi; q += NT) {
    int i, j, l;
    if (rb_cell(g, q, 1, i, j, l)) pnew[q] = prow(q);
    if (rb_cell(g, q, 0, i, j, l)) {
      // v = D_r^{-1} T^T p = D_r^{-1} T^T z + beta v_old (v_old = D_r^{-1} T^T p_old from
      // the previous iteration): the neighbours' z only, not their p recomputed
      double acc = 0.0;
      for_neighbours<K7>(op, g, i, j, l, i + g.nx * (j + g.ny * l),
                         [&](int bi, int bj, int bl, int, double t, int) { acc = fma(t, z[rb_slot(g, bi, bj, bl)], acc); });
      const double vz = acc * rinv[q];
      v[q] = mask * (po ? fma(beta, v[q], vz) : vz);
    }
  }
}

// Sweep B: q = D_b p - T v at the black slots (0 at padding); partials p.q, p.r
template <bool K7, int NT>
__global__ __launch_bounds__(NT) void k_rbf_dirb(OpDev<double> op, RbGeom g, const double* __restrict__ db,
                                                 const double* __restrict__ p, const double* __restrict__ v,
                                                 const double* __restrict__ r, double* __restrict__ qv, double* pout) {
  __shared__ double red[2 * (NT / 64)];
  double acc[2] = {0.0, 0.0};
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, g.nb, lo, hi);
  for (int q = lo + threadIdx.x; q < hi; q += NT) {
    int i, j, l;
    if (!rb_cell(g, q, 1, i, j, l)) {
      qv[q] = 0.0;
      continue;
    }
    const double pq = p[q];
    double w = db[q] * pq;
    for_neighbours<K7>(op, g, i, j, l, i + g.nx * (j + g.ny * l),
                       [&](int ri, int rj, int rl, int, double t, int) { w = fma(-t, v[rb_slot(g, ri, rj, rl)], w); });
    qv[q] = w;
    acc[0] = fma(pq, w, acc[0]);
    acc[1] = fma(pq, r[q], acc[1]);
  }
  write_partial<2, NT>(acc, red, pout);
}

inline RbGeom rb_geom(const OpDev<double>& op) {
  RbGeom g;
  g.nx = op.nx;
  g.ny = op.ny;
  g.nz = op.nz;
  g.hx = ((op.nx + 1) / 2 + 3) / 4 * 4;  // a multiple of 4 (the network's vector loads)
  g.nb = g.hx * g.ny * g.nz;
  return g;
}

}  // namespace

// ------------------------------------------------------------------ host
void InnerCG::setup_rb() {
  LYAP_REQUIRE(op_.kind == LYAP_OP_STENCIL5 || op_.kind == LYAP_OP_STENCIL7, LYAP_E_UNSUPPORTED,
               "IC(0) in red-black order needs a 5- or 7-point stencil operator (a grid to colour)");
  const RbGeom g = rb_geom(op_);
  const size_t slots = (size_t)g.nb;
  rb_rinv_.alloc(slots * sizeof(double));
  rb_db_.alloc(slots * sizeof(double));
  rb_sinv_.alloc(slots * sizeof(double));
  const size_t blk = slots * S_ * sizeof(double);
  for (DevBuf* b : {&rb_x_, &rb_p_, &rb_r0_, &rb_r1_, &rb_w0_, &rb_w1_, &rb_s0_, &rb_s1_, &rb_u_, &rb_v_}) {
    b->alloc(blk);
    LYAP_HIP(hipMemsetAsync(b->p, 0, blk, st_));
  }
  for (DevBuf* b : {&rb_rinv_, &rb_db_, &rb_sinv_}) LYAP_HIP(hipMemsetAsync(b->p, 0, b->bytes, st_));
  rb_grid_ = stream_grid(g.nb);
  LYAP_HIP(hipMemsetAsync(flag_.p, 0, 64, st_));
  const int gs = grid_for(g.nb, 1, 1024);
  if (op_.kind == LYAP_OP_STENCIL7)
    hipLaunchKernelGGL((k_rb_setup<true>), dim3(gs), dim3(kBlock), 0, st_, op_, g, rb_rinv_.as<double>(),
                       rb_db_.as<double>(), rb_sinv_.as<double>(), flag_.as<int>());
  else
    hipLaunchKernelGGL((k_rb_setup<false>), dim3(gs), dim3(kBlock), 0, st_, op_, g, rb_rinv_.as<double>(),
                       rb_db_.as<double>(), rb_sinv_.as<double>(), flag_.as<int>());
  LYAP_LAUNCHED("k_rb_setup");
  int hf[2] = {0, 0};
  LYAP_HIP(hipMemcpyAsync(hf, flag_.p, sizeof(hf), hipMemcpyDeviceToHost, st_));
  LYAP_HIP(hipStreamSynchronize(st_));
  LYAP_REQUIRE(hf[0] == 0, LYAP_E_INDEFINITE,
               "IC(0) pivot is not positive: A is not negative definite with a diagonally dominant pattern");
  rb_ready_ = true;
}

void InnerCG::schur_apply(const double* x, double* y) {
  LYAP_REQUIRE(rb_ready_ && S_ == 1, LYAP_E_UNSUPPORTED, "Sigma x needs the red-black split and one column");
  const RbGeom g = rb_geom(op_);
  const int gs = grid_for(g.nb, 1, 1024);
  if (op_.kind == LYAP_OP_STENCIL7) {
    hipLaunchKernelGGL((k_rb_vx<true>), dim3(gs), dim3(kBlock), 0, st_, op_, g, rb_rinv_.as<double>(), x,
                       rb_v_.as<double>());
    hipLaunchKernelGGL((k_rb_yx<true>), dim3(gs), dim3(kBlock), 0, st_, op_, g, rb_db_.as<double>(), x,
                       rb_v_.as<double>(), y);
  } else {
    hipLaunchKernelGGL((k_rb_vx<false>), dim3(gs), dim3(kBlock), 0, st_, op_, g, rb_rinv_.as<double>(), x,
                       rb_v_.as<double>());
    hipLaunchKernelGGL((k_rb_yx<false>), dim3(gs), dim3(kBlock), 0, st_, op_, g, rb_db_.as<double>(), x,
                       rb_v_.as<double>(), y);
  }
  LYAP_LAUNCHED("schur_apply");
}

std::unique_ptr<PcNetGpu> InnerCG::make_schur_net(int C) {
  LYAP_REQUIRE(rb_ready_ && S_ == 1, LYAP_E_UNSUPPORTED,
               "the learned correction of IC(0) needs a stencil operator and one right-hand side");
  const RbGeom g = rb_geom(op_);
  return std::make_unique<PcNetGpu>(g.hx, g.ny, g.nz, rb_sinv_.as<double>(),
                                    [this](const double* x, double* y) { schur_apply(x, y); }, C, st_);
}

double InnerCG::rb_iter_bytes() const {
  // sweep 1 (LYAP_K_CG_DIR): at the black cells x, r, w, s, p and 1 / Sigma_bb in, x, r, s, p, u
  // out; at the red cells D_r^{-1} and the faces in, v out
  const double half = (double)n_ / 2.0;
  const double faces = op_.kind == LYAP_OP_STENCIL7 ? (op_.nz > 1 ? 3.0 : 2.0) * 8.0 * n_ : 0.0;
  return half * (10.0 * S_ * 8 + 8.0) + half * (8.0 + S_ * 8.0) + faces;
}

double InnerCG::rb_w_bytes() const {
  // sweep 2 (LYAP_K_CG_UPD): r, u, D_b at the black cells, v at the red cells and the faces in, w out
  const double half = (double)n_ / 2.0;
  const double faces = op_.kind == LYAP_OP_STENCIL7 ? (op_.nz > 1 ? 3.0 : 2.0) * 8.0 * n_ : 0.0;
  return half * (3.0 * S_ * 8 + 8.0) + half * S_ * 8.0 + faces;
}

template <bool K7, int S>
void InnerCG::rb_solve_templ(const double* B, double* X, int restarts, int chunk, KernelTimer* kt) {
  constexpr int NT = stream_threads(S);
  const auto t0 = Clock::now();
  const RbGeom g = rb_geom(op_);
  const double eta_rec = 0.5 * eta_;  // recursive target, so that the true residual passes
  const double eta2 = eta_rec * eta_rec;
  const int G = rb_grid_;
  double* rb[2] = {rb_r0_.as<double>(), rb_r1_.as<double>()};
  double* wb[2] = {rb_w0_.as<double>(), rb_w1_.as<double>()};
  double* sb[2] = {rb_s0_.as<double>(), rb_s1_.as<double>()};
  const double* rinv = rb_rinv_.as<double>();
  const double* db = rb_db_.as<double>();
  const double* sinv = rb_sinv_.as<double>();
  int total = 0;
  double worst = 0.0;
  for (int start = 0; start <= restarts; ++start) {
    const int mode = start == 0 ? 0 : 1;
    hipLaunchKernelGGL((k_rb_rhs<K7, S, NT>), dim3(G), dim3(NT), 0, st_, op_, g, B, r_.as<double>(), mode, rinv,
                       rb[0], rb_x_.as<double>(), partA_.as<double>());
    LYAP_LAUNCHED("k_rb_rhs");
    if (start == 0) {
      hipLaunchKernelGGL((k_rb_thr<S>), dim3(1), dim3(256), 0, st_, partA_.as<double>(), G, eta2,
                         state_.as<double>());
      LYAP_LAUNCHED("k_rb_thr");
    }
    hipLaunchKernelGGL((k_rb_upd<K7, S, NT, true>), dim3(G), dim3(NT), 0, st_, op_, g, rinv, sinv,
                       rb_x_.as<double>(), rb[0], rb[1], wb[0], rb_p_.as<double>(), sb[1], sb[0], rb_u_.as<double>(),
                       rb_v_.as<double>(), log_.as<CgIter>(), 0, state_.as<double>(), partA_.as<double>(), G,
                       flag_.as<int>());
    hipLaunchKernelGGL((k_rb_w<K7, S, NT>), dim3(G), dim3(NT), 0, st_, op_, g, db, rb[0], rb_u_.as<double>(),
                       rb_v_.as<double>(), wb[0], partA_.as<double>());
    LYAP_LAUNCHED("k_rb_start");
    int it = 0;
    bool done = false;
    const bool harvesting = S == 1 && harvest_every_ > 0 && start == 0;
    auto snapshot = [&]() {
      if (!harvesting || (int)hr_.size() >= harvest_keep_) return;
      const size_t bytes = (size_t)g.nb * sizeof(double);
      hr_.emplace_back(bytes);
      hx_.emplace_back(bytes);
      LYAP_HIP(hipMemcpyAsync(hr_.back().p, rb[it % 2], bytes, hipMemcpyDeviceToDevice, st_));
      LYAP_HIP(hipMemcpyAsync(hx_.back().p, rb_x_.p, bytes, hipMemcpyDeviceToDevice, st_));
    };
    snapshot();
    int nchk = 0;
    bool spec = false;  // the last chunk also computed x and its true residual
    const int gf = grid_for(g.nb, 1, 1024);
    while (!done && total + it < max_iter_) {
      const int it0 = it;
      int cnt = std::min(start == 0 ? chunk_len(it, nchk, chunk, chunk / 4) : chunk, max_iter_ - total - it);
      ++nchk;
      if (harvesting) cnt = std::min(cnt, harvest_every_ - it % harvest_every_);
      for (int c = 0; c < cnt; ++c, ++it) {
        if (kt) kt->mark(LYAP_K_CG_DIR);
        hipLaunchKernelGGL((k_rb_upd<K7, S, NT, false>), dim3(G), dim3(NT), 0, st_, op_, g, rinv, sinv,
                           rb_x_.as<double>(), rb[it % 2], rb[(it + 1) % 2], wb[it % 2], rb_p_.as<double>(),
                           sb[(it + 1) % 2], sb[it % 2], rb_u_.as<double>(), rb_v_.as<double>(), log_.as<CgIter>(),
                           it, state_.as<double>(), partA_.as<double>(), G, flag_.as<int>());
        if (kt) kt->mark(LYAP_K_CG_UPD);
        hipLaunchKernelGGL((k_rb_w<K7, S, NT>), dim3(G), dim3(NT), 0, st_, op_, g, db, rb[(it + 1) % 2],
                           rb_u_.as<double>(), rb_v_.as<double>(), wb[(it + 1) % 2], partA_.as<double>());
      }
      LYAP_LAUNCHED("k_rb_iter");
      if (kt) kt->collect();
      // a chunk expected to end the solve also forms x and its true residual
      // (x does not change after convergence; mode 0 overwrites X)
      spec = start == 0 && !harvesting && pred_ > 0;
      if (spec) {
        hipLaunchKernelGGL((k_rb_finish<K7, S>), dim3(gf), dim3(kBlock), 0, st_, op_, g, B, r_.as<double>(), 0, rinv,
                           rb_x_.as<double>(), X);
        spec_true(B, X);
      }
      LYAP_HIP(hipMemcpyAsync(hlog_.p, log_.as<CgIter>() + it0, (size_t)cnt * sizeof(CgIter), hipMemcpyDeviceToHost,
                              st_));
      LYAP_HIP(hipMemcpyAsync(htot_.as<char>() + 64 * sizeof(double), flag_.p, 8, hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipMemcpyAsync(htot_.p, state_.p, S * sizeof(double), hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipStreamSynchronize(st_));
      const int* hf = reinterpret_cast<const int*>(htot_.as<char>() + 64 * sizeof(double));
      LYAP_REQUIRE(hf[1] == 0, LYAP_E_INNER, "inner CG breakdown (p^T Sigma p <= 0) at iteration %d", hf[1]);
      const double* thr = htot_.as<double>();
      const CgIter* lg = hlog_.as<CgIter>();
      for (int c = 0; c < cnt && !done; ++c) {
        bool all = true;
        for (int k = 0; k < S; ++k) {
          LYAP_REQUIRE(std::isfinite(lg[c].rr[k]), LYAP_E_NUMERIC, "inner CG produced a non-finite residual");
          if (lg[c].rr[k] > thr[k]) all = false;
        }
        if (all) {
          done = true;
          it = it0 + c;  // iterations that changed x
        }
      }
      if (!done && harvesting && it % harvest_every_ == 0) snapshot();
    }
    total += it;
    if (start == 0 && done) learn_pred(it, nchk, chunk / 4, !harvesting);
    const double* h = htotT_.as<double>();
    if (!(done && spec)) {
      hipLaunchKernelGGL((k_rb_finish<K7, S>), dim3(gf), dim3(kBlock), 0, st_, op_, g, B, r_.as<double>(), mode, rinv,
                         rb_x_.as<double>(), X);
      LYAP_LAUNCHED("k_rb_finish");
      cg_true(op_, B, X, r_.as<double>(), n_, S, partA_.as<double>(), tot_.as<double>(), cgrid_, st_);
      LYAP_HIP(hipMemcpyAsync(htot_.p, tot_.p, 2 * S * sizeof(double), hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipStreamSynchronize(st_));
      h = htot_.as<double>();
    }
    worst = 0.0;
    for (int k = 0; k < S; ++k) {
      const double rel = h[S + k] > 0.0 ? std::sqrt(h[k] / h[S + k]) : 0.0;
      LYAP_REQUIRE(std::isfinite(rel), LYAP_E_NUMERIC, "inner solve produced non-finite values");
      worst = std::max(worst, rel);
    }
    if (worst <= eta_) {
      if (harvest_every_ > 0) {  // e_i = x* - x_i for the kept iterates (compact slots)
        for (auto& xi : hx_)
          hipLaunchKernelGGL(k_rb_err, dim3((g.nb + 255) / 256), dim3(256), 0, st_, rb_x_.as<double>(),
                             xi.as<double>(), g.nb);
        LYAP_LAUNCHED("k_rb_err");
        harvest_every_ = 0;
      }
      stats_.iters += total;
      stats_.solves += 1;
      stats_.restarts += start;
      stats_.worst_relres = std::max(stats_.worst_relres, worst);
      stats_.ms += ms_since(t0);
      return;
    }
    if (total >= max_iter_) break;
    // the restart starts from the true residual of x
    if (done && spec)
      LYAP_HIP(hipMemcpyAsync(r_.p, rt_.p, (size_t)n_ * S * sizeof(double), hipMemcpyDeviceToDevice, st_));
  }
  stats_.iters += total;
  stats_.worst_relres = std::max(stats_.worst_relres, worst);
  LYAP_REQUIRE(false, LYAP_E_INNER,
               "IC(0) CG did not reach the true relative residual %.1e in %d iterations", eta_, total);
}

template <bool K7>
static void rbf_launch_dir(hipStream_t st, int G, const OpDev<double>& op, const RbGeom& g, const double* rinv,
                           const double* db, const double* z, const double* po, double* pn, double* v,
                           const double* r, double* qv, CgIter* log, int it, const double* state,
                           const double* partR, int rparts, const double* partZ, int zparts, double* pout) {
  constexpr int NT = stream_threads(1);
  hipLaunchKernelGGL((k_rbf_dira<K7, NT>), dim3(G), dim3(NT), 0, st, op, g, rinv, z, po, pn, v, log, it, state,
                     partR, rparts, partZ, zparts);
  hipLaunchKernelGGL((k_rbf_dirb<K7, NT>), dim3(G), dim3(NT), 0, st, op, g, db, pn, v, r, qv, pout);
}

void InnerCG::solve_rb_fcg(const double* B, double* X, KernelTimer* kt) {
  constexpr int NT = stream_threads(1);
  constexpr int kChunk = 16, kRestarts = 3;
  const auto t0 = Clock::now();
  const RbGeom g = rb_geom(op_);
  const bool k7 = op_.kind == LYAP_OP_STENCIL7;
  const double eta_rec = 0.5 * eta_;
  const double eta2 = eta_rec * eta_rec;
  const int G = rb_grid_;
  const int gf = grid_for(g.nb, 1, 1024);
  const double* rinv = rb_rinv_.as<double>();
  const double* db = rb_db_.as<double>();
  double* x = rb_x_.as<double>();
  double* r = rb_r0_.as<double>();
  double* z = rb_u_.as<double>();
  double* qv = rb_w0_.as<double>();
  double* v = rb_v_.as<double>();
  double* pb[2] = {rb_p_.as<double>(), rb_s0_.as<double>()};
  if (!partZ_.p) partZ_.alloc((size_t)net_->max_out_parts() * sizeof(double));
  if (!partRR_.p) partRR_.alloc((size_t)net_->max_out_parts() * sizeof(double));
  // r alternates between two buffers: the update fused into the network's
  // first convolution reads the old r at the tile halos while writing the new
  double* rbuf[2] = {r, rb_r1_.as<double>()};
  int zparts = 0;
  int total = 0;
  double worst = 0.0;
  for (int start = 0; start <= kRestarts; ++start) {
    const int mode = start == 0 ? 0 : 1;
    if (k7)
      hipLaunchKernelGGL((k_rb_rhs<true, 1, NT>), dim3(G), dim3(NT), 0, st_, op_, g, B, r_.as<double>(), mode, rinv,
                         r, x, partA_.as<double>());
    else
      hipLaunchKernelGGL((k_rb_rhs<false, 1, NT>), dim3(G), dim3(NT), 0, st_, op_, g, B, r_.as<double>(), mode, rinv,
                         r, x, partA_.as<double>());
    if (start == 0)
      hipLaunchKernelGGL((k_rb_thr<1>), dim3(1), dim3(256), 0, st_, partA_.as<double>(), G, eta2, state_.as<double>());
    hipLaunchKernelGGL((k_rbf_rr<NT>), dim3(G), dim3(NT), 0, st_, g, r, partA_.as<double>());
    LYAP_LAUNCHED("k_rbf_start");
    net_->apply(r, z, nullptr, nullptr);
    int cur = 0;  // r in rbuf[cur] (the start's residual is in rbuf[0])
    const double* partR = partA_.as<double>();
    int rparts = G;
    int it = 0;
    bool done = false;
    int nchk = 0;
    bool spec = false;  // the last chunk also computed x and its true residual
    while (!done && total + it < max_iter_) {
      const int it0 = it;
      const int cnt = std::min(start == 0 ? chunk_len(it, nchk, kChunk, kChunk / 4) : kChunk, max_iter_ - total - it);
      ++nchk;
      for (int c = 0; c < cnt; ++c, ++it) {
        double* pn = pb[it % 2];
        const double* po = pb[(it + 1) % 2];
        if (kt) kt->mark(LYAP_K_CG_DIR);
        (k7 ? rbf_launch_dir<true> : rbf_launch_dir<false>)(st_, G, op_, g, rinv, db, z, po, pn, v, rbuf[cur], qv,
                                                          log_.as<CgIter>(), it, state_.as<double>(), partR, rparts,
                                                          partZ_.as<double>(), zparts, partB_.as<double>());
        LYAP_LAUNCHED("condensed fcg iteration");
        // x, r update fused into the network's first convolution; z = M r
        if (kt) kt->mark(LYAP_K_PCNET);
        const PcUpd u{x, rbuf[cur], rbuf[cur ^ 1], pn, qv, log_.as<CgIter>(), it, state_.as<double>(),
                      partB_.as<double>(), G, partRR_.as<double>(), flag_.as<int>()};
        zparts = net_->apply_upd(u, z, qv, partZ_.as<double>());
        cur ^= 1;
        partR = partRR_.as<double>();
        rparts = zparts;
      }
      if (kt) kt->collect();
      // a chunk expected to end the solve also forms x and its true residual
      // (x does not change after convergence; mode 0 overwrites X)
      spec = start == 0 && pred_ > 0;
      if (spec) {
        if (k7)
          hipLaunchKernelGGL((k_rb_finish<true, 1>), dim3(gf), dim3(kBlock), 0, st_, op_, g, B, r_.as<double>(), 0,
                             rinv, x, X);
        else
          hipLaunchKernelGGL((k_rb_finish<false, 1>), dim3(gf), dim3(kBlock), 0, st_, op_, g, B, r_.as<double>(), 0,
                             rinv, x, X);
        spec_true(B, X);
      }
      LYAP_HIP(hipMemcpyAsync(hlog_.p, log_.as<CgIter>() + it0, (size_t)cnt * sizeof(CgIter), hipMemcpyDeviceToHost,
                              st_));
      LYAP_HIP(hipMemcpyAsync(htot_.as<char>() + 64 * sizeof(double), flag_.p, 8, hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipMemcpyAsync(htot_.p, state_.p, sizeof(double), hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipStreamSynchronize(st_));
      const int* hf = reinterpret_cast<const int*>(htot_.as<char>() + 64 * sizeof(double));
      LYAP_REQUIRE(hf[1] == 0, LYAP_E_INNER, "flexible CG breakdown (p^T Sigma p <= 0) at iteration %d", hf[1]);
      const double thr = htot_.as<double>()[0];
      const CgIter* lg = hlog_.as<CgIter>();
      for (int c = 0; c < cnt && !done; ++c) {
        LYAP_REQUIRE(std::isfinite(lg[c].rr[0]), LYAP_E_NUMERIC, "flexible CG produced a non-finite residual");
        if (!(lg[c].rr[0] > thr)) {
          done = true;
          it = it0 + c;
        }
      }
    }
    total += it;
    if (start == 0 && done) learn_pred(it, nchk, kChunk / 4, true);
    const double* h = htotT_.as<double>();
    if (!(done && spec)) {
      if (k7)
        hipLaunchKernelGGL((k_rb_finish<true, 1>), dim3(gf), dim3(kBlock), 0, st_, op_, g, B, r_.as<double>(), mode,
                           rinv, x, X);
      else
        hipLaunchKernelGGL((k_rb_finish<false, 1>), dim3(gf), dim3(kBlock), 0, st_, op_, g, B, r_.as<double>(), mode,
                           rinv, x, X);
      LYAP_LAUNCHED("k_rb_finish");
      cg_true(op_, B, X, r_.as<double>(), n_, 1, partA_.as<double>(), tot_.as<double>(), cgrid_, st_);
      LYAP_HIP(hipMemcpyAsync(htot_.p, tot_.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipStreamSynchronize(st_));
      h = htot_.as<double>();
    }
    worst = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
    LYAP_REQUIRE(std::isfinite(worst), LYAP_E_NUMERIC, "inner solve produced non-finite values");
    if (worst <= eta_) {
      stats_.iters += total;
      stats_.solves += 1;
      stats_.restarts += start;
      stats_.worst_relres = std::max(stats_.worst_relres, worst);
      stats_.ms += ms_since(t0);
      return;
    }
    if (total >= max_iter_) break;
    // the restart starts from the true residual of x
    if (done && spec) LYAP_HIP(hipMemcpyAsync(r_.p, rt_.p, (size_t)n_ * sizeof(double), hipMemcpyDeviceToDevice, st_));
  }
  stats_.iters += total;
  stats_.worst_relres = std::max(stats_.worst_relres, worst);
  LYAP_REQUIRE(false, LYAP_E_INNER,
               "flexible CG on the Schur complement did not reach the true relative residual %.1e in %d iterations",
               eta_, total);
}

void InnerCG::solve_rb(const double* B, double* X, KernelTimer* kt) {
  const bool k7 = op_.kind == LYAP_OP_STENCIL7;
  constexpr int kChunk = 32, kRestarts = 3;
  switch (S_) {
    case 1: k7 ? rb_solve_templ<true, 1>(B, X, kRestarts, kChunk, kt)
               : rb_solve_templ<false, 1>(B, X, kRestarts, kChunk, kt); break;
    case 2: k7 ? rb_solve_templ<true, 2>(B, X, kRestarts, kChunk, kt)
               : rb_solve_templ<false, 2>(B, X, kRestarts, kChunk, kt); break;
    default: k7 ? rb_solve_templ<true, 4>(B, X, kRestarts, kChunk, kt)
                : rb_solve_templ<false, 4>(B, X, kRestarts, kChunk, kt); break;
  }
}

}  // namespace lyap
