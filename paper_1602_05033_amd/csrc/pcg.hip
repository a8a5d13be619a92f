// Preconditioned CG on -A for the inner solves of the extended Krylov method
// (and on the mass matrix for the generalized equation).
//
// With K = -A and the Jacobi preconditioner M, one iteration is a single
// streaming kernel (the single-reduction form below, k_cgcg_iter): the two
// inner products an iteration needs are taken in one grid-wide reduction, with
// the consumer-side scheme of the Lanczos step (each kernel writes one partial
// per workgroup, the next sums all partials in a fixed order).  The flexible
// CG of the learned preconditioner keeps two kernels per iteration (k_fcg_dir,
// k_fcg_upd), since its preconditioner is a network applied in between.
//
// The host launches iterations in chunks and reads the logged r^T r of each
// chunk once; a column whose recursive residual is below the threshold is
// frozen (alpha = beta = 0), so iterations after convergence change nothing.
// Every solve is then certified by the true residual ||b - A x|| / ||b||; a
// solve that fails it restarts from the current iterate (at most three times).
#include <cmath>

#include "pcg.hpp"
#include "pcnet.hpp"

namespace lyap {

constexpr int kCgChunk = 32;
constexpr int kCgRestarts = 3;

#define CG_ROWS(r, n) for (int r = blockIdx.x * NT + threadIdx.x; r < (n); r += gridDim.x * NT)

__global__ void k_cg_diag(OpDev<double> op, int n, int pc, double* dinv, int* flag) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const double d = -op_diag<double>(op, r);
    if (!(d > 0.0)) flag[0] = 1;
    dinv[r] = pc == LYAP_PC_NONE ? 1.0 : 1.0 / d;
  }
}

// mode 0: x = 0, r = -B (so that (-A) x = -B, i.e. A x = B); mode 1: r already
// holds the true residual of the current x.  Partials r^T z, r^T r.
template <int S, int NT>
__global__ __launch_bounds__(NT) void k_cg_init(const double* __restrict__ B, double* __restrict__ x,
                                                double* __restrict__ r, const double* __restrict__ dinv, int n,
                                                int mode, double* pout) {
  __shared__ double red[pow2_at_least(2 * S) * (NT / 64)];
  double acc[2 * S];
#pragma unroll
  for (int c = 0; c < 2 * S; ++c) acc[c] = 0.0;
  CG_ROWS(i, n) {
    double rv[S];
    if (mode == 0) {
      double bv[S], xv[S];
      load_row<double, S>(B + (size_t)i * S, bv);
#pragma unroll
      for (int c = 0; c < S; ++c) {
        rv[c] = -bv[c];
        xv[c] = 0.0;
      }
      store_row<double, S>(r + (size_t)i * S, rv);
      store_row<double, S>(x + (size_t)i * S, xv);
    } else {
      load_row<double, S>(r + (size_t)i * S, rv);
    }
    const double di = dinv[i];
#pragma unroll
    for (int c = 0; c < S; ++c) {
      acc[c] = fma(rv[c], rv[c] * di, acc[c]);
      acc[S + c] = fma(rv[c], rv[c], acc[S + c]);
    }
  }
  write_partial<2 * S, NT>(acc, red, pout);
}

// ------------------------------------------------------------------ single-reduction CG
// Preconditioned CG in the Chronopoulos-Gear form: with K = -A, M = D^{-1},
// u = M r and w = K u, the two inner products of an iteration, gamma = r.u and
// delta = w.u, are taken together, so one kernel (one grid-wide reduction)
// does a whole iteration:
//   beta = gamma_i / gamma_{i-1},  alpha = gamma_i / (delta_i - beta gamma_i / alpha_{i-1})
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//   u = M r,  w = K u  and the next gamma, delta, r.r.
// Mathematically the iterates are those of the two-kernel form above.  r, s
// and w are double buffered: the product K u at a row needs u = M r of the
// neighbouring rows, recomputed from the previous r, w, s there.

// u_j = M (r_j - alpha (w_j + beta s_j)) of the new iterate at row j.
template <int S>
__device__ __forceinline__ void cgcg_u(const double* __restrict__ r, const double* __restrict__ w,
                                       const double* __restrict__ sold, const double* __restrict__ dinv,
                                       const double (&alpha)[S], const double (&beta)[S], int j, double (&u)[S]) {
  double rv[S], wv[S];
  load_row<double, S>(r + (size_t)j * S, rv);
  load_row<double, S>(w + (size_t)j * S, wv);
  if (sold) {
    double sv[S];
    load_row<double, S>(sold + (size_t)j * S, sv);
#pragma unroll
    for (int c = 0; c < S; ++c) wv[c] = fma(beta[c], sv[c], wv[c]);
  }
  const double dj = dinv[j];
#pragma unroll
  for (int c = 0; c < S; ++c) u[c] = dj * fma(-alpha[c], wv[c], rv[c]);
}

// Start of a (re)started solve: r given, w = K M r; partials gamma, delta, r.r.
template <int S, int NT>
__global__ __launch_bounds__(NT) void k_cgcg_start(OpDev<double> op, const double* __restrict__ r,
                                                   const double* __restrict__ dinv, double* __restrict__ w,
                                                   double* pout, int n) {
  __shared__ double red[pow2_at_least(3 * S) * (NT / 64)];
  double acc[3 * S];
#pragma unroll
  for (int c = 0; c < 3 * S; ++c) acc[c] = 0.0;
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, n, lo, hi);
  for (int i = lo + threadIdx.x; i < hi; i += NT) {
    double wv[S], rv[S];
    op_row_fn<double, S>(op, i, [&](int j, double (&u)[S]) {
      double rj[S];
      load_row<double, S>(r + (size_t)j * S, rj);
      const double dj = dinv[j];
#pragma unroll
      for (int c = 0; c < S; ++c) u[c] = dj * rj[c];
    }, wv);
    load_row<double, S>(r + (size_t)i * S, rv);
    const double di = dinv[i];
#pragma unroll
    for (int c = 0; c < S; ++c) {
      wv[c] = -wv[c];
      const double u = di * rv[c];
      acc[c] = fma(rv[c], u, acc[c]);
      acc[S + c] = fma(wv[c], u, acc[S + c]);
      acc[2 * S + c] = fma(rv[c], rv[c], acc[2 * S + c]);
    }
    store_row<double, S>(w + (size_t)i * S, wv);
  }
  write_partial<3 * S, NT>(acc, red, pout);
}

// One iteration (it counted from the start of this (re)start).
template <int S, int NT>
__global__ __launch_bounds__(NT) void k_cgcg_iter(OpDev<double> op, double* __restrict__ x,
                                                  const double* __restrict__ rin, double* __restrict__ rout,
                                                  const double* __restrict__ win, double* __restrict__ wout,
                                                  double* __restrict__ p, const double* __restrict__ sin,
                                                  double* __restrict__ sout, const double* __restrict__ dinv,
                                                  CgIter* log, int it, int first, double* state, double eta2,
                                                  const double* pin, int nparts, double* pout, int* flag, int n) {
  __shared__ double red[pow2_at_least(3 * S) * (NT / 64)];
  reduce_partials<3 * S, NT>(pin, nparts, red);
  double alpha[S], beta[S];
#pragma unroll
  for (int c = 0; c < S; ++c) {
    const double g = uniform_d(red[c]);
    const double d = uniform_d(red[S + c]);
    const double rr = uniform_d(red[2 * S + c]);
    const double thr = (first && it == 0) ? eta2 * rr : uniform_d(state[c]);
    const bool active = rr > thr;
    double a = 0.0, b = 0.0;
    bool bad = false;
    if (active) {
      if (it == 0) {
        bad = !(d > 0.0);
        a = bad ? 0.0 : g / d;
      } else {
        const double gp = uniform_d(log[it - 1].rho[c]);
        const double ap = uniform_d(log[it - 1].alpha[c]);
        b = g / gp;
        const double den = d - b * g / ap;
        bad = !(den > 0.0) || !(gp > 0.0) || !(ap > 0.0);
        a = bad ? 0.0 : g / den;
        if (bad) b = 0.0;
      }
    }
    alpha[c] = a;
    beta[c] = b;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (first && it == 0) state[c] = thr;
      log[it].rho[c] = g;
      log[it].rr[c] = rr;
      log[it].sigma[c] = d;
      log[it].alpha[c] = a;
      if (bad) flag[1] = it + 1;
    }
  }
  __syncthreads();
  const double* so = it > 0 ? sin : nullptr;
  double acc[3 * S];
#pragma unroll
  for (int c = 0; c < 3 * S; ++c) acc[c] = 0.0;
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, n, lo, hi);
  for (int i = lo + threadIdx.x; i < hi; i += NT) {
    double rv[S], wv[S], pv[S], sv[S], xv[S];
    load_row<double, S>(rin + (size_t)i * S, rv);
    load_row<double, S>(win + (size_t)i * S, wv);
    load_row<double, S>(x + (size_t)i * S, xv);
    const double di = dinv[i];
    if (so) {
      load_row<double, S>(p + (size_t)i * S, pv);
      load_row<double, S>(so + (size_t)i * S, sv);
    } else {
#pragma unroll
      for (int c = 0; c < S; ++c) pv[c] = sv[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < S; ++c) {
      pv[c] = fma(beta[c], pv[c], di * rv[c]);
      sv[c] = fma(beta[c], sv[c], wv[c]);
      xv[c] = fma(alpha[c], pv[c], xv[c]);
      rv[c] = fma(-alpha[c], sv[c], rv[c]);
    }
    store_row<double, S>(p + (size_t)i * S, pv);
    store_row<double, S>(sout + (size_t)i * S, sv);
    store_row<double, S>(x + (size_t)i * S, xv);
    store_row<double, S>(rout + (size_t)i * S, rv);
    double wn[S];
    op_row_fn<double, S>(op, i, [&](int j, double (&u)[S]) { cgcg_u<S>(rin, win, so, dinv, alpha, beta, j, u); },
                         wn);
#pragma unroll
    for (int c = 0; c < S; ++c) {
      wn[c] = -wn[c];
      const double u = di * rv[c];
      acc[c] = fma(rv[c], u, acc[c]);
      acc[S + c] = fma(wn[c], u, acc[S + c]);
      acc[2 * S + c] = fma(rv[c], rv[c], acc[2 * S + c]);
    }
    store_row<double, S>(wout + (size_t)i * S, wn);
  }
  write_partial<3 * S, NT>(acc, red, pout);
}

// r = A x - B (the residual of (-A) x = -B); partials r^T r and B^T B.
template <int S, int NT>
__global__ __launch_bounds__(NT) void k_cg_true(OpDev<double> op, const double* __restrict__ B,
                                                const double* __restrict__ x, double* __restrict__ r, int n,
                                                double* pout) {
  __shared__ double red[pow2_at_least(2 * S) * (NT / 64)];
  double acc[2 * S];
#pragma unroll
  for (int c = 0; c < 2 * S; ++c) acc[c] = 0.0;
  CG_ROWS(i, n) {
    double w[S], bv[S];
    op_row<double, S>(op, x, i, w);
    load_row<double, S>(B + (size_t)i * S, bv);
#pragma unroll
    for (int c = 0; c < S; ++c) {
      w[c] = w[c] - bv[c];
      acc[c] = fma(w[c], w[c], acc[c]);
      acc[S + c] = fma(bv[c], bv[c], acc[S + c]);
    }
    store_row<double, S>(r + (size_t)i * S, w);
  }
  write_partial<2 * S, NT>(acc, red, pout);
}

template <int K>
__global__ __launch_bounds__(256) void k_sum_partials(const double* pin, int nparts, double* out) {
  __shared__ double red[pow2_at_least(K) * 4];
  reduce_partials<K, 256>(pin, nparts, red);
  if (threadIdx.x < K) out[threadIdx.x] = red[threadIdx.x];
}

// ------------------------------------------------------------------ flexible CG (one column)
// D: beta = -(z.q_old) / (p_old.q_old) (0 at it = 0); p = z + beta p_old;
//    q = (-A) p (rows of p recomputed from z, p_old); partials p.q, p.r
template <int NT>
__global__ __launch_bounds__(NT) void k_fcg_dir(OpDev<double> op, const double* __restrict__ z,
                                                const double* __restrict__ pold, double* __restrict__ pnew,
                                                double* __restrict__ q, const double* __restrict__ r, CgIter* log,
                                                int it, int first, double* state, double eta2, const double* partR,
                                                int nparts, const double* partZ, int nzparts, double* pout, int n) {
  __shared__ double red[pow2_at_least(2) * (NT / 64)];
  reduce_partials<2, NT>(partR, nparts, red);
  const double rr = uniform_d(red[1]);
  __syncthreads();
  double zq = 0.0;
  if (it > 0) {
    reduce_partials<1, NT>(partZ, nzparts, red);
    zq = uniform_d(red[0]);
    __syncthreads();
  }
  const double thr = (first && it == 0) ? eta2 * rr : uniform_d(state[0]);
  const bool active = rr > thr;
  const double pq_old = it > 0 ? uniform_d(log[it - 1].sigma[0]) : 1.0;
  const double beta = (active && it > 0 && pq_old > 0.0) ? -zq / pq_old : 0.0;
  const double mask = active ? 1.0 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (first && it == 0) state[0] = thr;
    log[it].rr[0] = rr;
  }
  const double* po = it > 0 ? pold : nullptr;
  auto prow = [&](int i) -> double {
    const double zi = z[i];
    return mask * (po ? fma(beta, po[i], zi) : zi);
  };
  double acc[2] = {0.0, 0.0};
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, n, lo, hi);
  for (int i = lo + threadIdx.x; i < hi; i += NT) {
    const double pi = prow(i);
    pnew[i] = pi;
    double w[1];
    op_row_fn<double, 1>(op, i, [&](int j, double (&v)[1]) { v[0] = prow(j); }, w);
    const double qi = -w[0];
    q[i] = qi;
    acc[0] = fma(pi, qi, acc[0]);
    acc[1] = fma(pi, r[i], acc[1]);
  }
  write_partial<2, NT>(acc, red, pout);
}

// U: alpha = p.r / p.q; x += alpha p; r -= alpha q; partials (r.r, r.r)
template <int NT>
__global__ __launch_bounds__(NT) void k_fcg_upd(double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ q, CgIter* log,
                                                int it, const double* state, const double* pin, int nparts,
                                                double* pout, int* flag, int n) {
  __shared__ double red[pow2_at_least(2) * (NT / 64)];
  reduce_partials<2, NT>(pin, nparts, red);
  const double pq = uniform_d(red[0]), pr = uniform_d(red[1]);
  __syncthreads();
  const bool active = uniform_d(log[it].rr[0]) > uniform_d(state[0]);
  const double alpha = (active && pq > 0.0) ? pr / pq : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    log[it].sigma[0] = pq;
    log[it].rho[0] = pr;
    log[it].alpha[0] = alpha;
    if (active && !(pq > 0.0)) flag[1] = it + 1;
  }
  double acc[2] = {0.0, 0.0};
  for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
    const double xi = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    x[i] = xi;
    r[i] = ri;
    acc[0] = fma(ri, ri, acc[0]);
  }
  acc[1] = acc[0];
  write_partial<2, NT>(acc, red, pout);
}

// e_i = x* - x_i in place
__global__ void k_cg_errors(const double* __restrict__ xs, double* __restrict__ xi, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) xi[p] = xs[p] - xi[p];
}

// ------------------------------------------------------------------ host
InnerCG::InnerCG(const OpDev<double>& op, int n, int S, int pc, double eta, int max_iter, hipStream_t st)
    : op_(op), n_(n), S_(S), pc_(pc), max_iter_(max_iter), eta_(eta), st_(st) {
  LYAP_REQUIRE(S == 1 || S == 2 || S == 4, LYAP_E_UNSUPPORTED, "inner CG supports 1, 2 or 4 right-hand sides");
  LYAP_REQUIRE(pc == LYAP_PC_NONE || pc == LYAP_PC_JACOBI || pc == LYAP_PC_IC0 || pc == LYAP_PC_LEARNED,
               LYAP_E_UNSUPPORTED, "inner preconditioner %d is not supported", pc);
  LYAP_REQUIRE(pc != LYAP_PC_LEARNED || S == 1, LYAP_E_UNSUPPORTED,
               "the learned preconditioner handles one right-hand side per solve");
  LYAP_REQUIRE(eta > 0.0 && eta < 1.0, LYAP_E_ARG, "inner_tol=%g must be in (0,1)", eta);
  LYAP_REQUIRE(max_iter >= 1, LYAP_E_ARG, "inner_max_iter must be >= 1");
  grid_ = stream_grid(n);
  // the single-reduction kernels use few registers (52 VGPRs at S = 1): once
  // one workgroup per CU would give each thread two rows or more, two
  // 1024-thread workgroups per CU hide more memory latency (C3: 1.30 -> 1.21 s);
  // below that the extra workgroups only add partials to reduce
  cgrid_ = (int64_t)n >= 2 * (int64_t)kSGrid * kSBlock ? 2 * kSGrid : grid_;
  const size_t blk = (size_t)n * S * sizeof(double);
  dinv_.alloc((size_t)n * sizeof(double));
  r_.alloc(blk);
  p0_.alloc(blk);
  p1_.alloc(blk);
  q_.alloc(blk);
  partA_.alloc((size_t)2 * kSGrid * 3 * S * sizeof(double));
  partB_.alloc((size_t)2 * kSGrid * 3 * S * sizeof(double));
  log_.alloc((size_t)(max_iter + kCgChunk) * sizeof(CgIter));
  state_.alloc(64 * sizeof(double));
  tot_.alloc(64 * sizeof(double));
  flag_.alloc(64);
  hlog_.alloc((size_t)(max_iter + kCgChunk) * sizeof(CgIter));  // a chunk may run to max_iter
  htot_.alloc(64 * sizeof(double) + 64);
  LYAP_HIP(hipMemsetAsync(flag_.p, 0, 64, st_));
  hipLaunchKernelGGL(k_cg_diag, dim3(grid_for(n, 1, 1024)), dim3(kBlock), 0, st_, op_, n_, pc_,
                     dinv_.as<double>(), flag_.as<int>());
  LYAP_LAUNCHED("k_cg_diag");
  int hf[2] = {0, 0};
  LYAP_HIP(hipMemcpyAsync(hf, flag_.p, sizeof(hf), hipMemcpyDeviceToHost, st_));
  LYAP_HIP(hipStreamSynchronize(st_));
  LYAP_REQUIRE(hf[0] == 0, LYAP_E_INDEFINITE, "A has a diagonal entry >= 0: not negative definite");
  if (pc_ == LYAP_PC_IC0 ||
      (pc_ == LYAP_PC_LEARNED && S_ == 1 && (op_.kind == LYAP_OP_STENCIL5 || op_.kind == LYAP_OP_STENCIL7)))
    setup_rb();
}

double InnerCG::iter_bytes() const {
  if (net_ && net_schur_) {
    // the two sweeps of q = Sigma p: z, p_old in and p out at the black slots, D_r^{-1}
    // and the faces, v out; then p, v, D_b, r in and q out with the faces again
    const double half = (double)n_ / 2.0;
    const double faces = op_.kind == LYAP_OP_STENCIL7 ? (op_.nz > 1 ? 3.0 : 2.0) * 8.0 * n_ : 0.0;
    return half * 24.0 + half * 16.0 + half * 40.0 + 2.0 * faces;
  }
  if (pc_ == LYAP_PC_IC0 || rb_ready_) return rb_iter_bytes();
  double coef = 0.0;
  if (op_.kind == LYAP_OP_STENCIL7) coef = 4.0 * 8.0;
  // single-reduction CG: x, r, w, s, p and M^{-1} in; x, r, w, s, p out (+ coefficients)
  return (double)n_ * (10.0 * S_ * 8 + 8 + coef);
}


template <int S>
static void cg_launch_init(const double* B, double* x, double* r, const double* dinv, int n, int mode, double* pout,
                           int grid, hipStream_t st) {
  constexpr int NT = stream_threads(S);
  hipLaunchKernelGGL((k_cg_init<S, NT>), dim3(grid), dim3(NT), 0, st, B, x, r, dinv, n, mode, pout);
  LYAP_LAUNCHED("k_cg_init");
}

template <int S>
static void cg_launch_cgcg_start(const OpDev<double>& op, const double* r, const double* dinv, double* w, double* pout,
                                 int n, int grid, hipStream_t st) {
  constexpr int NT = stream_threads(S);
  hipLaunchKernelGGL((k_cgcg_start<S, NT>), dim3(grid), dim3(NT), 0, st, op, r, dinv, w, pout, n);
  LYAP_LAUNCHED("k_cgcg_start");
}

template <int S>
static void cg_launch_cgcg_iter(const OpDev<double>& op, double* x, const double* rin, double* rout, const double* win,
                                double* wout, double* p, const double* sin, double* sout, const double* dinv,
                                CgIter* log, int it, int first, double* state, double eta2, const double* pin,
                                double* pout, int* flag, int n, int grid, hipStream_t st) {
  constexpr int NT = stream_threads(S);
  hipLaunchKernelGGL((k_cgcg_iter<S, NT>), dim3(grid), dim3(NT), 0, st, op, x, rin, rout, win, wout, p, sin, sout,
                     dinv, log, it, first, state, eta2, pin, grid, pout, flag, n);
  LYAP_LAUNCHED("k_cgcg_iter");
}

template <int S>
static void cg_launch_true(const OpDev<double>& op, const double* B, const double* x, double* r, int n, double* part,
                           double* tot, int grid, hipStream_t st) {
  constexpr int NT = stream_threads(S);
  hipLaunchKernelGGL((k_cg_true<S, NT>), dim3(grid), dim3(NT), 0, st, op, B, x, r, n, part);
  LYAP_LAUNCHED("k_cg_true");
  hipLaunchKernelGGL((k_sum_partials<2 * S>), dim3(1), dim3(256), 0, st, part, grid, tot);
  LYAP_LAUNCHED("k_sum_partials");
}

double InnerCG::upd_bytes() const {
  // (on the Schur complement the update is fused into the network's first convolution)
  if (net_ && net_schur_) return (double)n_ / 2.0 * 48.0;  // x, r, p, q in; x, r out (black slots)
  if (pc_ == LYAP_PC_IC0 || (rb_ready_ && !net_)) return rb_w_bytes();
  // the flexible-CG update of the learned-preconditioner runs: x, r, p, q in; x, r out
  return (double)n_ * (6.0 * S_ * 8 + 8);
}

void cg_true(const OpDev<double>& op, const double* B, const double* x, double* r, int n, int S, double* part,
             double* tot, int grid, hipStream_t st) {
  switch (S) {
    case 1: cg_launch_true<1>(op, B, x, r, n, part, tot, grid, st); break;
    case 2: cg_launch_true<2>(op, B, x, r, n, part, tot, grid, st); break;
    default: cg_launch_true<4>(op, B, x, r, n, part, tot, grid, st); break;
  }
}

void InnerCG::spec_true(const double* B, const double* X) {
  if (!rt_.p) {
    rt_.alloc((size_t)n_ * S_ * sizeof(double));
    partT_.alloc(partA_.bytes);
    totT_.alloc(64 * sizeof(double));
    htotT_.alloc(64 * sizeof(double));
  }
  cg_true(op_, B, X, rt_.as<double>(), n_, S_, partT_.as<double>(), totT_.as<double>(), cgrid_, st_);
  LYAP_HIP(hipMemcpyAsync(htotT_.p, totT_.p, 2 * S_ * sizeof(double), hipMemcpyDeviceToHost, st_));
}

void InnerCG::solve_fcg(const double* B, double* X, KernelTimer* kt) {
  const auto t0 = Clock::now();
  constexpr int NT = stream_threads(1);
  constexpr int kChunk = 16;
  const double eta_rec = 0.5 * eta_;
  const double eta2 = eta_rec * eta_rec;
  if (!z_.p) {
    z_.alloc((size_t)n_ * sizeof(double));
    partZ_.alloc((size_t)net_->max_out_parts() * sizeof(double));
  }
  int zparts = 0;
  int total = 0;
  double worst = 0.0;
  for (int start = 0; start <= kCgRestarts; ++start) {
    cg_launch_init<1>(B, X, r_.as<double>(), dinv_.as<double>(), n_, start == 0 ? 0 : 1, partA_.as<double>(), grid_,
                      st_);
    net_->apply(r_.as<double>(), z_.as<double>(), nullptr, nullptr);
    int it = 0;
    bool done = false;
    while (!done && total + it < max_iter_) {
      const int it0 = it;
      const int cnt = std::min(kChunk, max_iter_ - total - it);
      for (int c = 0; c < cnt; ++c, ++it) {
        double* pn = (it % 2 == 0) ? p0_.as<double>() : p1_.as<double>();
        const double* po = (it % 2 == 0) ? p1_.as<double>() : p0_.as<double>();
        if (kt) kt->mark(LYAP_K_CG_DIR);
        hipLaunchKernelGGL((k_fcg_dir<NT>), dim3(grid_), dim3(NT), 0, st_, op_, z_.as<double>(), po, pn,
                           q_.as<double>(), r_.as<double>(), log_.as<CgIter>(), it, start == 0 ? 1 : 0,
                           state_.as<double>(), eta2, partA_.as<double>(), grid_, partZ_.as<double>(), zparts,
                           partB_.as<double>(), n_);
        if (kt) kt->mark(LYAP_K_CG_UPD);
        hipLaunchKernelGGL((k_fcg_upd<NT>), dim3(grid_), dim3(NT), 0, st_, X, r_.as<double>(), pn, q_.as<double>(),
                           log_.as<CgIter>(), it, state_.as<double>(), partB_.as<double>(), grid_,
                           partA_.as<double>(), flag_.as<int>(), n_);
        LYAP_LAUNCHED("fcg iteration");
        if (kt) kt->mark(LYAP_K_PCNET);
        zparts = net_->apply(r_.as<double>(), z_.as<double>(), q_.as<double>(), partZ_.as<double>());
      }
      if (kt) kt->collect();
      LYAP_HIP(hipMemcpyAsync(hlog_.p, log_.as<CgIter>() + it0, (size_t)cnt * sizeof(CgIter), hipMemcpyDeviceToHost,
                              st_));
      LYAP_HIP(hipMemcpyAsync(htot_.as<char>() + 64 * sizeof(double), flag_.p, 8, hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipMemcpyAsync(htot_.p, state_.p, sizeof(double), hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipStreamSynchronize(st_));
      const int* hf = reinterpret_cast<const int*>(htot_.as<char>() + 64 * sizeof(double));
      LYAP_REQUIRE(hf[1] == 0, LYAP_E_INNER, "flexible CG breakdown (p^T A p <= 0) at iteration %d", hf[1]);
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
    cg_launch_true<1>(op_, B, X, r_.as<double>(), n_, partA_.as<double>(), tot_.as<double>(), grid_, st_);
    LYAP_HIP(hipMemcpyAsync(htot_.p, tot_.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st_));
    LYAP_HIP(hipStreamSynchronize(st_));
    const double* h = htot_.as<double>();
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
  }
  stats_.iters += total;
  stats_.worst_relres = std::max(stats_.worst_relres, worst);
  LYAP_REQUIRE(false, LYAP_E_INNER, "flexible CG did not reach the true relative residual %.1e in %d iterations",
               eta_, total);
}

void InnerCG::solve(const double* B, double* X, KernelTimer* kt) {
  if (net_) return net_schur_ ? solve_rb_fcg(B, X, kt) : solve_fcg(B, X, kt);
  if (rb_ready_) return solve_rb(B, X, kt);
  const auto t0 = Clock::now();
  const int S = S_;
  const double eta_rec = 0.5 * eta_;  // recursive target, so that the true residual passes
  const double eta2 = eta_rec * eta_rec;
  auto init = [&](int mode) {
    switch (S) {
      case 1: cg_launch_init<1>(B, X, r_.as<double>(), dinv_.as<double>(), n_, mode, partA_.as<double>(), cgrid_, st_); break;
      case 2: cg_launch_init<2>(B, X, r_.as<double>(), dinv_.as<double>(), n_, mode, partA_.as<double>(), cgrid_, st_); break;
      default: cg_launch_init<4>(B, X, r_.as<double>(), dinv_.as<double>(), n_, mode, partA_.as<double>(), cgrid_, st_); break;
    }
  };
  if (!w0_.p) {
    const size_t blk = (size_t)n_ * S * sizeof(double);
    r1_.alloc(blk);
    w0_.alloc(blk);
    w1_.alloc(blk);
    s0_.alloc(blk);
    s1_.alloc(blk);
  }
  // buffers of iteration it: r, w in [it % 2], out [(it + 1) % 2]; s out [it % 2]
  auto rbuf = [&](int k) { return (k % 2 == 0) ? r_.as<double>() : r1_.as<double>(); };
  auto wbuf = [&](int k) { return (k % 2 == 0) ? w0_.as<double>() : w1_.as<double>(); };
  auto sbuf = [&](int k) { return (k % 2 == 0) ? s0_.as<double>() : s1_.as<double>(); };
  auto start_k = [&]() {
    switch (S) {
      case 1: cg_launch_cgcg_start<1>(op_, r_.as<double>(), dinv_.as<double>(), w0_.as<double>(), partA_.as<double>(), n_, cgrid_, st_); break;
      case 2: cg_launch_cgcg_start<2>(op_, r_.as<double>(), dinv_.as<double>(), w0_.as<double>(), partA_.as<double>(), n_, cgrid_, st_); break;
      default: cg_launch_cgcg_start<4>(op_, r_.as<double>(), dinv_.as<double>(), w0_.as<double>(), partA_.as<double>(), n_, cgrid_, st_); break;
    }
  };
  auto iter = [&](int it, int first) {
    double* pin = (it % 2 == 0) ? partA_.as<double>() : partB_.as<double>();
    double* pout = (it % 2 == 0) ? partB_.as<double>() : partA_.as<double>();
    CgIter* lg = log_.as<CgIter>();
    if (kt) kt->mark(LYAP_K_CG_DIR);
    switch (S) {
      case 1: cg_launch_cgcg_iter<1>(op_, X, rbuf(it), rbuf(it + 1), wbuf(it), wbuf(it + 1), p0_.as<double>(),
                                     sbuf(it + 1), sbuf(it), dinv_.as<double>(), lg, it, first, state_.as<double>(),
                                     eta2, pin, pout, flag_.as<int>(), n_, cgrid_, st_); break;
      case 2: cg_launch_cgcg_iter<2>(op_, X, rbuf(it), rbuf(it + 1), wbuf(it), wbuf(it + 1), p0_.as<double>(),
                                     sbuf(it + 1), sbuf(it), dinv_.as<double>(), lg, it, first, state_.as<double>(),
                                     eta2, pin, pout, flag_.as<int>(), n_, cgrid_, st_); break;
      default: cg_launch_cgcg_iter<4>(op_, X, rbuf(it), rbuf(it + 1), wbuf(it), wbuf(it + 1), p0_.as<double>(),
                                      sbuf(it + 1), sbuf(it), dinv_.as<double>(), lg, it, first, state_.as<double>(),
                                      eta2, pin, pout, flag_.as<int>(), n_, cgrid_, st_); break;
    }
  };
  auto true_res = [&]() {
    switch (S) {
      case 1: cg_launch_true<1>(op_, B, X, r_.as<double>(), n_, partA_.as<double>(), tot_.as<double>(), cgrid_, st_); break;
      case 2: cg_launch_true<2>(op_, B, X, r_.as<double>(), n_, partA_.as<double>(), tot_.as<double>(), cgrid_, st_); break;
      default: cg_launch_true<4>(op_, B, X, r_.as<double>(), n_, partA_.as<double>(), tot_.as<double>(), cgrid_, st_); break;
    }
  };

  int total = 0;
  double worst = 0.0;
  for (int start = 0; start <= kCgRestarts; ++start) {
    init(start == 0 ? 0 : 1);
    start_k();
    int it = 0;
    bool done = false;
    const bool harvesting = harvest_every_ > 0 && start == 0;
    auto snapshot = [&]() {
      if (!harvesting || (int)hr_.size() >= harvest_keep_) return;
      hr_.emplace_back((size_t)n_ * S * sizeof(double));
      hx_.emplace_back((size_t)n_ * S * sizeof(double));
      LYAP_HIP(hipMemcpyAsync(hr_.back().p, rbuf(it), (size_t)n_ * S * sizeof(double), hipMemcpyDeviceToDevice, st_));
      LYAP_HIP(hipMemcpyAsync(hx_.back().p, X, (size_t)n_ * S * sizeof(double), hipMemcpyDeviceToDevice, st_));
    };
    snapshot();
    int nchk = 0;
    bool spec = false;  // the last chunk also computed the true residual of X
    while (!done && total + it < max_iter_) {
      const int it0 = it;
      const int want = start == 0 && !harvesting ? chunk_len(it, nchk, kCgChunk, kCgChunk / 4) : kCgChunk;
      const int cnt = std::min(want, max_iter_ - total - it);
      ++nchk;
      for (int c = 0; c < cnt; ++c) iter(it++, start == 0 ? 1 : 0);
      if (harvesting && it % std::max(1, harvest_every_) == 0) snapshot();
      kt ? kt->collect() : (void)0;
      // when the chunk is expected to end the solve, its true residual goes
      // out with the same host wait (X does not change after convergence)
      spec = start == 0 && !harvesting && pred_ > 0;
      if (spec) spec_true(B, X);
      LYAP_HIP(hipMemcpyAsync(hlog_.p, log_.as<CgIter>() + it0, (size_t)cnt * sizeof(CgIter), hipMemcpyDeviceToHost,
                              st_));
      LYAP_HIP(hipMemcpyAsync(htot_.as<char>() + 64 * sizeof(double), flag_.p, 8, hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipMemcpyAsync(htot_.p, state_.p, S * sizeof(double), hipMemcpyDeviceToHost, st_));
      LYAP_HIP(hipStreamSynchronize(st_));
      const int* hf = reinterpret_cast<const int*>(htot_.as<char>() + 64 * sizeof(double));
      LYAP_REQUIRE(hf[1] == 0, LYAP_E_INNER, "inner CG breakdown (p^T A p <= 0) at iteration %d", hf[1]);
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
    }
    total += it;
    if (start == 0 && done) learn_pred(it, nchk, kCgChunk / 4, !harvesting);
    const double* h = htotT_.as<double>();
    if (!(done && spec)) {
      true_res();
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
      if (harvest_every_ > 0) {  // e_i = x* - x_i for the kept iterates
        for (auto& x : hx_)
          hipLaunchKernelGGL(k_cg_errors, dim3((n_ * S + 255) / 256), dim3(256), 0, st_, X, x.as<double>(), n_ * S);
        LYAP_LAUNCHED("k_cg_errors");
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
  LYAP_REQUIRE(false, LYAP_E_INNER, "inner CG did not reach the true relative residual %.1e in %d iterations", eta_,
               total);
}

template <int S>
__global__ void k_pack_cols(const double* __restrict__ B, int64_t ldb, int n, double* __restrict__ out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double v[S];
#pragma unroll
    for (int c = 0; c < S; ++c) v[c] = B[(size_t)c * ldb + r];
    store_row<double, S>(out + (size_t)r * S, v);
  }
}

template <int S>
__global__ void k_unpack_cols(const double* __restrict__ in, int n, double* __restrict__ X, int64_t ldx) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double v[S];
    load_row<double, S>(in + (size_t)r * S, v);
#pragma unroll
    for (int c = 0; c < S; ++c) X[(size_t)c * ldx + r] = v[c];
  }
}

}  // namespace lyap

extern "C" lyap_status lyap_inner_solve(const lyap_op* A, const double* B, int64_t ldb, double* X, int64_t ldx,
                                        int32_t s, const lyap_opts* opts, int64_t* iters, double* relres) {
  using namespace lyap;
  clear_error();
  lyap_opts o;
  if (opts) o = *opts;
  else lyap_opts_default(&o);
  try {
    validate_op(A);
    LYAP_REQUIRE(B != nullptr && X != nullptr, LYAP_E_ARG, "B or X is NULL");
    LYAP_REQUIRE(s == 1 || s == 2 || s == 4, LYAP_E_UNSUPPORTED, "s=%d: the inner solver takes 1, 2 or 4 columns", s);
    LYAP_REQUIRE(ldb >= A->n && ldx >= A->n, LYAP_E_ARG, "leading dimension below n");
    LYAP_REQUIRE(o.inner_pc != LYAP_PC_LEARNED, LYAP_E_UNSUPPORTED,
                 "the learned preconditioner is trained inside an extended Krylov solve (lyap_solve)");
    hipStream_t st = (hipStream_t)o.stream;
    const int n = (int)A->n;
    OpHolder<double> op;
    make_op_f64(A, op, st);
    InnerCG cg(op.dev, n, s, o.inner_pc, o.inner_tol, o.inner_max_iter, st);
    DevBuf Bi((size_t)n * s * sizeof(double)), Xi((size_t)n * s * sizeof(double));
    const int g = grid_for(n, 1, 1024);
    auto pack = [&]() {
      switch (s) {
        case 1: hipLaunchKernelGGL((k_pack_cols<1>), dim3(g), dim3(kBlock), 0, st, B, ldb, n, Bi.as<double>()); break;
        case 2: hipLaunchKernelGGL((k_pack_cols<2>), dim3(g), dim3(kBlock), 0, st, B, ldb, n, Bi.as<double>()); break;
        default: hipLaunchKernelGGL((k_pack_cols<4>), dim3(g), dim3(kBlock), 0, st, B, ldb, n, Bi.as<double>()); break;
      }
      LYAP_LAUNCHED("k_pack_cols");
    };
    auto unpack = [&]() {
      switch (s) {
        case 1: hipLaunchKernelGGL((k_unpack_cols<1>), dim3(g), dim3(kBlock), 0, st, Xi.as<double>(), n, X, ldx); break;
        case 2: hipLaunchKernelGGL((k_unpack_cols<2>), dim3(g), dim3(kBlock), 0, st, Xi.as<double>(), n, X, ldx); break;
        default: hipLaunchKernelGGL((k_unpack_cols<4>), dim3(g), dim3(kBlock), 0, st, Xi.as<double>(), n, X, ldx); break;
      }
      LYAP_LAUNCHED("k_unpack_cols");
    };
    pack();
    lyap_status status = LYAP_OK;
    try {
      cg.solve(Bi.as<double>(), Xi.as<double>());
    } catch (const Error& e) {
      if (e.st != LYAP_E_INNER) throw;
      status = LYAP_E_INNER;
    }
    unpack();
    LYAP_HIP(hipStreamSynchronize(st));
    if (iters) *iters = cg.stats().iters;
    if (relres) *relres = cg.stats().worst_relres;
    return status;
  } catch (const Error& e) {
    return e.st;
  }
}
