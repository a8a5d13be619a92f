// lyap_solve_gen: A X E + E X A + C C^T = 0 with A symmetric negative
// definite and E symmetric positive definite, treated as the standard
// equation of A~ = L^{-1} A L^{-T} and C~ = L^{-1} C (E = L L^T; Section 6,
// Example 3) without forming L: block Lanczos for E^{-1} A in the E inner
// product.  With W_j = L^{-T} V~_j (W^T E W = I) the recurrence reads
//   E^{-1} A W_j = W_{j+1} tau_{j+1,j} + W_j alpha_j + W_{j-1} tau_{j,j-1}^T,
// its coefficients are those of the standard Lanczos run on A~ (so T_m, gamma,
// Proposition 1 and the truncation are unchanged), and X = W Y W^T, Z = W_m M.
//
// One step: Q = A W_j; X = (-E)^{-1} Q by the FP64 inner CG (so U = -X =
// E^{-1} A W_j); G = (-E) X = E U by a product with E; two sweeps of block MGS
// against W_{j-1}, W_j in the E inner product (alpha = P_i^T U with P_i = E W_i
// kept alongside W_i, U -= W_i alpha, G -= P_i alpha, so G = E U throughout);
// E-norm Cholesky QR twice (Gram U^T G).  Every reduction is deterministic,
// so a second pass that repeats the steps regenerates the blocks bit for bit.
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "check.hpp"
#include "pcg.hpp"
#include "small.hpp"
#include "solver.hpp"

namespace lyap {

constexpr int kGenNT = 256;
// per-step log: alpha_1..alpha_4, R1, R2, tau (S x S row-major each)
constexpr size_t gen_log_stride(int S) { return (size_t)7 * S * S; }

__global__ void k_gen_pack(const double* C, int64_t ldc, int n, int S, double* B) {
  const int64_t tot = (int64_t)n * S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / S), c = (int)(e - (int64_t)r * S);
    B[e] = C[(size_t)c * ldc + r];
  }
}

// -(E) from E: the same operator with every coefficient negated.
__global__ void k_gen_negate(const double* x, int64_t len, double* y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = -x[e];
}

// U = -X, G = (-E) X = E U; partial Gram Pa^T U (mode 0) or U^T G (mode 1).
template <int S>
__global__ __launch_bounds__(kGenNT) void k_gen_first(OpDev<double> negE, const double* __restrict__ X,
                                                      double* __restrict__ U, double* __restrict__ G,
                                                      const double* __restrict__ Pa, int mode, double* part, int n) {
  __shared__ double red[pow2_at_least(S * S) * (kGenNT / 64)];
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, n, lo, hi);
  for (int r = lo + threadIdx.x; r < hi; r += kGenNT) {
    double g[S], x[S], u[S];
    op_row<double, S>(negE, X, r, g);
    load_row<double, S>(X + (size_t)r * S, x);
#pragma unroll
    for (int c = 0; c < S; ++c) u[c] = -x[c];
    store_row<double, S>(G + (size_t)r * S, g);
    store_row<double, S>(U + (size_t)r * S, u);
    if (mode == 0) {
      double pa[S];
      load_row<double, S>(Pa + (size_t)r * S, pa);
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) acc[a * S + b] = fma(pa[a], u[b], acc[a * S + b]);
    } else {
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) acc[a * S + b] = fma(u[a], g[b], acc[a * S + b]);
    }
  }
  write_partial<S * S, kGenNT>(acc, red, part);
}

// alpha = sum of the previous partials (logged by workgroup 0); U -= Wa alpha,
// G -= Pa alpha; partial Gram Pb^T U (mode 0) or U^T G (mode 1).
template <int S>
__global__ __launch_bounds__(kGenNT) void k_gen_upd(double* __restrict__ U, double* __restrict__ G,
                                                    const double* __restrict__ Wa, const double* __restrict__ Pa,
                                                    const double* __restrict__ part_in, int nparts,
                                                    const double* __restrict__ Pb, int mode, double* part_out,
                                                    double* alpha_log, int n) {
  __shared__ double red[pow2_at_least(S * S) * (kGenNT / 64)];
  __shared__ double al[S * S];
  reduce_partials<S * S, kGenNT>(part_in, nparts, red);
  if (threadIdx.x < S * S) {
    al[threadIdx.x] = red[threadIdx.x];
    if (blockIdx.x == 0) alpha_log[threadIdx.x] = red[threadIdx.x];
  }
  __syncthreads();
  double alpha[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) alpha[i] = al[i];
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, n, lo, hi);
  for (int r = lo + threadIdx.x; r < hi; r += kGenNT) {
    double u[S], g[S], wa[S], pa[S];
    load_row<double, S>(U + (size_t)r * S, u);
    load_row<double, S>(G + (size_t)r * S, g);
    load_row<double, S>(Wa + (size_t)r * S, wa);
    load_row<double, S>(Pa + (size_t)r * S, pa);
#pragma unroll
    for (int b = 0; b < S; ++b)
#pragma unroll
      for (int a = 0; a < S; ++a) {
        u[b] = fma(-wa[a], alpha[a * S + b], u[b]);
        g[b] = fma(-pa[a], alpha[a * S + b], g[b]);
      }
    store_row<double, S>(U + (size_t)r * S, u);
    store_row<double, S>(G + (size_t)r * S, g);
    if (mode == 0) {
      double pb[S];
      load_row<double, S>(Pb + (size_t)r * S, pb);
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) acc[a * S + b] = fma(pb[a], u[b], acc[a * S + b]);
    } else {
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) acc[a * S + b] = fma(u[a], g[b], acc[a * S + b]);
    }
  }
  write_partial<S * S, kGenNT>(acc, red, part_out);
}

// E-norm Cholesky QR: R = chol(sym(U^T G)) from the previous partials,
// U R^{-1}, G R^{-1}.  final == 0: written back to U, G with the partial Gram
// of the result and R logged as R1; final == 1: written to Wout, Pout, R logged
// as R2, tau = R2 R1, and (band != nullptr) the block column j of T_m: the
// diagonal block sym(alpha_2 + alpha_4) and tau below it.
template <int S>
__global__ __launch_bounds__(kGenNT) void k_gen_chol(double* __restrict__ U, double* __restrict__ G,
                                                     const double* __restrict__ part_in, int nparts, int final,
                                                     double* __restrict__ Wout, double* __restrict__ Pout,
                                                     double* part_out, double* log, double* band, int j, int* flags,
                                                     int n) {
  __shared__ double red[pow2_at_least(S * S) * (kGenNT / 64)];
  __shared__ double ri_s[S * S];
  reduce_partials<S * S, kGenNT>(part_in, nparts, red);
  if (threadIdx.x == 0) {
    double Gm[S * S], R[S * S], Ri[S * S];
    bool finite = true;
    for (int a = 0; a < S; ++a)
      for (int b = 0; b < S; ++b) {
        Gm[a * S + b] = 0.5 * (red[a * S + b] + red[b * S + a]);
        finite = finite && isfinite(Gm[a * S + b]);
      }
    const double ratio = chol_upper<S>(Gm, R);
    inv_upper<S>(R, Ri);
    for (int i = 0; i < S * S; ++i) ri_s[i] = Ri[i];
    if (blockIdx.x == 0) {
      double* R1 = log + 4 * S * S;
      double* R2 = log + 5 * S * S;
      double* tau = log + 6 * S * S;
      if (!final) {
        for (int i = 0; i < S * S; ++i) R1[i] = R[i];
        if (flags && j >= 0) {
          if (ratio < kBreakdownRatio && flags[0] == 0) flags[0] = j + 1;
          if (!finite && flags[1] == 0) flags[1] = j + 1;
        }
      } else {
        for (int i = 0; i < S * S; ++i) R2[i] = R[i];
        mul_upper<S>(R, R1, tau);
        if (band) {
          const double* a2 = log + 1 * S * S;
          const double* a4 = log + 3 * S * S;
          constexpr int LD = S + 1;
          for (int b = 0; b < S; ++b) {
            for (int a = b; a < S; ++a) {
              const double d = 0.5 * ((a2[a * S + b] + a4[a * S + b]) + (a2[b * S + a] + a4[b * S + a]));
              band[(size_t)(j * S + b) * LD + (a - b)] = d;
            }
            for (int a = 0; a <= b; ++a) band[(size_t)(j * S + b) * LD + S + a - b] = tau[a * S + b];
          }
        }
        if (flags && j >= 0 && !finite && flags[1] == 0) flags[1] = j + 1;
      }
    }
  }
  __syncthreads();
  double Ri[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) Ri[i] = ri_s[i];
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  double* Uo = final ? Wout : U;
  double* Go = final ? Pout : G;
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, n, lo, hi);
  for (int r = lo + threadIdx.x; r < hi; r += kGenNT) {
    double u[S], g[S], uo[S], go[S];
    load_row<double, S>(U + (size_t)r * S, u);
    load_row<double, S>(G + (size_t)r * S, g);
#pragma unroll
    for (int b = 0; b < S; ++b) {
      double x = 0.0, y = 0.0;
#pragma unroll
      for (int a = 0; a <= b; ++a) {
        x = fma(u[a], Ri[a * S + b], x);
        y = fma(g[a], Ri[a * S + b], y);
      }
      uo[b] = x;
      go[b] = y;
    }
    store_row<double, S>(Uo + (size_t)r * S, uo);
    store_row<double, S>(Go + (size_t)r * S, go);
    if (!final) {
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) acc[a * S + b] = fma(uo[a], go[b], acc[a * S + b]);
    }
  }
  if (!final) write_partial<S * S, kGenNT>(acc, red, part_out);
}

namespace {

// The device state of one run and its step (used by both passes).
struct GenRun {
  int n, S, grid;
  OpHolder<double> opA, opNegE;
  DevBuf negE_diag, negE_tx, negE_ty, negE_tz, negE_val;
  std::unique_ptr<InnerCG> cg;
  DevBuf Q, X, U, G, zero, partA, partB;
  hipStream_t st;

  template <int S>
  void step_t(const double* Wprev, const double* Wcur, const double* Pprev, const double* Pcur, double* Wnext,
              double* Pnext, double* log, double* band, int j, int* flags) {
    const int g = grid;
    double* pa = partA.as<double>();
    double* pb = partB.as<double>();
    double* u = U.as<double>();
    double* gg = G.as<double>();
    hipLaunchKernelGGL((k_gen_first<S>), dim3(g), dim3(kGenNT), 0, st, opNegE.dev, X.as<double>(), u, gg, Pprev, 0,
                       pa, n);
    // two sweeps against W_{j-1}, W_j (alpha_1..alpha_4)
    hipLaunchKernelGGL((k_gen_upd<S>), dim3(g), dim3(kGenNT), 0, st, u, gg, Wprev, Pprev, pa, g, Pcur, 0, pb,
                       log + 0 * S * S, n);
    hipLaunchKernelGGL((k_gen_upd<S>), dim3(g), dim3(kGenNT), 0, st, u, gg, Wcur, Pcur, pb, g, Pprev, 0, pa,
                       log + 1 * S * S, n);
    hipLaunchKernelGGL((k_gen_upd<S>), dim3(g), dim3(kGenNT), 0, st, u, gg, Wprev, Pprev, pa, g, Pcur, 0, pb,
                       log + 2 * S * S, n);
    hipLaunchKernelGGL((k_gen_upd<S>), dim3(g), dim3(kGenNT), 0, st, u, gg, Wcur, Pcur, pb, g, Pcur, 1, pa,
                       log + 3 * S * S, n);
    hipLaunchKernelGGL((k_gen_chol<S>), dim3(g), dim3(kGenNT), 0, st, u, gg, pa, g, 0, nullptr, nullptr, pb, log,
                       nullptr, j, flags, n);
    hipLaunchKernelGGL((k_gen_chol<S>), dim3(g), dim3(kGenNT), 0, st, u, gg, pb, g, 1, Wnext, Pnext, pa, log, band,
                       j, flags, n);
    LYAP_LAUNCHED("gen step");
  }

  template <int S>
  void start_t(double* W1, double* P1, double* glog) {
    const int g = grid;
    double* pa = partA.as<double>();
    double* pb = partB.as<double>();
    hipLaunchKernelGGL((k_gen_first<S>), dim3(g), dim3(kGenNT), 0, st, opNegE.dev, X.as<double>(), U.as<double>(),
                       G.as<double>(), zero.as<double>(), 1, pa, n);
    hipLaunchKernelGGL((k_gen_chol<S>), dim3(g), dim3(kGenNT), 0, st, U.as<double>(), G.as<double>(), pa, g, 0,
                       nullptr, nullptr, pb, glog, nullptr, -1, nullptr, n);
    hipLaunchKernelGGL((k_gen_chol<S>), dim3(g), dim3(kGenNT), 0, st, U.as<double>(), G.as<double>(), pb, g, 1, W1,
                       P1, pa, glog, nullptr, -1, nullptr, n);
    LYAP_LAUNCHED("gen start");
  }

  // W_1, P_1 and gamma (glog + 6 S^2) from C: X = (-E)^{-1} C, U = -X = E^{-1} C.
  void start(const double* C, int64_t ldc, double* W1, double* P1, double* glog) {
    hipLaunchKernelGGL(k_gen_pack, dim3(grid_for((int64_t)n * S, 1, 2048)), dim3(kBlock), 0, st, C, ldc, n, S,
                       Q.as<double>());
    LYAP_LAUNCHED("k_gen_pack");
    cg->solve(Q.as<double>(), X.as<double>());
    if (S == 1) start_t<1>(W1, P1, glog);
    else if (S == 2) start_t<2>(W1, P1, glog);
    else start_t<4>(W1, P1, glog);
  }

  // One block Lanczos step j (0-based): W_{j+1}, P_{j+1}, the log and T_m's
  // block column j.
  void step(const double* Wprev, const double* Wcur, const double* Pprev, const double* Pcur, double* Wnext,
            double* Pnext, double* log, double* band, int j, int* flags) {
    launch_apply<double>(opA.dev, S, Wcur, Q.as<double>(), xcd_grid(grid_for(n, 2, 4096)), st);
    cg->solve(Q.as<double>(), X.as<double>());
    if (S == 1) step_t<1>(Wprev, Wcur, Pprev, Pcur, Wnext, Pnext, log, band, j, flags);
    else if (S == 2) step_t<2>(Wprev, Wcur, Pprev, Pcur, Wnext, Pnext, log, band, j, flags);
    else step_t<4>(Wprev, Wcur, Pprev, Pcur, Wnext, Pnext, log, band, j, flags);
  }
};

// A lyap_op for -E: scalar coefficients negated, coefficient arrays copied
// negated into the run's buffers.
lyap_op negated_op(const lyap_op* E, GenRun& run, hipStream_t st) {
  lyap_op ne = *E;
  ne.shift = -E->shift;
  auto neg = [&](const double* src, int64_t len, DevBuf& dst) -> const double* {
    dst.alloc((size_t)std::max<int64_t>(1, len) * sizeof(double));
    hipLaunchKernelGGL(k_gen_negate, dim3(grid_for(len, 1, 2048)), dim3(kBlock), 0, st, src, len, dst.as<double>());
    LYAP_LAUNCHED("k_gen_negate");
    return dst.as<double>();
  };
  if (E->kind == LYAP_OP_STENCIL5) {
    ne.cc = -E->cc;
    ne.co = -E->co;
  } else if (E->kind == LYAP_OP_STENCIL7) {
    ne.diag = neg(E->diag, E->n, run.negE_diag);
    ne.tx = neg(E->tx, E->n, run.negE_tx);
    ne.ty = neg(E->ty, E->n, run.negE_ty);
    if (E->nz > 1) ne.tz = neg(E->tz, E->n, run.negE_tz);
  } else {
    ne.val = neg(E->val, E->nnz, run.negE_val);
  }
  return ne;
}

lyap_status gen_impl(const lyap_op* A, const lyap_op* E, const double* C, int S, int64_t ldc, const lyap_opts& o,
                     lyap_result* out) {
  const auto t_entry = Clock::now();
  hipStream_t st = (hipStream_t)o.stream;
  const int n = (int)A->n;
  out->n = n;
  out->s = S;
  out->ell = S;
  const int maxit = o.max_iter;
  GenRun run;
  run.n = n;
  run.S = S;
  run.st = st;
  run.grid = xcd_grid(stream_grid(n));
  make_op_f64(A, run.opA, st);
  const lyap_op ne = negated_op(E, run, st);
  make_op_f64(&ne, run.opNegE, st);
  try {
    run.cg.reset(new InnerCG(run.opNegE.dev, n, S, o.inner_pc, o.inner_tol, o.inner_max_iter, st));
  } catch (const Error& e) {
    if (e.st == LYAP_E_INDEFINITE) set_error("E has a diagonal entry <= 0: not positive definite");
    throw;
  }
  const size_t blk = (size_t)n * S * sizeof(double);
  run.Q.alloc(blk);
  run.X.alloc(blk);
  run.U.alloc(blk);
  run.G.alloc(blk);
  run.zero.alloc(blk);
  LYAP_HIP(hipMemsetAsync(run.zero.p, 0, blk, st));
  run.partA.alloc((size_t)run.grid * S * S * sizeof(double));
  run.partB.alloc((size_t)run.grid * S * S * sizeof(double));
  const size_t LS = gen_log_stride(S);
  DevBuf logb((size_t)(maxit + 1) * LS * sizeof(double)), glog(LS * sizeof(double));
  DevBuf band((size_t)(S + 1) * (size_t)(maxit + 1) * S * sizeof(double));
  DevBuf flags(64);
  LYAP_HIP(hipMemsetAsync(flags.p, 0, 64, st));
  LYAP_HIP(hipMemsetAsync(band.p, 0, band.bytes, st));

  const bool two_pass = o.two_pass != 0;
  // basis: every block kept (stored basis) or three rotating W slots; three P slots
  std::vector<DevBuf> Wst;
  DevBuf Pb[3];
  for (auto& p : Pb) p.alloc(blk);
  auto wslot = [&](int i) -> double* {
    if (two_pass) return Wst[i % 3].as<double>();
    while ((int)Wst.size() <= i) Wst.emplace_back(blk);
    return Wst[i].as<double>();
  };
  if (two_pass)
    for (int i = 0; i < 3; ++i) Wst.emplace_back(blk);

  run.start(C, ldc, wslot(0), Pb[0].as<double>(), glog.as<double>());
  std::vector<double> gam(S * S);
  LYAP_HIP(hipMemcpyAsync(gam.data(), glog.as<double>() + 6 * S * S, S * S * sizeof(double), hipMemcpyDeviceToHost,
                          st));
  LYAP_HIP(hipStreamSynchronize(st));
  double beta2 = 0.0, gmax = 0.0, gmin = INFINITY;
  for (double x : gam) beta2 += x * x;
  for (int a = 0; a < S; ++a) {
    gmax = std::max(gmax, std::fabs(gam[a * S + a]));
    gmin = std::min(gmin, std::fabs(gam[a * S + a]));
  }
  LYAP_REQUIRE(std::isfinite(beta2) && beta2 > 0.0, LYAP_E_NUMERIC, "E^{-1} C is zero or not finite");
  LYAP_REQUIRE(gmin > 1e-7 * gmax, LYAP_E_BREAKDOWN, "C is numerically rank deficient in the E^{-1} inner product");
  out->beta = std::sqrt(beta2);
  const double* gamma_dev = glog.as<double>() + 6 * S * S;

  // The residual check runs on a stream of its own while the next steps
  // proceed: a check at mm reads only the band's first mm S columns, gamma and
  // the log entry of step mm - 1, which later steps never write.  It always
  // runs at the scheduled m, so the results do not depend on timing; a step
  // that fails while a check is pending first lets that check decide (the
  // steps past the converging check are not used).
  struct CheckStream {
    hipStream_t s = nullptr;
    hipEvent_t ev_step = nullptr, ev_chk = nullptr;
    ~CheckStream() {
      if (s) (void)hipStreamSynchronize(s);
      if (ev_step) (void)hipEventDestroy(ev_step);
      if (ev_chk) (void)hipEventDestroy(ev_chk);
      if (s) (void)hipStreamDestroy(s);
    }
  } cstr;
  LYAP_HIP(hipStreamCreateWithFlags(&cstr.s, hipStreamNonBlocking));
  LYAP_HIP(hipEventCreateWithFlags(&cstr.ev_step, hipEventDisableTiming));
  LYAP_HIP(hipEventCreateWithFlags(&cstr.ev_chk, hipEventDisableTiming));
  Checker ck(S, S, cstr.s);
  DevBuf chk(sizeof(CheckOut));
  HostBuf hchk(sizeof(CheckOut) + 2 * sizeof(int) + 2 * sizeof(double));
  CheckSchedule sched{o.check_every, maxit};
  std::vector<int> hm;
  std::vector<double> hr;
  int next_check = sched.first(), m = 0;
  double check_ms = 0.0, t_to_tol = 0.0, last_res = INFINITY, lam_abs = 0.0;
  lyap_status status = LYAP_NOT_CONVERGED;
  CheckOut* hc = hchk.as<CheckOut>();
  int* hf = reinterpret_cast<int*>(hchk.as<char>() + sizeof(CheckOut));
  double* hl = reinterpret_cast<double*>(hchk.as<char>() + sizeof(CheckOut) + 2 * sizeof(int));
  auto step_at = [&](int j) {
    const double* Wp = j > 0 ? wslot(j - 1) : run.zero.as<double>();
    const double* Pp = j > 0 ? Pb[(j - 1) % 3].as<double>() : run.zero.as<double>();
    run.step(Wp, wslot(j), Pp, Pb[j % 3].as<double>(), wslot(j + 1), Pb[(j + 1) % 3].as<double>(),
             logb.as<double>() + (size_t)j * LS, band.as<double>(), j, flags.as<int>());
  };
  bool pending = false;
  int pending_mm = 0, last_launched = 0;
  auto launch_check = [&](int mm) {
    const int k = mm * S;
    LYAP_HIP(hipEventRecord(cstr.ev_step, st));
    LYAP_HIP(hipStreamWaitEvent(cstr.s, cstr.ev_step, 0));
    ck.run(band.as<double>(), k, gamma_dev, logb.as<double>() + (size_t)(mm - 1) * LS + 6 * S * S, chk.as<CheckOut>());
    LYAP_HIP(hipMemcpyAsync(hc, chk.p, sizeof(CheckOut), hipMemcpyDeviceToHost, cstr.s));
    LYAP_HIP(hipMemcpyAsync(hf, flags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, cstr.s));
    LYAP_HIP(hipMemcpyAsync(&hl[0], ck.lam(), sizeof(double), hipMemcpyDeviceToHost, cstr.s));
    LYAP_HIP(hipMemcpyAsync(&hl[1], ck.lam() + k - 1, sizeof(double), hipMemcpyDeviceToHost, cstr.s));
    LYAP_HIP(hipEventRecord(cstr.ev_chk, cstr.s));
    pending = true;
    pending_mm = mm;
    last_launched = mm;
  };
  // waits for the pending check and reads it; returns true when the iteration stops
  auto finish_check = [&]() -> bool {
    const auto t0 = Clock::now();
    LYAP_HIP(hipEventSynchronize(cstr.ev_chk));
    check_ms += ms_since(t0);
    pending = false;
    const int mm = pending_mm;
    const int k = mm * S;
    out->n_checks++;
    // flags of steps after mm (run beside the check) do not concern this check
    const int fb = hf[0] > 0 && hf[0] <= mm ? hf[0] : 0, fn = hf[1] > 0 && hf[1] <= mm ? hf[1] : 0;
    LYAP_REQUIRE(!(fn > 0 && (fb == 0 || fn <= fb)), LYAP_E_NUMERIC,
                 "non-finite values in the Lanczos recurrence at step %d", fn);
    LYAP_REQUIRE(std::isfinite(hc->res), LYAP_E_NUMERIC, "residual is not finite at m=%d", mm);
    const double rel = hc->res / beta2;
    hm.push_back(mm);
    hr.push_back(rel);
    last_res = rel;
    lam_abs = std::max(std::fabs(hl[0]), std::fabs(hl[1]));
    if (o.verbose) std::fprintf(stderr, "[gen] m=%d k=%d res=%.3e\n", mm, k, rel);
    LYAP_REQUIRE(hc->lam_max < 0.0, LYAP_E_INDEFINITE, "Ritz value %.3e >= 0 at m=%d: A is not negative definite",
                 hc->lam_max, mm);
    m = mm;
    if (rel <= o.tol) {
      status = LYAP_OK;
      t_to_tol = ms_since(t_entry);
      return true;
    }
    if (fb > 0) {
      status = LYAP_E_BREAKDOWN;
      set_error("block Lanczos breakdown at m=%d with residual %.3e above tol", fb, rel);
      return true;
    }
    if (mm >= maxit) return true;
    next_check = sched.next(mm, rel, o.tol);
    return false;
  };
  const auto t_pass1 = Clock::now();
  int steps = 0;  // steps enqueued
  bool stop = false;
  // inner-solve counts after each step: the steps run beside the converging
  // check are not counted, so that the reported counts do not depend on timing
  std::vector<std::pair<int64_t, int>> cg_at{{run.cg->stats().iters, run.cg->stats().solves}};
  while (!stop) {
    if (pending && (steps >= maxit || hipEventQuery(cstr.ev_chk) == hipSuccess)) {
      stop = finish_check();
      continue;
    }
    if (!pending && next_check > last_launched && steps >= std::min(next_check, maxit)) {
      launch_check(std::min(next_check, maxit));
      continue;
    }
    if (steps >= maxit) break;  // (not reached: the check at maxit ends the iteration)
    if (!pending) {
      step_at(steps++);
      cg_at.emplace_back(run.cg->stats().iters, run.cg->stats().solves);
      continue;
    }
    try {
      step_at(steps);
      ++steps;
      cg_at.emplace_back(run.cg->stats().iters, run.cg->stats().solves);
    } catch (const Error&) {
      // the pending check decides first; the step's error stands only if it does not stop
      if (finish_check()) break;
      throw;
    }
  }
  const double pass1_ms = ms_since(t_pass1) - check_ms;
  const std::pair<int64_t, int> past_m{run.cg->stats().iters - cg_at[std::min<size_t>(m, cg_at.size() - 1)].first,
                                      run.cg->stats().solves - cg_at[std::min<size_t>(m, cg_at.size() - 1)].second};
  store_history(out, hm, hr);
  out->m = m;
  out->res = last_res;

  // ---- finalisation (as lyap_solve)
  const auto t_fin = Clock::now();
  std::vector<double> tau_h(S * S);
  LYAP_HIP(hipMemcpyAsync(tau_h.data(), logb.as<double>() + (size_t)(m - 1) * LS + 6 * S * S, S * S * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  double tf = 0.0;
  for (double x : tau_h) tf += x * x;
  const double nu = lam_abs + std::sqrt(tf);
  double eps = o.trunc_eps;
  if (!(eps >= 0.0)) eps = std::min(1e-12, 0.05 * o.tol / nu) * beta2;
  out->trunc_eps = eps;
  DevBuf M;
  const int t = finalise_factor(ck, band.as<double>(), gamma_dev, eps, M, st);
  out->t = t;
  const double fin_ms = ms_since(t_fin);

  // ---- Z = W_m M: stored blocks, or a second pass that repeats the steps
  const auto t_p2 = Clock::now();
  bool own = false;
  out->Z = alloc_output(o, (size_t)n * std::max(t, 1) * sizeof(double), &own);
  out->owns_Z = own ? 1 : 0;
  if (t > 0) {
    LYAP_HIP(hipMemsetAsync(out->Z, 0, (size_t)n * t * sizeof(double), st));
    const int QB = zflush_max_blocks(S);
    if (!two_pass) {
      std::vector<const void*> ptrs;
      for (int i = 0; i < m; ++i) ptrs.push_back(Wst[i].p);
      launch_zflush<double>(ptrs.data(), m, n, S, M.as<double>(), t, out->Z, n, 0, st);
    } else {
      // ring of QB + 3 W blocks: a block is flushed before its slot comes round again
      const int R = QB + 3;
      std::vector<DevBuf> ring;
      for (int i = 0; i < R; ++i) ring.emplace_back(blk);
      DevBuf P2[3];
      for (auto& p : P2) p.alloc(blk);
      DevBuf log2((size_t)m * LS * sizeof(double)), glog2(LS * sizeof(double));
      run.start(C, ldc, ring[0].as<double>(), P2[0].as<double>(), glog2.as<double>());
      std::vector<const void*> pend;
      int first = 0;
      for (int i = 0; i < m; ++i) {
        if (i + 1 < m) {
          const double* Wp = i > 0 ? ring[(i - 1) % R].as<double>() : run.zero.as<double>();
          const double* Pp = i > 0 ? P2[(i - 1) % 3].as<double>() : run.zero.as<double>();
          run.step(Wp, ring[i % R].as<double>(), Pp, P2[i % 3].as<double>(), ring[(i + 1) % R].as<double>(),
                   P2[(i + 1) % 3].as<double>(), log2.as<double>() + (size_t)i * LS, nullptr, i, nullptr);
        }
        if (pend.empty()) first = i;
        pend.push_back(ring[i % R].p);
        if ((int)pend.size() == QB || i == m - 1) {
          launch_zflush<double>(pend.data(), (int)pend.size(), n, S, M.as<double>() + (size_t)first * S * t, t,
                                out->Z, n, 0, st);
          pend.clear();
        }
      }
      LYAP_HIP(hipStreamSynchronize(st));  // the ring is released on return
    }
  }
  LYAP_HIP(hipStreamSynchronize(st));
  const double p2_ms = ms_since(t_p2);

  if (o.want_T) {
    const int k = m * S;
    out->T_band = (double*)std::malloc((size_t)(S + 1) * k * sizeof(double));
    LYAP_HIP(hipMemcpy(out->T_band, band.p, (size_t)(S + 1) * k * sizeof(double), hipMemcpyDeviceToHost));
    for (int c = 0; c < k; ++c)
      for (int d = 0; d <= S; ++d)
        if (c + d >= k) out->T_band[(size_t)c * (S + 1) + d] = 0.0;
    out->gamma = (double*)std::malloc(S * S * sizeof(double));
    out->tau = (double*)std::malloc(S * S * sizeof(double));
    rowmajor_to_colmajor(gam.data(), S, S, out->gamma);
    rowmajor_to_colmajor(tau_h.data(), S, S, out->tau);
  }
  const CgStats& cs = run.cg->stats();
  out->inner_iters = cs.iters - past_m.first;
  out->n_inner = cs.solves - past_m.second;
  out->times_ms[LYAP_T_PASS1] = pass1_ms;
  out->times_ms[LYAP_T_CHECKS] = check_ms;
  out->times_ms[LYAP_T_FINAL] = fin_ms;
  out->times_ms[LYAP_T_PASS2] = p2_ms;
  out->times_ms[LYAP_T_INNER] = cs.ms;
  out->times_ms[LYAP_T_TOTAL] = ms_since(t_entry);
  out->times_ms[LYAP_T_TO_TOL] = t_to_tol;
  out->status = status;
  return status;
}

}  // namespace
}  // namespace lyap

extern "C" lyap_status lyap_solve_gen(const lyap_op* A, const lyap_op* E, const double* C, int32_t s, int64_t ldc,
                                      const lyap_opts* opts, lyap_result* out) {
  using namespace lyap;
  clear_error();
  if (!out) {
    set_error("out is NULL");
    return LYAP_E_ARG;
  }
  std::memset(out, 0, sizeof(*out));
  lyap_opts o;
  if (opts) o = *opts;
  else lyap_opts_default(&o);
  try {
    validate_op(A);
    validate_op(E);
    LYAP_REQUIRE(E->n == A->n, LYAP_E_ARG, "E has %lld rows, A has %lld", (long long)E->n, (long long)A->n);
    LYAP_REQUIRE(C != nullptr, LYAP_E_ARG, "C is NULL");
    LYAP_REQUIRE(s == 1 || s == 2 || s == 4, LYAP_E_ARG, "s=%d: the generalized solver takes s = 1, 2 or 4", s);
    LYAP_REQUIRE(ldc >= A->n && s <= A->n, LYAP_E_ARG, "ldc below n or s > n");
    LYAP_REQUIRE(o.tol > 0.0 && o.tol < 1.0, LYAP_E_ARG, "tol=%g must be in (0,1)", o.tol);
    LYAP_REQUIRE(o.max_iter >= 1 && (int64_t)o.max_iter * s <= (int64_t)1 << 20, LYAP_E_ARG,
                 "max_iter=%d out of range", o.max_iter);
    LYAP_REQUIRE(o.check_every >= 0, LYAP_E_ARG, "check_every must be >= 0");
    LYAP_REQUIRE(o.method == LYAP_METHOD_STD, LYAP_E_UNSUPPORTED,
                 "lyap_solve_gen builds a standard Krylov space (method must be LYAP_METHOD_STD)");
    LYAP_REQUIRE(o.storage == LYAP_STORE_F64, LYAP_E_UNSUPPORTED, "lyap_solve_gen stores the basis in FP64 only");
    LYAP_REQUIRE(o.inner_pc == LYAP_PC_NONE || o.inner_pc == LYAP_PC_JACOBI, LYAP_E_UNSUPPORTED,
                 "lyap_solve_gen solves with E by CG with inner_pc NONE or JACOBI");
    lyap_status st = gen_impl(A, E, C, s, ldc, o, out);
    out->status = st;
    return st;
  } catch (const Error& e) {
    out->status = e.st;
    return e.st;
  }
}
