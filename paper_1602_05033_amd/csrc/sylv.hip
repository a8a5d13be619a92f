// sylv_solve: A X + X B + C1 C2^T = 0 with A, B symmetric negative definite,
// by two standard block Krylov spaces K_m(A, C1) and K_m(B, C2) of the same
// dimension (Section 5.1), driven in lockstep on one stream.
//
// Residual (eq. (resSylv) evaluated without Y_m, Algorithm 4): with
// T_m = Q Lambda Q^T, J_m = P Upsilon P^T, g1 = (E_1^T Q)^T gamma_1,
// g2 = (E_1^T P)^T gamma_2, S = g1 g2^T, F = (E_m^T Q)^T tau^T and
// G = (E_m^T P)^T iota^T, the solution of the reduced equation is
// Y = Q Y~ P^T with Y~_ij = -S_ij / (lambda_i + upsilon_j), and
//   ||R||_F^2 = sum_i || e_i^T S (lambda_i I + Upsilon)^{-1} G ||^2
//             + sum_j || e_j^T S^T (upsilon_j I + Lambda)^{-1} F ||^2.
// (Algorithm 4 as printed pairs the shifts the other way round; this form is
// the one that equals eq. (resSylv).)
//
// Finalisation: Y~ (k x k, nonsymmetric) is approximated by a cross / skeleton
// factorisation Y~ ~= Y~(:, J) Y~(I, J)^{-1} Y~(I, :) built by Gaussian
// elimination with complete pivoting, stopped when the Frobenius norm of the
// remaining Schur complement -- exactly the approximation error -- is at most
// eps (the error bound of the paper's truncated SVD, at a possibly larger
// rank).  Q Y~(:, j) and P Y~(i, :)^T come from banded shifted solves, so
// neither Q nor P is formed:
//   Q Y~(:, j)   = -(T_m + upsilon_j I)^{-1} E_1 gamma_1 g2_j,
//   P Y~(i, :)^T = -(J_m + lambda_i I)^{-1} E_1 gamma_2 g1_i.
// With Y~(I, J) = L U (unit lower L, the pivots on U's diagonal):
//   M1 = [Q Y~(:, J)] U^{-1},  M2 = [P Y~(I, :)^T] L^{-T},  Z1 = V_m M1,
//   Z2 = U_m M2 (second pass on each side), Z1 Z2^T ~= X.
#include <algorithm>
#include <cmath>
#include <memory>
#include <type_traits>
#include <vector>

#include "aca.hpp"
#include "check.hpp"
#include "side.hpp"
#include "solver.hpp"
#include "sylv.hpp"

namespace lyap {

constexpr int kSylMaxEll = 16;

// Rows r < k: sum over j of the A-side row i = r; rows r >= k: the B-side row
// j = r - k (same formula with the roles of the two spaces exchanged).
__global__ __launch_bounds__(kBlock) void k_sylv_sum(const double* lamA, const double* gA, const double* WA,
                                                     const double* lamB, const double* gB, const double* WB, int k,
                                                     int ell, int nt, double* part, unsigned* counter,
                                                     CheckOut* out) {
  __shared__ double red[pow2_at_least(kSylMaxEll) * kWaves];
  double blocksum = 0.0;
  for (int r = blockIdx.x; r < 2 * k; r += gridDim.x) {
    const bool sideA = r < k;
    const int i = sideA ? r : r - k;
    const double* lx = sideA ? lamA : lamB;
    const double* gx = sideA ? gA : gB;
    const double* ly = sideA ? lamB : lamA;
    const double* gy = sideA ? gB : gA;
    const double* Wy = sideA ? WB : WA;
    double gi[kSylMaxEll];
#pragma unroll
    for (int a = 0; a < kSylMaxEll; ++a) gi[a] = a < ell ? gx[(size_t)i * ell + a] : 0.0;
    const double li = lx[i];
    double acc[kSylMaxEll];
#pragma unroll
    for (int c = 0; c < kSylMaxEll; ++c) acc[c] = 0.0;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
      double dot = 0.0;
#pragma unroll
      for (int a = 0; a < kSylMaxEll; ++a)
        if (a < ell) dot = fma(gi[a], gy[(size_t)j * ell + a], dot);
      const double coef = dot / (li + ly[j]);
#pragma unroll
      for (int c = 0; c < kSylMaxEll; ++c)
        if (c < nt) acc[c] = fma(coef, Wy[(size_t)j * nt + c], acc[c]);
    }
    block_sum<kSylMaxEll>(acc, red);
    double v = 0.0;
    for (int c = 0; c < nt; ++c) v += red[c] * red[c];
    blocksum += v;
    __syncthreads();
  }
  double tot[1] = {threadIdx.x == 0 ? blocksum : 0.0};
  __shared__ double red1[kWaves];
  if (grid_sum_last<1>(tot, red1, part, counter)) {
    if (threadIdx.x == 0) {
      out->res = sqrt(red1[0]);
      out->lam_max = fmax(lamA[k - 1], lamB[k - 1]);
      out->lam_min = fmin(lamA[0], lamB[0]);
    }
  }
}

// ------------------------------------------------------------------ cross approximation
struct AcaState {
  double norm2;  // ||E||_F^2 at the last pick
  double pivot;
  int i, j;
  int t;         // pivots taken
  int stop;
};

constexpr int kAcaThreads = 256;

__device__ __forceinline__ double ytilde(const double* lamA, const double* gA, const double* lamB, const double* gB,
                                         int ell, int i, int j) {
  double dot = 0.0;
  for (int a = 0; a < ell; ++a) dot = fma(gA[(size_t)i * ell + a], gB[(size_t)j * ell + a], dot);
  return -dot / (lamA[i] + lamB[j]);
}

__global__ void k_ytilde(const double* lamA, const double* gA, const double* lamB, const double* gB, int k, int ell,
                         double* E) {
  const int64_t tot = (int64_t)k * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / k), j = (int)(e - (int64_t)i * k);
    E[e] = ytilde(lamA, gA, lamB, gB, ell, i, j);
  }
}

// E -= u v^T (when apply and not stopped); partial max |E| (first index on
// ties) and sum of squares per workgroup.
__global__ __launch_bounds__(kAcaThreads) void k_aca_update_scan(double* E, int rows, int cols, const double* u,
                                                                 const double* v, const AcaState* stt, int apply,
                                                                 double* pmax, int64_t* pidx, double* pnorm) {
  __shared__ double red[kAcaThreads / 64];
  __shared__ double sv[kAcaThreads / 64];
  __shared__ int64_t si[kAcaThreads / 64];
  const bool upd = apply && !stt->stop;
  const int64_t tot = (int64_t)rows * cols;
  double best = -1.0, nrm = 0.0;
  int64_t bi = tot;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    double x = E[e];
    if (upd) {
      const int i = (int)(e / cols), j = (int)(e - (int64_t)i * cols);
      x = fma(-u[i], v[j], x);
      E[e] = x;
    }
    const double ax = fabs(x);
    nrm = fma(x, x, nrm);
    if (ax > best) {  // e increases within a thread: the first maximum is kept
      best = ax;
      bi = e;
    }
  }
  // wave: (value, index) max with the lower index on ties; sum of squares
  auto merge = [&](double ob, int64_t oi) {
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  };
  {
    double ob;
    int lo, hi;
#define LYAP_ACA_XOR(M)                                                 \
    ob = lane_xor<M>(best);                                             \
    lo = lane_xor<M>((int)(bi & 0xffffffff));                           \
    hi = lane_xor<M>((int)(bi >> 32));                                  \
    merge(ob, ((int64_t)hi << 32) | (int64_t)(unsigned)lo);
    LYAP_ACA_XOR(1) LYAP_ACA_XOR(2) LYAP_ACA_XOR(7) LYAP_ACA_XOR(15) LYAP_ACA_XOR(16) LYAP_ACA_XOR(32)
#undef LYAP_ACA_XOR
  }
  nrm = wave_sum(nrm);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sv[wave] = best;
    si[wave] = bi;
    red[wave] = nrm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sv[0], s = red[0];
    int64_t ii = si[0];
    for (int w = 1; w < kAcaThreads / 64; ++w) {
      if (sv[w] > b || (sv[w] == b && si[w] < ii)) { b = sv[w]; ii = si[w]; }
      s += red[w];
    }
    pmax[blockIdx.x] = b;
    pidx[blockIdx.x] = ii;
    pnorm[blockIdx.x] = s;
  }
}

// Total over the partials (fixed order); stop when ||E||_F <= eps, otherwise
// record the pivot (I[t], J[t]).
__global__ void k_aca_pick(const double* pmax, const int64_t* pidx, const double* pnorm, int nparts, const double* E,
                           int rows, int cols, double eps2, int tmax, AcaState* stt, int* I, int* J) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || stt->stop) return;
  double b = -1.0, s = 0.0;
  int64_t ii = (int64_t)rows * cols;
  for (int p = 0; p < nparts; ++p) {
    if (pmax[p] > b || (pmax[p] == b && pidx[p] < ii)) { b = pmax[p]; ii = pidx[p]; }
    s += pnorm[p];
  }
  stt->norm2 = s;
  if (!(s > eps2) || stt->t >= tmax || !(b > 0.0)) {
    stt->stop = 1;
    return;
  }
  const int i = (int)(ii / cols), j = (int)(ii - (int64_t)i * cols);
  stt->i = i;
  stt->j = j;
  stt->pivot = E[ii];
  I[stt->t] = i;
  J[stt->t] = j;
  stt->t += 1;
}

// u = E(:, j), v = E(i, :) / pivot.
__global__ void k_aca_copy(const double* E, int rows, int cols, const AcaState* stt, double* u, double* v) {
  if (stt->stop) return;
  const int i = stt->i, j = stt->j;
  const double pinv = 1.0 / stt->pivot;
  const int len = rows > cols ? rows : cols;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < len; r += gridDim.x * blockDim.x) {
    if (r < rows) u[r] = E[(size_t)r * cols + j];
    if (r < cols) v[r] = E[(size_t)i * cols + r] * pinv;
  }
}

// Core W = Y~(I, J) of the two-sided method, generated from lambda and g.
__global__ void k_core_fill_ytilde(const double* lamA, const double* gA, const double* lamB, const double* gB,
                                   int ell, const int* I, const int* J, int t, double* W) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < t * t; e += gridDim.x * blockDim.x) {
    const int a = e / t, b = e - a * t;
    W[e] = ytilde(lamA, gA, lamB, gB, ell, I[a], J[b]);
  }
}

// Core W = E0(I, J) of an explicit row-major matrix (leading dimension lde).
__global__ void k_core_fill(const double* E0, int64_t lde, const int* I, const int* J, int t, double* W) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < t * t; e += gridDim.x * blockDim.x) {
    const int a = e / t, b = e - a * t;
    W[e] = E0[(size_t)I[a] * lde + J[b]];
  }
}

// Core W = L U without further pivoting (the complete-pivoting order makes
// every pivot the largest remaining entry); B1 = U^{-1}, B2 = L^{-T} (t x t,
// row-major).  One workgroup; W is overwritten by the factors.
__global__ __launch_bounds__(1024) void k_core_lu(int t, double* W, double* B1, double* B2) {
  const int nt = blockDim.x;
  for (int p = 0; p < t; ++p) {
    const double piv = W[(size_t)p * t + p];
    for (int a = p + 1 + threadIdx.x; a < t; a += nt) W[(size_t)a * t + p] /= piv;
    __syncthreads();
    const int rem = t - p - 1;
    for (int e = threadIdx.x; e < rem * rem; e += nt) {
      const int a = p + 1 + e / rem, b = p + 1 + e % rem;
      W[(size_t)a * t + b] = fma(-W[(size_t)a * t + p], W[(size_t)p * t + b], W[(size_t)a * t + b]);
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < t; c += nt) {
    // column c of U^{-1}
    for (int a = t - 1; a >= 0; --a) {
      double x = (a == c) ? 1.0 : 0.0;
      if (a <= c)
        for (int b = a + 1; b <= c; ++b) x = fma(-W[(size_t)a * t + b], B1[(size_t)b * t + c], x);
      B1[(size_t)a * t + c] = a <= c ? x / W[(size_t)a * t + a] : 0.0;
    }
    // column c of L^{-1} (unit lower), stored transposed: B2[c][a] = Linv[a][c]
    for (int a = 0; a < t; ++a) {
      double x = (a == c) ? 1.0 : 0.0;
      if (a > c)
        for (int b = c; b < a; ++b) x = fma(-W[(size_t)a * t + b], B2[(size_t)c * t + b], x);
      B2[(size_t)c * t + a] = a >= c ? x : 0.0;
    }
  }
}

// Cross approximation of the rows x cols row-major matrix E (overwritten by
// the Schur complements): pivots I (rows), J (columns), t of them, chosen by
// complete pivoting until ||E - E(:, J) E(I, J)^{-1} E(I, :)||_F <= eps.
int aca_cross(double* E, int rows, int cols, double eps, int tmax, DevBuf& I, DevBuf& J, hipStream_t st) {
  const int64_t tot = (int64_t)rows * cols;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((tot + kAcaThreads - 1) / kAcaThreads, 1024));
  DevBuf u((size_t)rows * sizeof(double)), v((size_t)cols * sizeof(double));
  DevBuf pmax(grid * sizeof(double)), pidx(grid * sizeof(int64_t)), pnorm(grid * sizeof(double));
  DevBuf stt(sizeof(AcaState));
  I.alloc(std::max(1, tmax) * sizeof(int));
  J.alloc(std::max(1, tmax) * sizeof(int));
  LYAP_HIP(hipMemsetAsync(stt.p, 0, sizeof(AcaState), st));
  const int len = std::max(rows, cols);
  AcaState h{};
  const double eps2 = eps * eps;
  for (int step = 0; step <= tmax; ++step) {
    hipLaunchKernelGGL(k_aca_update_scan, dim3(grid), dim3(kAcaThreads), 0, st, E, rows, cols, u.as<double>(),
                       v.as<double>(), stt.as<AcaState>(), step > 0 ? 1 : 0, pmax.as<double>(),
                       pidx.as<int64_t>(), pnorm.as<double>());
    hipLaunchKernelGGL(k_aca_pick, dim3(1), dim3(64), 0, st, pmax.as<double>(), pidx.as<int64_t>(),
                       pnorm.as<double>(), grid, E, rows, cols, eps2, tmax, stt.as<AcaState>(), I.as<int>(),
                       J.as<int>());
    hipLaunchKernelGGL(k_aca_copy, dim3(std::max(1, std::min((len + 255) / 256, 256))), dim3(256), 0, st, E, rows,
                       cols, stt.as<AcaState>(), u.as<double>(), v.as<double>());
    LYAP_LAUNCHED("aca step");
    if ((step + 1) % 16 == 0 || step == tmax) {
      LYAP_HIP(hipMemcpyAsync(&h, stt.p, sizeof(AcaState), hipMemcpyDeviceToHost, st));
      LYAP_HIP(hipStreamSynchronize(st));
      if (h.stop) break;
    }
  }
  LYAP_REQUIRE(h.stop, LYAP_E_UNSUPPORTED, "truncation rank exceeds %d", tmax);
  LYAP_REQUIRE(!(h.norm2 > eps2) || h.t < tmax || tmax == std::min(rows, cols), LYAP_E_UNSUPPORTED,
               "truncation rank exceeds %d", tmax);
  return h.t;
}

void core_lu_explicit(const double* E0, int64_t lde, const int* I, const int* J, int t, double* B1, double* B2,
                      hipStream_t st) {
  DevBuf W((size_t)t * t * sizeof(double));
  hipLaunchKernelGGL(k_core_fill, dim3(std::max(1, std::min((t * t + 255) / 256, 1024))), dim3(256), 0, st, E0, lde,
                     I, J, t, W.as<double>());
  hipLaunchKernelGGL(k_core_lu, dim3(1), dim3(1024), 0, st, t, W.as<double>(), B1, B2);
  LYAP_LAUNCHED("k_core_lu");
  LYAP_HIP(hipStreamSynchronize(st));  // W is released on return
}

void launch_sylv_sum(const Checker& ca, const Checker& cb, int k, int ell, int nt, double* part, unsigned* counter,
                     CheckOut* out, hipStream_t st) {
  const int grid = std::max(1, std::min(2 * k, 2048));
  hipLaunchKernelGGL(k_sylv_sum, dim3(grid), dim3(kBlock), 0, st, ca.lam(), ca.g(), ca.Wm(), cb.lam(), cb.g(),
                     cb.Wm(), k, ell, nt, part, counter, out);
  LYAP_LAUNCHED("k_sylv_sum");
}

// Returns t; M1, M2: k x t row-major.
int finalise_sylv(const Checker& ca, const Checker& cb, const double* bandA, const double* bandB,
                  const double* gamma1, const double* gamma2, int ell, double eps, DevBuf& M1, DevBuf& M2,
                  hipStream_t st) {
  const int k = ca.k();
  LYAP_REQUIRE(k <= 16384, LYAP_E_UNSUPPORTED, "Sylvester truncation limited to k <= 16384 (got %d)", k);
  const int tmax = std::min(k, 1024);
  DevBuf E((size_t)k * k * sizeof(double));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)k * k + 255) / 256, 1024));
  hipLaunchKernelGGL(k_ytilde, dim3(grid), dim3(256), 0, st, ca.lam(), ca.g(), cb.lam(), cb.g(), k, ell,
                     E.as<double>());
  LYAP_LAUNCHED("k_ytilde");
  DevBuf I, J;
  const int t = aca_cross(E.as<double>(), k, k, eps, tmax, I, J, st);
  if (t <= 0) {
    M1.alloc(8);
    M2.alloc(8);
    return 0;
  }
  DevBuf W((size_t)t * t * sizeof(double)), B1((size_t)t * t * sizeof(double)), B2((size_t)t * t * sizeof(double));
  hipLaunchKernelGGL(k_core_fill_ytilde, dim3(std::max(1, std::min((t * t + 255) / 256, 1024))), dim3(256), 0, st,
                     ca.lam(), ca.g(), cb.lam(), cb.g(), ell, I.as<int>(), J.as<int>(), t, W.as<double>());
  hipLaunchKernelGGL(k_core_lu, dim3(1), dim3(1024), 0, st, t, W.as<double>(), B1.as<double>(), B2.as<double>());
  LYAP_LAUNCHED("k_core_lu");
  DevBuf Lb((size_t)(ell + 1) * k * t * sizeof(double));
  DevBuf XC((size_t)k * t * sizeof(double)), XR((size_t)k * t * sizeof(double));
  DevBuf fail(sizeof(int) * 4);
  LYAP_HIP(hipMemsetAsync(fail.p, 0, sizeof(int) * 4, st));
  // Q Y~(:, J): shifts upsilon_J on T_m, right-hand sides E_1 gamma_1 g2_J
  launch_shift_solve(bandA, ell + 1, ell, k, cb.lam(), cb.g(), gamma1, J.as<int>(), t, Lb.as<double>(),
                     XC.as<double>(), fail.as<int>(), st);
  // P Y~(I, :)^T: shifts lambda_I on J_m, right-hand sides E_1 gamma_2 g1_I
  launch_shift_solve(bandB, ell + 1, ell, k, ca.lam(), ca.g(), gamma2, I.as<int>(), t, Lb.as<double>(),
                     XR.as<double>(), fail.as<int>(), st);
  M1.alloc((size_t)k * t * sizeof(double));
  M2.alloc((size_t)k * t * sizeof(double));
  launch_gemm_xb(XC.as<double>(), k, t, B1.as<double>(), t, M1.as<double>(), st);
  launch_gemm_xb(XR.as<double>(), k, t, B2.as<double>(), t, M2.as<double>(), st);
  int hfail = 0;
  LYAP_HIP(hipMemcpyAsync(&hfail, fail.p, sizeof(int), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  LYAP_REQUIRE(hfail == 0, LYAP_E_INDEFINITE, "shifted operator not positive definite in the Sylvester factor");
  return t;
}

namespace {

double host_fro(const std::vector<double>& v) {
  double s = 0.0;
  for (double x : v) s += x * x;
  return std::sqrt(s);
}

// One Sylvester check in flight: its stream (owned unless it is the
// solver's), completion event, the two sides' workspaces, result buffers (the
// check's output, the extreme Ritz values of both sides, their Lanczos flags)
// and the step it checks.
struct SylvSlot {
  hipStream_t st = nullptr;
  bool own = false;
  hipEvent_t ev = nullptr;
  std::unique_ptr<Checker> ca, cb;
  DevBuf part, counter, chk;
  HostBuf hchk;
  int mm = 0;
  CheckOut* hc() const { return hchk.as<CheckOut>(); }
  double* hl() const { return reinterpret_cast<double*>(hchk.as<char>() + sizeof(CheckOut)); }
  int* hf() const { return reinterpret_cast<int*>(hchk.as<char>() + sizeof(CheckOut) + 4 * sizeof(double)); }
  ~SylvSlot() {
    // a check still running reads the Lanczos sides' buffers: let it end
    if (own && st) (void)hipStreamSynchronize(st);
    if (ev) (void)hipEventDestroy(ev);
    if (own && st) (void)hipStreamDestroy(st);
  }
};

template <typename T>
lyap_status sylv_impl(const lyap_op* A, const lyap_op* B, const double* C1, int64_t ldc1, const double* C2,
                      int64_t ldc2, int S, const lyap_opts& o, sylv_result* out) {
  const auto t_entry = Clock::now();
  hipStream_t st = (hipStream_t)o.stream;
  const int n1 = (int)A->n, n2 = (int)B->n;
  out->n1 = n1;
  out->n2 = n2;
  out->s = S;
  out->ell = S;
  const int maxit = o.max_iter;
  KernelTimer kt;
  kt.st = st;
  kt.on = o.profile != 0;
  LanczosSide<T> sa(A, C1, S, ldc1, maxit, o.two_pass != 0, st, &kt);
  LanczosSide<T> sb(B, C2, S, ldc2, maxit, o.two_pass != 0, st, &kt);
  sa.init();
  sb.init();
  out->beta1 = sa.beta();
  out->beta2 = sb.beta();
  const double b12 = sa.beta() * sb.beta();

  // Checks run on other streams while both sides keep stepping (see
  // solve_std): a check at mm reads only the two leading bands and logs.
  // With a fixed schedule up to kSlots checks are in flight at once, each
  // with a stream and workspaces of its own, read in the order issued (the
  // first under the tolerance ends the iteration, as with one at a time); the
  // steps stay at most kAhead past the next check point.
  constexpr int kAhead = 24, kSlots = 3;
  const bool overlap = o.profile == 0;
  const bool fixed = o.check_every > 0;
  const int nslots = overlap && fixed ? kSlots : 1;
  std::vector<std::unique_ptr<SylvSlot>> slots;
  for (int i = 0; i < nslots; ++i) {
    slots.emplace_back(new SylvSlot);
    SylvSlot& sl = *slots.back();
    if (overlap) {
      LYAP_HIP(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking));
      sl.own = true;
    } else {
      sl.st = st;
    }
    LYAP_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    sl.ca.reset(new Checker(S, S, sl.st));
    sl.cb.reset(new Checker(S, S, sl.st));
    sl.part.alloc(4096 * sizeof(double));
    sl.counter.alloc(64);
    sl.chk.alloc(sizeof(CheckOut));
    sl.hchk.alloc(sizeof(CheckOut) + 4 * sizeof(double) + 4 * sizeof(int));
    LYAP_HIP(hipMemsetAsync(sl.counter.p, 0, 64, st));
  }
  struct EventRing {
    std::vector<hipEvent_t> ev;
    ~EventRing() { for (auto e : ev) (void)hipEventDestroy(e); }
  } er;
  er.ev.resize(kAhead + 1);
  for (auto& e : er.ev) LYAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipEvent_t ev_step = er.ev[kAhead];
  LYAP_HIP(hipStreamSynchronize(st));

  CheckSchedule sched{o.check_every, maxit};
  std::vector<int> hm;
  std::vector<double> hr;
  double check_ms = 0.0, t_to_tol = 0.0, lamA_abs = 0.0, lamB_abs = 0.0, last_res = INFINITY;
  int next_check = sched.first(), m = 0;
  lyap_status status = LYAP_NOT_CONVERGED;
  int head = 0, npend = 0;  // checks in flight: slots head, head + 1, ... (mod nslots)
  int last_launched = 0;
  SylvSlot* done_slot = slots[0].get();  // the slot of the last check read

  auto launch_check = [&](SylvSlot& sl, int mm) {
    LYAP_HIP(hipEventRecord(ev_step, st));
    LYAP_HIP(hipStreamWaitEvent(sl.st, ev_step, 0));
    kt.mark(LYAP_K_CHECK);
    const int k = mm * S;
    Checker &ca = *sl.ca, &cb = *sl.cb;
    ca.prepare(sa.band(), k, sa.gamma_dev(), sa.tau_dev(mm));
    cb.prepare(sb.band(), k, sb.gamma_dev(), sb.tau_dev(mm));
    const int grid = std::max(1, std::min(2 * k, 2048));
    hipLaunchKernelGGL(k_sylv_sum, dim3(grid), dim3(kBlock), 0, sl.st, ca.lam(), ca.g(), ca.Wm(), cb.lam(), cb.g(),
                       cb.Wm(), k, S, S, sl.part.as<double>(), sl.counter.as<unsigned>(), sl.chk.as<CheckOut>());
    LYAP_LAUNCHED("k_sylv_sum");
    double* hl = sl.hl();
    int* hf = sl.hf();
    LYAP_HIP(hipMemcpyAsync(sl.hc(), sl.chk.p, sizeof(CheckOut), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(&hl[0], ca.lam(), sizeof(double), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(&hl[1], ca.lam() + k - 1, sizeof(double), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(&hl[2], cb.lam(), sizeof(double), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(&hl[3], cb.lam() + k - 1, sizeof(double), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(&hf[0], sa.flags_dev(), 2 * sizeof(int), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(&hf[2], sb.flags_dev(), 2 * sizeof(int), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipEventRecord(sl.ev, sl.st));
    sl.mm = mm;
  };
  auto wait_check = [&](SylvSlot& sl) {
    const auto t0 = Clock::now();
    LYAP_HIP(hipEventSynchronize(sl.ev));
    check_ms += ms_since(t0);
    kt.collect();
  };
  auto record = [&](SylvSlot& sl, int mm) -> double {
    const CheckOut c = *sl.hc();
    const double* hl = sl.hl();
    LYAP_REQUIRE(std::isfinite(c.res), LYAP_E_NUMERIC, "residual is not finite at m=%d", mm);
    const double rel = c.res / b12;
    hm.push_back(mm);
    hr.push_back(rel);
    last_res = rel;
    lamA_abs = std::max(std::fabs(hl[0]), std::fabs(hl[1]));
    lamB_abs = std::max(std::fabs(hl[2]), std::fabs(hl[3]));
    if (o.verbose) std::fprintf(stderr, "[sylv] m=%d k=%d res=%.3e\n", mm, mm * S, rel);
    LYAP_REQUIRE(c.lam_max < 0.0, LYAP_E_INDEFINITE,
                 "Ritz value %.3e >= 0 at m=%d: an operator is not negative definite", c.lam_max, mm);
    return rel;
  };
  // returns true when the iteration stops
  auto finish_check = [&](SylvSlot& sl) -> bool {
    done_slot = &sl;
    out->n_checks++;
    const int mm = sl.mm;
    const int* hf = sl.hf();
    int fbk = 0, fnf = 0;
    for (int f : {hf[0], hf[2]})
      if (f > 0 && f <= mm && (fbk == 0 || f < fbk)) fbk = f;
    for (int f : {hf[1], hf[3]})
      if (f > 0 && f <= mm && (fnf == 0 || f < fnf)) fnf = f;
    // non-finite values that follow a breakdown belong to the breakdown
    LYAP_REQUIRE(!(fnf > 0 && (fbk == 0 || fnf <= fbk)), LYAP_E_NUMERIC,
                 "non-finite values in the Lanczos recurrences at step %d", fnf);
    if (fbk > 0) {  // a rank-deficient block: check the basis it ends instead
      LYAP_HIP(hipStreamSynchronize(st));
      launch_check(sl, fbk);
      out->n_checks++;
      wait_check(sl);
      const double rel = record(sl, fbk);
      m = fbk;
      if (rel <= o.tol) {
        status = LYAP_OK;
        t_to_tol = ms_since(t_entry);
      } else {
        status = LYAP_E_BREAKDOWN;
        set_error("block Lanczos breakdown at m=%d with residual %.3e above tol", fbk, rel);
      }
      return true;
    }
    const double rel = record(sl, mm);
    if (rel <= o.tol) {
      status = LYAP_OK;
      m = mm;
      t_to_tol = ms_since(t_entry);
      return true;
    }
    if (mm >= maxit) {
      m = mm;
      return true;
    }
    if (!fixed) next_check = sched.next(mm, rel, o.tol);
    return false;
  };

  const auto t_pass1 = Clock::now();
  int steps = 0;
  while (true) {
    if (npend > 0) {
      SylvSlot& sl = *slots[head];
      const hipError_t q = hipEventQuery(sl.ev);
      const bool stuck = steps >= maxit || (fixed && npend == nslots && steps >= next_check + kAhead);
      if (q == hipSuccess || stuck || !overlap) {
        if (q != hipSuccess) wait_check(sl);
        --npend;
        head = (head + 1) % nslots;
        if (finish_check(sl)) break;
        continue;
      } else if (q != hipErrorNotReady) {
        LYAP_HIP(q);
      }
    }
    if (npend < nslots && next_check > last_launched && (steps >= next_check || steps >= maxit)) {
      const int mm = std::min(next_check, steps);
      launch_check(*slots[(head + npend) % nslots], mm);
      ++npend;
      last_launched = mm;
      if (fixed) next_check = std::min(mm + sched.d, maxit);
      continue;
    }
    if (steps >= maxit) continue;
    if (fixed && steps >= next_check + kAhead) continue;  // waits for a slot
    if (steps >= kAhead) LYAP_HIP(hipEventSynchronize(er.ev[steps % kAhead]));
    sa.step();
    sb.step();
    LYAP_HIP(hipEventRecord(er.ev[steps % kAhead], st));
    ++steps;
  }
  // finalisation reads the eigendecompositions of the check that ended the iteration
  if (overlap) LYAP_HIP(hipStreamWaitEvent(st, done_slot->ev, 0));
  Checker &ca = *done_slot->ca, &cb = *done_slot->cb;
  const double pass1_ms = ms_since(t_pass1) - check_ms;
  out->m = m;
  out->res = last_res;
  out->n_hist = (int)hm.size();
  out->hist_m = (int32_t*)std::malloc(std::max<size_t>(1, hm.size()) * sizeof(int32_t));
  out->hist_res = (double*)std::malloc(std::max<size_t>(1, hr.size()) * sizeof(double));
  for (size_t i = 0; i < hm.size(); ++i) {
    out->hist_m[i] = hm[i];
    out->hist_res[i] = hr[i];
  }

  // ---- finalisation
  const auto t_fin = Clock::now();
  std::vector<double> tau_h(S * S), iota_h(S * S);
  LYAP_HIP(hipMemcpyAsync(tau_h.data(), sa.tau_dev(m), S * S * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipMemcpyAsync(iota_h.data(), sb.tau_dev(m), S * S * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  // ||R(Y) - R(Y + dY)|| <= (||T_m underline|| + ||J_m underline||) ||dY||_F
  const double nu = lamA_abs + host_fro(tau_h) + lamB_abs + host_fro(iota_h);
  double eps = o.trunc_eps;
  if (!(eps >= 0.0)) eps = std::min(1e-12, 0.05 * o.tol / nu) * b12;
  out->trunc_eps = eps;
  DevBuf M1, M2;
  kt.mark(LYAP_K_FINAL);
  const int t = finalise_sylv(ca, cb, sa.band(), sb.band(), sa.gamma_dev(), sb.gamma_dev(), S, eps, M1, M2, st);
  kt.collect();
  out->t = t;
  const double fin_ms = ms_since(t_fin);

  // ---- Z1, Z2 (second pass on each side, or the stored bases)
  const auto t_p2 = Clock::now();
  lyap_opts oz = o;
  bool own1 = false, own2 = false;
  out->Z1 = alloc_output(oz, (size_t)n1 * std::max(t, 1) * sizeof(double), &own1);
  out->Z2 = alloc_output(oz, (size_t)n2 * std::max(t, 1) * sizeof(double), &own2);
  out->owns_Z = own1 ? 1 : 0;
  double zbytes = 0.0;
  sa.accumulate_Z(m, M1.as<double>(), t, out->Z1, n1, &zbytes);
  sb.accumulate_Z(m, M2.as<double>(), t, out->Z2, n2, &zbytes);
  LYAP_HIP(hipStreamSynchronize(st));
  kt.collect();
  const double p2_ms = ms_since(t_p2);

  if (o.want_T) {
    const int k = m * S;
    auto band_out = [&](const double* dev) {
      double* h = (double*)std::malloc((size_t)(S + 1) * k * sizeof(double));
      LYAP_HIP(hipMemcpy(h, dev, (size_t)(S + 1) * k * sizeof(double), hipMemcpyDeviceToHost));
      for (int c = 0; c < k; ++c)
        for (int d = 0; d <= S; ++d)
          if (c + d >= k) h[(size_t)c * (S + 1) + d] = 0.0;
      return h;
    };
    out->T_band = band_out(sa.band());
    out->J_band = band_out(sb.band());
    auto sq = [&](const double* rm) {
      double* h = (double*)std::malloc(S * S * sizeof(double));
      rowmajor_to_colmajor(rm, S, S, h);
      return h;
    };
    out->gamma1 = sq(sa.gamma_host());
    out->gamma2 = sq(sb.gamma_host());
    out->tau = sq(tau_h.data());
    out->iota = sq(iota_h.data());
  }
  out->times_ms[LYAP_T_PASS1] = pass1_ms;
  out->times_ms[LYAP_T_CHECKS] = check_ms;
  out->times_ms[LYAP_T_FINAL] = fin_ms;
  out->times_ms[LYAP_T_PASS2] = p2_ms;
  out->times_ms[LYAP_T_TOTAL] = ms_since(t_entry);
  out->times_ms[LYAP_T_TO_TOL] = t_to_tol;
  for (int i = 0; i < LYAP_K_COUNT; ++i) {
    out->kern_ms[i] = kt.ms[i];
    out->kern_n[i] = kt.n[i];
  }
  // streaming kernels of both sides alternate: bytes per launch averaged over the two operators
  double kb1[12] = {0}, kb2[12] = {0};
  fill_kernel_bytes<T>(n1, S, sa.op().coef_bytes_per_row(), kt, zbytes, kb1);
  fill_kernel_bytes<T>(n2, S, sb.op().coef_bytes_per_row(), kt, zbytes, kb2);
  for (int i = 0; i < LYAP_K_COUNT; ++i) out->kern_bytes[i] = 0.5 * (kb1[i] + kb2[i]);
  out->kern_bytes[LYAP_K_ZFLUSH] = kb1[LYAP_K_ZFLUSH];
  out->status = status;
  return status;
}

}  // namespace
}  // namespace lyap

extern "C" lyap_status sylv_solve(const lyap_op* A, const lyap_op* B, const double* C1, int64_t ldc1,
                                  const double* C2, int64_t ldc2, int32_t s, const lyap_opts* opts,
                                  sylv_result* out) {
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
    validate_op(B);
    LYAP_REQUIRE(C1 != nullptr && C2 != nullptr, LYAP_E_ARG, "C1 or C2 is NULL");
    LYAP_REQUIRE(s >= 1 && s <= 8, LYAP_E_ARG, "s=%d out of range 1..8", s);
    LYAP_REQUIRE(ldc1 >= A->n && ldc2 >= B->n, LYAP_E_ARG, "leading dimension below n");
    LYAP_REQUIRE(s <= A->n && s <= B->n, LYAP_E_ARG, "s > n");
    LYAP_REQUIRE(o.tol > 0.0 && o.tol < 1.0, LYAP_E_ARG, "tol=%g must be in (0,1)", o.tol);
    LYAP_REQUIRE(o.max_iter >= 1 && (int64_t)o.max_iter * s <= (int64_t)1 << 20, LYAP_E_ARG,
                 "max_iter=%d out of range", o.max_iter);
    LYAP_REQUIRE(o.check_every >= 0, LYAP_E_ARG, "check_every must be >= 0");
    LYAP_REQUIRE(o.method == LYAP_METHOD_STD || o.method == LYAP_METHOD_EXT, LYAP_E_ARG, "unknown method %d",
                 o.method);
    LYAP_REQUIRE(o.storage == LYAP_STORE_F64 || o.storage == LYAP_STORE_F32, LYAP_E_ARG, "unknown storage %d",
                 o.storage);
    if (o.method == LYAP_METHOD_EXT) {
      lyap_status st = solve_sylv_ext(A, B, C1, ldc1, C2, ldc2, s, o, out);
      out->status = st;
      return st;
    }
    lyap_status st = o.storage == LYAP_STORE_F64 ? sylv_impl<double>(A, B, C1, ldc1, C2, ldc2, s, o, out)
                                                 : sylv_impl<float>(A, B, C1, ldc1, C2, ldc2, s, o, out);
    out->status = st;
    return st;
  } catch (const Error& e) {
    out->status = e.st;
    return e.st;
  }
}

extern "C" void sylv_result_free(sylv_result* r) {
  if (!r) return;
  std::free(r->hist_m);
  std::free(r->hist_res);
  std::free(r->T_band);
  std::free(r->J_band);
  std::free(r->gamma1);
  std::free(r->gamma2);
  std::free(r->tau);
  std::free(r->iota);
  if (r->owns_Z) {
    if (r->Z1) (void)hipFree(r->Z1);
    if (r->Z2) (void)hipFree(r->Z2);
  }
  std::memset(r, 0, sizeof(*r));
}
