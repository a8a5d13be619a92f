// sylv_solve_small_b: A X + X B + C1 C2^T = 0 with A large and sparse and B
// small and dense (Section 5.2, "Large A and small B").  Only A is projected:
// V_m spans K_m(A, C1) (the block Lanczos side of lyap_solve), X_m = V_m Y_m,
// and the one-sided Galerkin condition V_m^T R_m = 0 gives the k x n2 reduced
// equation T_m Y + Y B + E_1 gamma_1 C2^T = 0.
//
// B = P Upsilon P^T is computed once, before the iteration, by parallel
// cyclic Jacobi (k_jac_round), and H = P^T C2 with it.  With
// T_m = Q Lambda Q^T and g = (E_1^T Q)^T gamma_1 (k x ell) the solution is
// Y_m = Q Y~ P^T, Y~_ji = -(g_j . H_i) / (lambda_j + upsilon_i), and the
// residual R_m = V_{m+1} tau E_m^T Y_m is evaluated without Y_m (Algorithm 5):
//   ||R_m||_F^2 = sum_i || sum_j (g_j . H_i) / (upsilon_i + lambda_j) W_j ||^2,
// W = (E_m^T Q)^T tau^T (k x ell), one workgroup per eigenvalue of B
// (k_alg5_sum).
//
// Finalisation: the columns of Y1 = Q Y~ (k x n2) are banded shifted solves,
//   Y1(:, i) = -(T_m + upsilon_i I)^{-1} E_1 gamma_1 H_i^T,
// so Q is never formed; Y1 is truncated by cross approximation with complete
// pivoting (error = norm of the remaining Schur complement <= eps), giving
// Y1 ~= M1 N^T; Z1 = V_m M1 (second Lanczos pass or stored basis) and
// Z2 = P N, so that Z1 Z2^T ~= V_m Y1 P^T = X_m.
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "aca.hpp"
#include "check.hpp"
#include "side.hpp"
#include "solver.hpp"

namespace lyap {

constexpr int kSymEigMax = 2048;  // largest B (n2) handled
constexpr int kSmallBMaxEll = 8;

// ------------------------------------------------------------------ Jacobi eigensolver
// Pair a (0 <= a < np/2) of round r (0 <= r < np-1) of the round-robin
// ordering: every index meets every other exactly once per np-1 rounds and
// the np/2 pairs of one round are disjoint, so their rotations commute.
__device__ __forceinline__ void jac_pair(int r, int a, int np, int& p, int& q) {
  const int M = np - 1;
  int x, y;
  if (a == 0) {
    x = r;
    y = M;
  } else {
    x = (r + a) % M;
    y = (r - a + M) % M;
  }
  p = x < y ? x : y;
  q = x < y ? y : x;
}

// Rotation J = [[c, s], [-s, c]] on (p, q) with (J^T B J)_pq = 0 (the smaller
// of the two angles): t = tan = sign(th) / (|th| + sqrt(1 + th^2)),
// th = (b_qq - b_pp) / (2 b_pq).
__device__ __forceinline__ void jac_rot(double app, double aqq, double apq, double& c, double& s, double& t) {
  if (apq == 0.0) {
    c = 1.0;
    s = 0.0;
    t = 0.0;
    return;
  }
  const double th = (aqq - app) / (2.0 * apq);
  const double ath = fabs(th);
  double tt;
  if (ath > 1e150) tt = 0.5 / th;  // th^2 would overflow; tan ~ 1 / (2 th)
  else tt = 1.0 / (ath + sqrt(1.0 + th * th));
  if (th < 0.0) tt = -tt;
  t = tt;
  c = 1.0 / sqrt(1.0 + tt * tt);
  s = tt * c;
}

// Bw (np x np row-major, np even) = symmetric B from its lower triangle
// (column-major, ldb), zero padding; V = I.
__global__ void k_jac_init(const double* B, int n, int64_t ldb, int np, double* Bw, double* V) {
  const int64_t tot = (int64_t)np * np;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / np), j = (int)(e - (int64_t)i * np);
    double v = 0.0;
    if (i < n && j < n) v = i >= j ? B[(size_t)j * ldb + i] : B[(size_t)i * ldb + j];
    Bw[e] = v;
    V[e] = i == j ? 1.0 : 0.0;
  }
}

// One round: Bout = J^T Bin J for the np/2 disjoint rotations of round r, and
// V <- V J.  Thread (a, b) owns the 2 x 2 block (pair a rows, pair b columns)
// and the rows 2b, 2b+1 of V in pair a's columns.  Blocks (a, b) and (b, a)
// are computed with the same operations (the one with a <= b, transposed), so
// Bout stays exactly symmetric; the rotated pair's own off-diagonal entry is
// set to zero.
__global__ __launch_bounds__(256) void k_jac_round(const double* __restrict__ Bin, double* __restrict__ Bout,
                                                   double* __restrict__ V, int np, int r) {
  const int h = np / 2;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= h * h) return;
  const int a = idx / h, b = idx - a * h;
  int pa, qa, pb, qb;
  jac_pair(r, a, np, pa, qa);
  jac_pair(r, b, np, pb, qb);
  double ca, sa, ta, cb, sb, tb;
  jac_rot(Bin[(size_t)pa * np + pa], Bin[(size_t)qa * np + qa], Bin[(size_t)pa * np + qa], ca, sa, ta);
  jac_rot(Bin[(size_t)pb * np + pb], Bin[(size_t)qb * np + qb], Bin[(size_t)pb * np + qb], cb, sb, tb);
  if (a == b) {
    const double apq = Bin[(size_t)pa * np + qa];
    Bout[(size_t)pa * np + pa] = Bin[(size_t)pa * np + pa] - ta * apq;
    Bout[(size_t)qa * np + qa] = Bin[(size_t)qa * np + qa] + ta * apq;
    Bout[(size_t)pa * np + qa] = 0.0;
    Bout[(size_t)qa * np + pa] = 0.0;
  } else {
    // canonical block: rows of pair u, columns of pair v, u < v
    const bool fw = a < b;
    const int pu = fw ? pa : pb, qu = fw ? qa : qb, pv = fw ? pb : pa, qv = fw ? qb : qa;
    const double cu = fw ? ca : cb, su = fw ? sa : sb, cv = fw ? cb : ca, sv = fw ? sb : sa;
    const double x11 = Bin[(size_t)pu * np + pv], x12 = Bin[(size_t)pu * np + qv];
    const double x21 = Bin[(size_t)qu * np + pv], x22 = Bin[(size_t)qu * np + qv];
    // X J_v
    const double y11 = cv * x11 - sv * x12, y12 = sv * x11 + cv * x12;
    const double y21 = cv * x21 - sv * x22, y22 = sv * x21 + cv * x22;
    // J_u^T (X J_v)
    const double z11 = cu * y11 - su * y21, z21 = su * y11 + cu * y21;
    const double z12 = cu * y12 - su * y22, z22 = su * y12 + cu * y22;
    if (fw) {
      Bout[(size_t)pu * np + pv] = z11;
      Bout[(size_t)pu * np + qv] = z12;
      Bout[(size_t)qu * np + pv] = z21;
      Bout[(size_t)qu * np + qv] = z22;
    } else {  // this thread's block is the transpose
      Bout[(size_t)pv * np + pu] = z11;
      Bout[(size_t)qv * np + pu] = z12;
      Bout[(size_t)pv * np + qu] = z21;
      Bout[(size_t)qv * np + qu] = z22;
    }
  }
#pragma unroll
  for (int rr = 2 * b; rr < 2 * b + 2; ++rr) {
    const double vp = V[(size_t)rr * np + pa], vq = V[(size_t)rr * np + qa];
    V[(size_t)rr * np + pa] = ca * vp - sa * vq;
    V[(size_t)rr * np + qa] = sa * vp + ca * vq;
  }
}

// Convergence measures over the leading n x n part: max over p != q of
// |b_pq| / sqrt(|b_pp b_qq|) (infinite when that is 0 and b_pq != 0), the
// sum of squares of the off-diagonal entries and of all entries.
// part: 3 doubles per workgroup.
__global__ __launch_bounds__(256) void k_jac_off(const double* Bw, int np, int n, double* part) {
  __shared__ double red[3 * 4];
  double mx = 0.0, off = 0.0, all = 0.0;
  const int64_t tot = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    const double x = Bw[(size_t)i * np + j];
    all = fma(x, x, all);
    if (i != j) {
      off = fma(x, x, off);
      if (x != 0.0) {
        const double d = sqrt(fabs(Bw[(size_t)i * np + i]) * fabs(Bw[(size_t)j * np + j]));
        const double rt = d > 0.0 ? fabs(x) / d : INFINITY;
        mx = fmax(mx, rt);
      }
    }
  }
  off = wave_sum(off);
  all = wave_sum(all);
  mx = fmax(mx, lane_xor<1>(mx));
  mx = fmax(mx, lane_xor<2>(mx));
  mx = fmax(mx, lane_xor<7>(mx));
  mx = fmax(mx, lane_xor<15>(mx));
  mx = fmax(mx, lane_xor<16>(mx));
  mx = fmax(mx, lane_xor<32>(mx));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[w * 3 + 0] = mx;
    red[w * 3 + 1] = off;
    red[w * 3 + 2] = all;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = red[0], b = red[1], c = red[2];
    for (int q = 1; q < 4; ++q) {
      a = fmax(a, red[q * 3]);
      b += red[q * 3 + 1];
      c += red[q * 3 + 2];
    }
    part[blockIdx.x * 3 + 0] = a;
    part[blockIdx.x * 3 + 1] = b;
    part[blockIdx.x * 3 + 2] = c;
  }
}

__global__ void k_jac_off_final(const double* part, int nparts, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int q = 0; q < nparts; ++q) {
    a = fmax(a, part[q * 3]);
    b += part[q * 3 + 1];
    c += part[q * 3 + 2];
  }
  out[0] = a;
  out[1] = b;
  out[2] = c;
}

// Ascending order of the diagonal (ties by index).
__global__ void k_jac_rank(const double* Bw, int np, int n, int* rank) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = Bw[(size_t)i * np + i];
  int r = 0;
  for (int j = 0; j < n; ++j) {
    const double dj = Bw[(size_t)j * np + j];
    r += (dj < di || (dj == di && j < i)) ? 1 : 0;
  }
  rank[i] = r;
}

// w[rank_i] = b_ii, P(:, rank_i) = V(0:n, i)  (P column-major, ldp).
__global__ void k_jac_out(const double* Bw, const double* V, int np, int n, const int* rank, double* w, double* P,
                          int64_t ldp) {
  const int64_t tot = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), row = (int)(e - (int64_t)i * n);
    const int ri = rank[i];
    P[(size_t)ri * ldp + row] = V[(size_t)row * np + i];
    if (row == 0) w[ri] = Bw[(size_t)i * np + i];
  }
}

// B = P diag(w) P^T; returns the number of sweeps.
int sym_eig(const double* B, int n, int64_t ldb, double* w, double* P, int64_t ldp, hipStream_t st) {
  const int npad = (n % 2 == 0) ? n : n + 1;
  const size_t mat = (size_t)npad * npad * sizeof(double);
  DevBuf B0(mat), B1(mat), V(mat), rank((size_t)n * sizeof(int));
  const int64_t tot = (int64_t)npad * npad;
  const int gfill = (int)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 4096));
  hipLaunchKernelGGL(k_jac_init, dim3(gfill), dim3(256), 0, st, B, n, ldb, npad, B0.as<double>(), V.as<double>());
  LYAP_LAUNCHED("k_jac_init");
  const int h = npad / 2;
  const int ground = (h * h + 255) / 256;
  const int goff = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n * n + 255) / 256, 256));
  DevBuf part((size_t)goff * 3 * sizeof(double)), conv(4 * sizeof(double));
  double hc[3] = {0.0, 0.0, 0.0};
  double* cur = B0.as<double>();
  double* nxt = B1.as<double>();
  constexpr double kEpsMach = 2.220446049250313e-16;
  constexpr int kMaxSweeps = 60;
  int sweeps = 0;
  while (true) {
    hipLaunchKernelGGL(k_jac_off, dim3(goff), dim3(256), 0, st, cur, npad, n, part.as<double>());
    hipLaunchKernelGGL(k_jac_off_final, dim3(1), dim3(64), 0, st, part.as<double>(), goff, conv.as<double>());
    LYAP_LAUNCHED("k_jac_off");
    LYAP_HIP(hipMemcpyAsync(hc, conv.p, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipStreamSynchronize(st));
    LYAP_REQUIRE(std::isfinite(hc[1]) && std::isfinite(hc[2]), LYAP_E_NUMERIC, "B has non-finite entries");
    // relative accuracy (every |b_pq| <= eps sqrt(|b_pp b_qq|)) or, for a
    // matrix with zero diagonal entries, norm-wise accuracy
    if (hc[0] <= kEpsMach || std::sqrt(hc[1]) <= 0.125 * kEpsMach * std::sqrt(hc[2])) break;
    LYAP_REQUIRE(sweeps < kMaxSweeps, LYAP_E_NUMERIC, "Jacobi eigensolver did not converge in %d sweeps",
                 kMaxSweeps);
    for (int r = 0; r < npad - 1; ++r) {
      hipLaunchKernelGGL(k_jac_round, dim3(ground), dim3(256), 0, st, cur, nxt, V.as<double>(), npad, r);
      std::swap(cur, nxt);
    }
    LYAP_LAUNCHED("k_jac_round");
    ++sweeps;
  }
  hipLaunchKernelGGL(k_jac_rank, dim3((n + 255) / 256), dim3(256), 0, st, cur, npad, n, rank.as<int>());
  const int gout = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n * n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_jac_out, dim3(gout), dim3(256), 0, st, cur, V.as<double>(), npad, n, rank.as<int>(), w, P,
                     ldp);
  LYAP_LAUNCHED("k_jac_out");
  LYAP_HIP(hipStreamSynchronize(st));  // the work buffers are released on return
  return sweeps;
}

// ------------------------------------------------------------------ Algorithm 5 inputs and sum
// H = P^T C2 (n2 x S, row-major); P column-major n2 x n2, C2 column-major (ldc).
__global__ void k_pt_c2(const double* P, int n2, int64_t ldp, const double* C2, int64_t ldc, int S, double* H) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2 * S) return;
  const int i = e / S, c = e - i * S;
  double acc = 0.0;
  for (int r = 0; r < n2; ++r) acc = fma(P[(size_t)i * ldp + r], C2[(size_t)c * ldc + r], acc);
  H[e] = acc;
}

// ||C||_F^2 of an n x S column-major block (one workgroup).
__global__ __launch_bounds__(kBlock) void k_fro2(const double* C, int n, int64_t ldc, int S, double* out) {
  __shared__ double red[kWaves];
  double acc[1] = {0.0};
  for (int c = 0; c < S; ++c)
    for (int r = threadIdx.x; r < n; r += kBlock) acc[0] = fma(C[(size_t)c * ldc + r], C[(size_t)c * ldc + r], acc[0]);
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) out[0] = red[0];
}

// Algorithm 5: workgroup row i (grid-stride over the n2 eigenvalues of B)
// forms sum_j (H_i . g_j) / (upsilon_i + lambda_j) W_j and adds its squared
// norm; the last workgroup totals the partials in a fixed order.
__global__ __launch_bounds__(kBlock) void k_alg5_sum(const double* lam, const double* g, const double* Wm, int k,
                                                     int ell, const double* ups, const double* H, int n2,
                                                     double* part, unsigned* counter, CheckOut* out) {
  __shared__ double red[pow2_at_least(kSmallBMaxEll) * kWaves];
  double blocksum = 0.0;
  for (int i = blockIdx.x; i < n2; i += gridDim.x) {
    double hi[kSmallBMaxEll];
#pragma unroll
    for (int a = 0; a < kSmallBMaxEll; ++a) hi[a] = a < ell ? H[(size_t)i * ell + a] : 0.0;
    const double ui = ups[i];
    double acc[kSmallBMaxEll];
#pragma unroll
    for (int c = 0; c < kSmallBMaxEll; ++c) acc[c] = 0.0;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
      double dot = 0.0;
#pragma unroll
      for (int a = 0; a < kSmallBMaxEll; ++a)
        if (a < ell) dot = fma(hi[a], g[(size_t)j * ell + a], dot);
      const double coef = dot / (ui + lam[j]);
#pragma unroll
      for (int c = 0; c < kSmallBMaxEll; ++c)
        if (c < ell) acc[c] = fma(coef, Wm[(size_t)j * ell + c], acc[c]);
    }
    block_sum<kSmallBMaxEll>(acc, red);
    double v = 0.0;
    for (int c = 0; c < ell; ++c) v += red[c] * red[c];
    blocksum += v;
    __syncthreads();
  }
  double tot[1] = {threadIdx.x == 0 ? blocksum : 0.0};
  __shared__ double red1[kWaves];
  if (grid_sum_last<1>(tot, red1, part, counter)) {
    if (threadIdx.x == 0) {
      out->res = sqrt(red1[0]);
      out->lam_max = lam[k - 1];
      out->lam_min = lam[0];
    }
  }
}

// ------------------------------------------------------------------ finalisation kernels
__global__ void k_iota(int* v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// X1 (k x t column-major) = Y1(:, I): columns I of the k x n2 column-major Y1.
__global__ void k_gather_cols(const double* Y1, int k, const int* I, int t, double* X1) {
  const int64_t tot = (int64_t)k * t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / k), r = (int)(e - (int64_t)b * k);
    X1[e] = Y1[(size_t)I[b] * k + r];
  }
}

// X2 (n2 x t column-major) = Y1(J, :)^T.
__global__ void k_gather_rows(const double* Y1, int k, int n2, const int* J, int t, double* X2) {
  const int64_t tot = (int64_t)n2 * t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / n2), i = (int)(e - (int64_t)b * n2);
    X2[e] = Y1[(size_t)i * k + J[b]];
  }
}

// Z2 (n2 x t column-major, ldz) = P N, N n2 x t row-major.
__global__ void k_pn(const double* P, int n2, int64_t ldp, const double* N, int t, double* Z2, int64_t ldz) {
  const int64_t tot = (int64_t)n2 * t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / n2), row = (int)(e - (int64_t)c * n2);
    double acc = 0.0;
    for (int a = 0; a < n2; ++a) acc = fma(P[(size_t)a * ldp + row], N[(size_t)a * t + c], acc);
    Z2[(size_t)c * ldz + row] = acc;
  }
}

namespace {

inline int grid_for_elems(int64_t tot, int cap = 4096) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, cap));
}

// One Algorithm 5 check in flight: its stream (owned unless it is the
// solver's), completion event, workspace, result buffers (the check's output,
// the extreme Ritz values, the Lanczos flags) and the step it checks.
struct Alg5Slot {
  hipStream_t st = nullptr;
  bool own = false;
  hipEvent_t ev = nullptr;
  std::unique_ptr<Checker> ck;
  DevBuf part, counter, chk;
  HostBuf hchk;
  int mm = 0;
  CheckOut* hc() const { return hchk.as<CheckOut>(); }
  double* hl() const { return reinterpret_cast<double*>(hchk.as<char>() + sizeof(CheckOut)); }
  int* hf() const { return reinterpret_cast<int*>(hchk.as<char>() + sizeof(CheckOut) + 2 * sizeof(double)); }
  ~Alg5Slot() {
    // a check still running reads the Lanczos side's buffers: let it end
    if (own && st) (void)hipStreamSynchronize(st);
    if (ev) (void)hipEventDestroy(ev);
    if (own && st) (void)hipStreamDestroy(st);
  }
};


template <typename T>
lyap_status smallb_impl(const lyap_op* A, const double* B, int n2, int64_t ldb, const double* C1, int64_t ldc1,
                        const double* C2, int64_t ldc2, int S, const lyap_opts& o, sylv_result* out) {
  const auto t_entry = Clock::now();
  hipStream_t st = (hipStream_t)o.stream;
  const int n1 = (int)A->n;
  out->n1 = n1;
  out->n2 = n2;
  out->s = S;
  out->ell = S;
  const int maxit = o.max_iter;
  KernelTimer kt;
  kt.st = st;
  kt.on = o.profile != 0;
  LanczosSide<T> sa(A, C1, S, ldc1, maxit, o.two_pass != 0, st, &kt);
  sa.init();
  out->beta1 = sa.beta();

  // B = P Upsilon P^T and H = P^T C2, once (Section 5.2); beta2 = ||C2||_F
  DevBuf ups((size_t)n2 * sizeof(double)), P((size_t)n2 * n2 * sizeof(double)), H((size_t)n2 * S * sizeof(double));
  DevBuf b2(sizeof(double));
  sym_eig(B, n2, ldb, ups.as<double>(), P.as<double>(), n2, st);
  hipLaunchKernelGGL(k_pt_c2, dim3((n2 * S + 255) / 256), dim3(256), 0, st, P.as<double>(), n2, (int64_t)n2, C2, ldc2,
                     S, H.as<double>());
  hipLaunchKernelGGL(k_fro2, dim3(1), dim3(kBlock), 0, st, C2, n2, ldc2, S, b2.as<double>());
  LYAP_LAUNCHED("k_pt_c2");
  double hb[3];
  LYAP_HIP(hipMemcpyAsync(&hb[0], b2.p, sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipMemcpyAsync(&hb[1], ups.as<double>(), sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipMemcpyAsync(&hb[2], ups.as<double>() + n2 - 1, sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  out->beta2 = std::sqrt(hb[0]);
  LYAP_REQUIRE(std::isfinite(out->beta2) && out->beta2 > 0.0, LYAP_E_ARG, "C2 is zero or not finite");
  LYAP_REQUIRE(hb[2] < 0.0, LYAP_E_INDEFINITE, "B has the eigenvalue %.3e >= 0: not negative definite", hb[2]);
  const double ups_abs = std::max(std::fabs(hb[1]), std::fabs(hb[2]));
  const double b12 = out->beta1 * out->beta2;

  // Checks on other streams while the Lanczos steps proceed (as in
  // lyap_solve): a check at mm reads only the leading band and the log.  With
  // a fixed schedule up to kSlots checks are in flight at once, each with a
  // stream and workspace of its own, read in the order issued (the first
  // under the tolerance ends the iteration, as with one at a time); the steps
  // stay at most kAhead past the next check point.
  constexpr int kAhead = 24, kSlots = 3;
  const bool overlap = o.profile == 0;
  const bool fixed = o.check_every > 0;
  const int nslots = overlap && fixed ? kSlots : 1;
  std::vector<std::unique_ptr<Alg5Slot>> slots;
  for (int i = 0; i < nslots; ++i) {
    slots.emplace_back(new Alg5Slot);
    Alg5Slot& sl = *slots.back();
    if (overlap) {
      LYAP_HIP(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking));
      sl.own = true;
    } else {
      sl.st = st;
    }
    LYAP_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    sl.ck.reset(new Checker(S, S, sl.st));
    sl.part.alloc(4096 * sizeof(double));
    sl.counter.alloc(64);
    sl.chk.alloc(sizeof(CheckOut));
    sl.hchk.alloc(sizeof(CheckOut) + 2 * sizeof(double) + 2 * sizeof(int));
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
  double check_ms = 0.0, t_to_tol = 0.0, lam_abs = 0.0, last_res = INFINITY;
  int next_check = sched.first(), m = 0;
  lyap_status status = LYAP_NOT_CONVERGED;
  int head = 0, npend = 0;  // checks in flight: slots head, head + 1, ... (mod nslots)
  int last_launched = 0;
  Alg5Slot* done_slot = slots[0].get();  // the slot of the last check read

  auto launch_check = [&](Alg5Slot& sl, int mm) {
    LYAP_HIP(hipEventRecord(ev_step, st));
    LYAP_HIP(hipStreamWaitEvent(sl.st, ev_step, 0));
    kt.mark(LYAP_K_CHECK);
    const int k = mm * S;
    Checker& ca = *sl.ck;
    ca.prepare(sa.band(), k, sa.gamma_dev(), sa.tau_dev(mm));
    const int grid = std::max(1, std::min(n2, 2048));
    hipLaunchKernelGGL(k_alg5_sum, dim3(grid), dim3(kBlock), 0, sl.st, ca.lam(), ca.g(), ca.Wm(), k, S,
                       ups.as<double>(), H.as<double>(), n2, sl.part.as<double>(), sl.counter.as<unsigned>(),
                       sl.chk.as<CheckOut>());
    LYAP_LAUNCHED("k_alg5_sum");
    LYAP_HIP(hipMemcpyAsync(sl.hc(), sl.chk.p, sizeof(CheckOut), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(&sl.hl()[0], ca.lam(), sizeof(double), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(&sl.hl()[1], ca.lam() + k - 1, sizeof(double), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(&sl.hf()[0], sa.flags_dev(), 2 * sizeof(int), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipEventRecord(sl.ev, sl.st));
    sl.mm = mm;
  };
  auto wait_check = [&](Alg5Slot& sl) {
    const auto t0 = Clock::now();
    LYAP_HIP(hipEventSynchronize(sl.ev));
    check_ms += ms_since(t0);
    kt.collect();
  };
  auto record = [&](Alg5Slot& sl, int mm) -> double {
    const CheckOut c = *sl.hc();
    LYAP_REQUIRE(std::isfinite(c.res), LYAP_E_NUMERIC, "residual is not finite at m=%d", mm);
    const double rel = c.res / b12;
    hm.push_back(mm);
    hr.push_back(rel);
    last_res = rel;
    lam_abs = std::max(std::fabs(sl.hl()[0]), std::fabs(sl.hl()[1]));
    if (o.verbose) std::fprintf(stderr, "[sylv-small-b] m=%d k=%d res=%.3e\n", mm, mm * S, rel);
    LYAP_REQUIRE(c.lam_max < 0.0, LYAP_E_INDEFINITE,
                 "Ritz value %.3e >= 0 at m=%d: A is not negative definite", c.lam_max, mm);
    return rel;
  };
  auto finish_check = [&](Alg5Slot& sl) -> bool {
    done_slot = &sl;
    out->n_checks++;
    const int mm = sl.mm;
    const int fbk = sl.hf()[0], fnf = sl.hf()[1];
    const bool bk = fbk > 0 && fbk <= mm;
    // non-finite values that follow a breakdown belong to the breakdown
    LYAP_REQUIRE(!(fnf > 0 && fnf <= mm && (!bk || fnf <= fbk)), LYAP_E_NUMERIC,
                 "non-finite values in the Lanczos recurrence at step %d", fnf);
    if (bk) {  // a rank-deficient block: check the basis it ends instead
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
      Alg5Slot& sl = *slots[head];
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
    LYAP_HIP(hipEventRecord(er.ev[steps % kAhead], st));
    ++steps;
  }
  if (overlap) LYAP_HIP(hipStreamWaitEvent(st, done_slot->ev, 0));
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
  const int k = m * S;
  std::vector<double> tau_h(S * S);
  LYAP_HIP(hipMemcpyAsync(tau_h.data(), sa.tau_dev(m), S * S * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  double tau_f = 0.0;
  for (double x : tau_h) tau_f += x * x;
  // ||R(Y) - R(Y + dY)||_F <= (||T_m underline||_2 + ||B||_2) ||dY||_F
  const double nu = lam_abs + std::sqrt(tau_f) + ups_abs;
  double eps = o.trunc_eps;
  if (!(eps >= 0.0)) eps = std::min(1e-12, 0.05 * o.tol / nu) * b12;
  out->trunc_eps = eps;
  kt.mark(LYAP_K_FINAL);
  // Y1 = Q Y~ (k x n2 column-major) by shifted solves, in column chunks that
  // bound the factor scratch to about 256 MB
  DevBuf Y1((size_t)k * n2 * sizeof(double)), piv((size_t)n2 * sizeof(int)), fail(4 * sizeof(int));
  LYAP_HIP(hipMemsetAsync(fail.p, 0, 4 * sizeof(int), st));
  hipLaunchKernelGGL(k_iota, dim3((n2 + 255) / 256), dim3(256), 0, st, piv.as<int>(), n2);
  const size_t per_col = (size_t)(S + 1) * k * sizeof(double);
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)n2, ((size_t)256 << 20) / per_col));
  {
    DevBuf Lb(per_col * chunk);
    for (int c0 = 0; c0 < n2; c0 += chunk) {
      const int cn = std::min(chunk, n2 - c0);
      launch_shift_solve(sa.band(), S + 1, S, k, ups.as<double>(), H.as<double>(), sa.gamma_dev(),
                         piv.as<int>() + c0, cn, Lb.as<double>(), Y1.as<double>() + (size_t)c0 * k, fail.as<int>(),
                         st);
    }
    LYAP_HIP(hipStreamSynchronize(st));
  }
  int hfail = 0;
  LYAP_HIP(hipMemcpy(&hfail, fail.p, sizeof(int), hipMemcpyDeviceToHost));
  LYAP_REQUIRE(hfail == 0, LYAP_E_INDEFINITE, "shifted operator -(T_m + upsilon I) not positive definite");
  // cross approximation of E0 = Y1^T (n2 x k row-major: the same memory)
  const int tmax = std::min(std::min(n2, k), 1024);
  DevBuf E((size_t)k * n2 * sizeof(double)), I, J;
  LYAP_HIP(hipMemcpyAsync(E.p, Y1.p, (size_t)k * n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  const int t = aca_cross(E.as<double>(), n2, k, eps, tmax, I, J, st);
  DevBuf M1(8), N(8);
  if (t > 0) {
    DevBuf B1((size_t)t * t * sizeof(double)), B2((size_t)t * t * sizeof(double));
    core_lu_explicit(Y1.as<double>(), k, I.as<int>(), J.as<int>(), t, B1.as<double>(), B2.as<double>(), st);
    // E0 ~= [E0(:, J) U^{-1}] [L^{-1} E0(I, :)], so Y1 = E0^T ~= M1 N^T with
    // M1 = Y1(:, I) L^{-T} (k x t) and N = Y1(J, :)^T U^{-1} (n2 x t)
    DevBuf X1((size_t)k * t * sizeof(double)), X2((size_t)n2 * t * sizeof(double));
    hipLaunchKernelGGL(k_gather_cols, dim3(grid_for_elems((int64_t)k * t)), dim3(256), 0, st, Y1.as<double>(), k,
                       I.as<int>(), t, X1.as<double>());
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for_elems((int64_t)n2 * t)), dim3(256), 0, st, Y1.as<double>(), k,
                       n2, J.as<int>(), t, X2.as<double>());
    LYAP_LAUNCHED("gather");
    M1.alloc((size_t)k * t * sizeof(double));
    N.alloc((size_t)n2 * t * sizeof(double));
    launch_gemm_xb(X1.as<double>(), k, t, B2.as<double>(), t, M1.as<double>(), st);
    launch_gemm_xb(X2.as<double>(), n2, t, B1.as<double>(), t, N.as<double>(), st);
    LYAP_HIP(hipStreamSynchronize(st));
  }
  kt.collect();
  out->t = t;
  const double fin_ms = ms_since(t_fin);

  // ---- Z1 (second pass or stored basis), Z2 = P N
  const auto t_p2 = Clock::now();
  lyap_opts oz = o;
  bool own1 = false, own2 = false;
  out->Z1 = alloc_output(oz, (size_t)n1 * std::max(t, 1) * sizeof(double), &own1);
  out->Z2 = alloc_output(oz, (size_t)n2 * std::max(t, 1) * sizeof(double), &own2);
  out->owns_Z = own1 ? 1 : 0;
  double zbytes = 0.0;
  if (t > 0) {
    sa.accumulate_Z(m, M1.as<double>(), t, out->Z1, n1, &zbytes);
    hipLaunchKernelGGL(k_pn, dim3(grid_for_elems((int64_t)n2 * t)), dim3(256), 0, st, P.as<double>(), n2,
                       (int64_t)n2, N.as<double>(), t, out->Z2, (int64_t)n2);
    LYAP_LAUNCHED("k_pn");
  }
  LYAP_HIP(hipStreamSynchronize(st));
  kt.collect();
  const double p2_ms = ms_since(t_p2);

  if (o.want_T) {
    double* hbnd = (double*)std::malloc((size_t)(S + 1) * k * sizeof(double));
    LYAP_HIP(hipMemcpy(hbnd, sa.band(), (size_t)(S + 1) * k * sizeof(double), hipMemcpyDeviceToHost));
    for (int c = 0; c < k; ++c)
      for (int d = 0; d <= S; ++d)
        if (c + d >= k) hbnd[(size_t)c * (S + 1) + d] = 0.0;
    out->T_band = hbnd;
    out->gamma1 = (double*)std::malloc(S * S * sizeof(double));
    rowmajor_to_colmajor(sa.gamma_host(), S, S, out->gamma1);
    out->tau = (double*)std::malloc(S * S * sizeof(double));
    rowmajor_to_colmajor(tau_h.data(), S, S, out->tau);
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
  fill_kernel_bytes<T>(n1, S, sa.op().coef_bytes_per_row(), kt, zbytes, out->kern_bytes);
  out->status = status;
  return status;
}

}  // namespace
}  // namespace lyap

extern "C" lyap_status lyap_sym_eig(const double* B, int64_t n, int64_t ldb, double* w, double* P, int64_t ldp,
                                    void* stream, int32_t* sweeps) {
  using namespace lyap;
  clear_error();
  try {
    LYAP_REQUIRE(B != nullptr && w != nullptr && P != nullptr, LYAP_E_ARG, "B, w or P is NULL");
    LYAP_REQUIRE(n >= 1 && n <= kSymEigMax, LYAP_E_ARG, "n=%lld out of range 1..%d", (long long)n, kSymEigMax);
    LYAP_REQUIRE(ldb >= n && ldp >= n, LYAP_E_ARG, "leading dimension below n");
    const int sw = sym_eig(B, (int)n, ldb, w, P, ldp, (hipStream_t)stream);
    if (sweeps) *sweeps = sw;
    return LYAP_OK;
  } catch (const Error& e) {
    return e.st;
  }
}

extern "C" lyap_status sylv_solve_small_b(const lyap_op* A, const double* B, int64_t n2, int64_t ldb,
                                          const double* C1, int64_t ldc1, const double* C2, int64_t ldc2, int32_t s,
                                          const lyap_opts* opts, sylv_result* out) {
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
    LYAP_REQUIRE(B != nullptr && C1 != nullptr && C2 != nullptr, LYAP_E_ARG, "B, C1 or C2 is NULL");
    LYAP_REQUIRE(n2 >= 1 && n2 <= kSymEigMax, LYAP_E_ARG, "n2=%lld out of range 1..%d", (long long)n2, kSymEigMax);
    LYAP_REQUIRE(ldb >= n2, LYAP_E_ARG, "ldb below n2");
    LYAP_REQUIRE(s >= 1 && s <= kSmallBMaxEll, LYAP_E_ARG, "s=%d out of range 1..%d", s, kSmallBMaxEll);
    LYAP_REQUIRE(ldc1 >= A->n && ldc2 >= n2, LYAP_E_ARG, "leading dimension below n");
    LYAP_REQUIRE(s <= A->n, LYAP_E_ARG, "s > n1");
    LYAP_REQUIRE(o.tol > 0.0 && o.tol < 1.0, LYAP_E_ARG, "tol=%g must be in (0,1)", o.tol);
    LYAP_REQUIRE(o.max_iter >= 1 && (int64_t)o.max_iter * s <= (int64_t)1 << 20, LYAP_E_ARG,
                 "max_iter=%d out of range", o.max_iter);
    LYAP_REQUIRE(o.check_every >= 0, LYAP_E_ARG, "check_every must be >= 0");
    LYAP_REQUIRE(o.method == LYAP_METHOD_STD, LYAP_E_UNSUPPORTED,
                 "sylv_solve_small_b builds a standard Krylov space (method must be LYAP_METHOD_STD)");
    LYAP_REQUIRE(o.storage == LYAP_STORE_F64 || o.storage == LYAP_STORE_F32, LYAP_E_ARG, "unknown storage %d",
                 o.storage);
    lyap_status st =
        o.storage == LYAP_STORE_F64
            ? smallb_impl<double>(A, B, (int)n2, ldb, C1, ldc1, C2, ldc2, s, o, out)
            : smallb_impl<float>(A, B, (int)n2, ldb, C1, ldc1, C2, ldc2, s, o, out);
    out->status = st;
    return st;
  } catch (const Error& e) {
    out->status = e.st;
    return e.st;
  }
}
