// FP64 kernels for the residual check (Proposition 1 / Algorithm 3) and the
// finalisation (truncation of Y~ and Q Y-check), all on the GPU.
//
//  - k_jacobi: cyclic Jacobi eigensolver for a dense symmetric matrix, one
//    workgroup per matrix, parallel (round-robin) rotation order.  Used for
//    the divide-and-conquer leaves, for small T_m, and for the t' x t' Gram
//    matrix of the truncation.
//  - k_gw: g = (E_1^T Q)^T gamma and W_m = (E_m^T Q)^T tau^T from the first and
//    last ell rows of the eigenvector matrix.
//  - k_ctri_sum: ||R||_F^2 = 2 sum_i || e_i^T S D_i^{-1} W_m ||^2 with
//    S = g g^T never formed: entry (i,j) of S D_i^{-1} is (g_i . g_j)/(lambda_i+lambda_j).
//  - finalisation: pivoted Cholesky of Y~ (entries generated on the fly from
//    lambda and g), the Gram matrix of its factor, banded shifted solves that
//    give Q Y~(:,p) = -(T + lambda_p I)^{-1} E_1 gamma g_p^T without forming Q,
//    and the small triangular/GEMM steps that assemble M = Q Y-check.
#include "eig.hpp"

namespace lyap {

// ------------------------------------------------------------------ band -> dense
__global__ void k_band_to_dense(const double* band, int ldb, int ell, int k, double* A) {
  const int64_t tot = (int64_t)k * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    const int d = i > j ? i - j : j - i;
    const int c = i > j ? j : i;
    A[e] = d <= ell ? band[(size_t)c * ldb + d] : 0.0;
  }
}

// ------------------------------------------------------------------ Jacobi
// Matrix b of the batch: A + b*strideA (n x n, row-major, lda = n), eigenvector
// matrix Q + b*strideQ (row-major, eigenvector i in column i), eigenvalues
// lam + b*strideL, ascending.  On exit A is destroyed.
constexpr int kJacThreads = 256;
constexpr int kJacMaxN = 1024;

__global__ __launch_bounds__(kJacThreads) void k_jacobi(double* Aall, int64_t strideA, double* Qall, int64_t strideQ,
                                                       double* lamall, int64_t strideL, const int* nlist, int nfixed,
                                                       int max_sweeps) {
  const int bidx = blockIdx.x;
  const int n = nlist ? nlist[bidx] : nfixed;
  double* A = Aall + bidx * strideA;
  double* Q = Qall + bidx * strideQ;
  double* lam = lamall + bidx * strideL;
  __shared__ int sp[kJacMaxN / 2 + 1], sq[kJacMaxN / 2 + 1];
  __shared__ double sc[kJacMaxN / 2 + 1], ss[kJacMaxN / 2 + 1];
  __shared__ double red[2 * kWaves * 4];
  __shared__ int done;
  if (n <= 0) return;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) Q[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  if (n == 1) {
    if (threadIdx.x == 0) lam[0] = A[0];
    return;
  }
  const int np = (n + 1) & ~1;  // players (one dummy when n is odd)
  const int rot = np - 1;       // rotating players
  const int half = np / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence test: off-diagonal vs diagonal mass
    double off = 0.0, dia = 0.0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const double v = A[e];
      if (e / n == e % n) dia += v * v; else off += v * v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    off = wave_sum(off);
    dia = wave_sum(dia);
    if (lane == 0) { red[wave] = off; red[kWaves + wave] = dia; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double o = 0, d = 0;
      for (int w = 0; w < kJacThreads / 64; ++w) { o += red[w]; d += red[kWaves + w]; }
      done = (o <= 1e-30 * d) || (o == 0.0);
    }
    __syncthreads();
    if (done) break;
    for (int round = 0; round < rot; ++round) {
      for (int kp = threadIdx.x; kp < half; kp += blockDim.x) {
        int p, q;
        if (kp == 0) { p = 0; q = 1 + round; }
        else { p = 1 + (round + kp) % rot; q = 1 + (round - kp + rot) % rot; }
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          const double app = A[p * n + p], aqq = A[q * n + q];
          if (fabs(apq) > 1e-17 * (fabs(app) + fabs(aqq)) && fabs(apq) > 1e-300) {
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        sp[kp] = p; sq[kp] = q; sc[kp] = c; ss[kp] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = threadIdx.x; e < half * n; e += blockDim.x) {
        const int kp = e / n, col = e % n;
        const int p = sp[kp], q = sq[kp];
        if (q >= n || ss[kp] == 0.0) continue;
        const double c = sc[kp], s = ss[kp];
        const double ap = A[p * n + col], aq = A[q * n + col];
        A[p * n + col] = c * ap - s * aq;
        A[q * n + col] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, Q <- Q J
      for (int e = threadIdx.x; e < half * n; e += blockDim.x) {
        const int kp = e / n, row = e % n;
        const int p = sp[kp], q = sq[kp];
        if (q >= n || ss[kp] == 0.0) continue;
        const double c = sc[kp], s = ss[kp];
        const double ap = A[row * n + p], aq = A[row * n + q];
        A[row * n + p] = c * ap - s * aq;
        A[row * n + q] = s * ap + c * aq;
        const double qp = Q[row * n + p], qq = Q[row * n + q];
        Q[row * n + p] = c * qp - s * qq;
        Q[row * n + q] = s * qp + c * qq;
      }
      __syncthreads();
    }
  }
  // sort ascending: rank of each eigenvalue, then permute Q columns through A
  for (int i = threadIdx.x; i < n; i += blockDim.x) lam[i] = A[i * n + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double li = lam[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = lam[j];
      rank += (lj < li) || (lj == li && j < i);
    }
    for (int r = 0; r < n; ++r) A[r * n + rank] = Q[r * n + i];  // A reused as scratch
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) Q[e] = A[e];
  __syncthreads();
  // eigenvalues in sorted order (recomputed from the stored diagonal ranks)
  if (threadIdx.x == 0) {
    // simple insertion sort of lam (n <= kJacMaxN, once)
    for (int i = 1; i < n; ++i) {
      double v = lam[i];
      int j = i - 1;
      while (j >= 0 && lam[j] > v) { lam[j + 1] = lam[j]; --j; }
      lam[j + 1] = v;
    }
  }
}

// ------------------------------------------------------------------ g and W_m
// F, L: ell x k row-major (first / last ell rows of Q).  gamma: ell x ell,
// tau: nt x ell (row-major).  g: k x ell, Wm: k x nt (row-major).
__global__ void k_gw(const double* F, int64_t ldf, const double* L, int64_t ldl, int k, int ell, int nt,
                     const double* gamma, const double* tau, double* g, double* Wm) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    for (int c = 0; c < ell; ++c) {
      double acc = 0.0;
      for (int a = 0; a < ell; ++a) acc = fma(F[a * ldf + i], gamma[a * ell + c], acc);
      g[(size_t)i * ell + c] = acc;
    }
    for (int c = 0; c < nt; ++c) {
      double acc = 0.0;
      for (int a = 0; a < ell; ++a) acc = fma(L[a * ldl + i], tau[c * ell + a], acc);
      Wm[(size_t)i * nt + c] = acc;
    }
  }
}

// ------------------------------------------------------------------ Algorithm 3 sum
constexpr int kMaxEll = 16;

__global__ __launch_bounds__(kBlock) void k_ctri_sum(const double* lam, const double* g, const double* Wm, int k,
                                                     int ell, int nt, double* part, unsigned* counter,
                                                     CheckOut* out) {
  __shared__ double red[kMaxEll * kWaves];
  double blocksum = 0.0;
  for (int i = blockIdx.x; i < k; i += gridDim.x) {
    double gi[kMaxEll];
#pragma unroll
    for (int a = 0; a < kMaxEll; ++a) gi[a] = a < ell ? g[(size_t)i * ell + a] : 0.0;
    const double li = lam[i];
    double acc[kMaxEll];
#pragma unroll
    for (int c = 0; c < kMaxEll; ++c) acc[c] = 0.0;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
      double dot = 0.0;
#pragma unroll
      for (int a = 0; a < kMaxEll; ++a)
        if (a < ell) dot = fma(gi[a], g[(size_t)j * ell + a], dot);
      const double coef = dot / (li + lam[j]);
#pragma unroll
      for (int c = 0; c < kMaxEll; ++c)
        if (c < nt) acc[c] = fma(coef, Wm[(size_t)j * nt + c], acc[c]);
    }
    block_sum<kMaxEll>(acc, red);
    double v = 0.0;
    for (int c = 0; c < nt; ++c) v += red[c] * red[c];
    blocksum += v;  // identical in every thread
    __syncthreads();
  }
  double tot[1] = {threadIdx.x == 0 ? blocksum : 0.0};
  __shared__ double red1[kWaves];
  if (grid_sum_last<1>(tot, red1, part, counter)) {
    if (threadIdx.x == 0) {
      out->res = sqrt(2.0 * red1[0]);
      double lmax = lam[k - 1];
      out->lam_max = lmax;
      out->lam_min = lam[0];
    }
  }
}

// ------------------------------------------------------------------ pivoted Cholesky of Y~
// One workgroup.  Y~_ij = -(g_i . g_j)/(lambda_i + lambda_j).  Stops when the
// trace of the Schur complement is <= delta or tmax columns are formed.
constexpr int kPcThreads = 1024;

__global__ __launch_bounds__(kPcThreads) void k_pchol(const double* lam, const double* g, int k, int ell, double delta,
                                                      int tmax, double* d, double* Lc, int* piv, int* tout) {
  __shared__ double rv[kPcThreads / 64];
  __shared__ int ri[kPcThreads / 64];
  __shared__ double rsum[kPcThreads / 64];
  __shared__ int sp;
  __shared__ double spiv, strace;
  __shared__ double gp[kMaxEll];
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    double nn = 0.0;
    for (int a = 0; a < ell; ++a) nn = fma(g[(size_t)i * ell + a], g[(size_t)i * ell + a], nn);
    d[i] = -nn / (2.0 * lam[i]);
  }
  __syncthreads();
  int r = 0;
  for (; r < tmax; ++r) {
    // argmax and trace
    double best = -1.0, sum = 0.0;
    int bi = 0x7fffffff;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
      const double v = d[i];
      sum += v;
      if (v > best || (v == best && i < bi)) { best = v; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      sum += __shfl_xor(sum, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { rv[wave] = best; ri[wave] = bi; rsum[wave] = sum; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = rv[0]; int ii = ri[0]; double s = rsum[0];
      for (int w = 1; w < kPcThreads / 64; ++w) {
        if (rv[w] > b || (rv[w] == b && ri[w] < ii)) { b = rv[w]; ii = ri[w]; }
        s += rsum[w];
      }
      sp = ii; spiv = b; strace = s;
    }
    __syncthreads();
    if (!(strace > delta) || !(spiv > 0.0)) break;
    const int p = sp;
    const double sq = sqrt(spiv);
    if (threadIdx.x < ell) gp[threadIdx.x] = g[(size_t)p * ell + threadIdx.x];
    __syncthreads();
    const double lp = lam[p];
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
      double v;
      if (i == p) {
        v = sq;
      } else if (d[i] == 0.0) {
        v = 0.0;  // an earlier pivot (or an exactly represented row)
      } else {
        double dot = 0.0;
        for (int a = 0; a < ell; ++a) dot = fma(g[(size_t)i * ell + a], gp[a], dot);
        double y = -dot / (lam[i] + lp);
        for (int q = 0; q < r; ++q) y = fma(-Lc[(size_t)q * k + i], Lc[(size_t)q * k + p], y);
        v = y / sq;
      }
      Lc[(size_t)r * k + i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
      const double v = Lc[(size_t)r * k + i];
      double nd = (i == p) ? 0.0 : d[i] - v * v;
      d[i] = nd > 0.0 ? nd : 0.0;
    }
    if (threadIdx.x == 0) piv[r] = p;
    __syncthreads();
  }
  if (threadIdx.x == 0) *tout = r;
}

// G = Lc^T Lc (tp x tp, row-major); one workgroup per entry (a <= b).
__global__ __launch_bounds__(kBlock) void k_gram_cols(const double* Lc, int k, int tp, double* G) {
  __shared__ double red[kWaves];
  const int64_t npair = (int64_t)tp * (tp + 1) / 2;
  for (int64_t e = blockIdx.x; e < npair; e += gridDim.x) {
    // unrank e -> (a, b) with a <= b
    int a = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) / 2.0);
    while ((int64_t)(a + 1) * (a + 2) / 2 <= e) ++a;
    while ((int64_t)a * (a + 1) / 2 > e) --a;
    const int b = (int)(e - (int64_t)a * (a + 1) / 2);  // b <= a
    double acc[1] = {0.0};
    for (int i = threadIdx.x; i < k; i += blockDim.x) acc[0] = fma(Lc[(size_t)a * k + i], Lc[(size_t)b * k + i], acc[0]);
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) { G[(size_t)a * tp + b] = red[0]; G[(size_t)b * tp + a] = red[0]; }
    __syncthreads();
  }
}

// Banded shifted solves: thread p builds chol(-(T + lambda_{piv[p]} I)) (lower
// band, bandwidth ell) and solves for b = E_1 (gamma g_{piv[p]}^T).
// X: k x tp column-major.  Lb scratch: ((ell+1)*k) x tp, interleaved by thread.
__global__ void k_shift_solve(const double* band, int ldb, int ell, int k, const double* lam, const double* g,
                              const double* gamma, const int* piv, int tp, double* Lb, double* X, int* fail) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= tp) return;
  const int ip = piv[p];
  const double sh = lam[ip];
  const int lb = ell + 1;
#define LB(j, dd) Lb[((size_t)(j) * lb + (dd)) * tp + p]
  // factor: L(j+d, j) stored at LB(j, d)
  for (int j = 0; j < k; ++j) {
    // diagonal
    double djj = -(band[(size_t)j * ldb + 0] + sh);
    const int i0 = j - ell > 0 ? j - ell : 0;
    for (int i = i0; i < j; ++i) {
      const double lji = LB(i, j - i);
      djj -= lji * lji;
    }
    if (!(djj > 0.0)) { fail[0] = 1; djj = 1e-300; }
    const double ljj = sqrt(djj);
    LB(j, 0) = ljj;
    const int rmax = j + ell < k - 1 ? j + ell : k - 1;
    for (int r = j + 1; r <= rmax; ++r) {
      double v = -band[(size_t)j * ldb + (r - j)];
      const int i1 = r - ell > 0 ? r - ell : 0;
      for (int i = i1; i < j; ++i) v -= LB(i, r - i) * LB(i, j - i);
      LB(j, r - j) = v / ljj;
    }
  }
  // rhs
  double* x = X + (size_t)p * k;
  for (int i = 0; i < k; ++i) x[i] = 0.0;
  for (int a = 0; a < ell && a < k; ++a) {
    double acc = 0.0;
    for (int c = 0; c < ell; ++c) acc = fma(gamma[a * ell + c], g[(size_t)ip * ell + c], acc);
    x[a] = acc;
  }
  // forward L z = b
  for (int j = 0; j < k; ++j) {
    double v = x[j];
    const int i0 = j - ell > 0 ? j - ell : 0;
    for (int i = i0; i < j; ++i) v -= LB(i, j - i) * x[i];
    x[j] = v / LB(j, 0);
  }
  // backward L^T x = z
  for (int j = k - 1; j >= 0; --j) {
    double v = x[j];
    const int rmax = j + ell < k - 1 ? j + ell : k - 1;
    for (int r = j + 1; r <= rmax; ++r) v -= LB(j, r - j) * x[r];
    x[j] = v / LB(j, 0);
  }
#undef LB
}

// B = L_PP^{-T} V1: L_PP[a][b] = Lc[b*k + piv[a]] (lower triangular);
// V1 given as tp x t row-major.  One thread per column.
__global__ void k_trsm_lt(const double* Lc, int k, const int* piv, int tp, const double* V1, int t, double* B) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= t) return;
  for (int a = tp - 1; a >= 0; --a) {
    double v = V1[(size_t)a * t + c];
    for (int b = a + 1; b < tp; ++b) v -= Lc[(size_t)a * k + piv[b]] * B[(size_t)b * t + c];
    B[(size_t)a * t + c] = v / Lc[(size_t)a * k + piv[a]];
  }
}

// M (k x t, row-major) = X (k x tp, column-major) B (tp x t, row-major)
__global__ void k_gemm_xb(const double* X, int k, int tp, const double* B, int t, double* M) {
  const int64_t tot = (int64_t)k * t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / t), c = (int)(e % t);
    double acc = 0.0;
    for (int p = 0; p < tp; ++p) acc = fma(X[(size_t)p * k + i], B[(size_t)p * t + c], acc);
    M[e] = acc;
  }
}

// V1 (tp x t row-major) = top-t eigenvectors of the ascending Jacobi output
// Qg (tp x tp row-major, eigenvector i in column i), largest first.
__global__ void k_pick_top(const double* Qg, int tp, int t, double* V1) {
  const int64_t tot = (int64_t)tp * t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / t), c = (int)(e % t);
    V1[e] = Qg[(size_t)a * tp + (tp - 1 - c)];
  }
}

// ------------------------------------------------------------------ launchers
void launch_band_to_dense(const double* band, int ldb, int ell, int k, double* A, hipStream_t st) {
  int64_t tot = (int64_t)k * k;
  int grid = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_band_to_dense, dim3(grid), dim3(256), 0, st, band, ldb, ell, k, A);
  LYAP_LAUNCHED("band_to_dense");
}

void launch_jacobi(double* A, int64_t strideA, double* Q, int64_t strideQ, double* lam, int64_t strideL,
                   const int* nlist, int nfixed, int batch, hipStream_t st) {
  LYAP_REQUIRE(nfixed <= kJacMaxN, LYAP_E_UNSUPPORTED, "dense eigensolver limited to n <= %d (got %d)", kJacMaxN,
               nfixed);
  hipLaunchKernelGGL(k_jacobi, dim3(batch), dim3(kJacThreads), 0, st, A, strideA, Q, strideQ, lam, strideL, nlist,
                     nfixed, 40);
  LYAP_LAUNCHED("jacobi");
}

void launch_gw(const double* F, int64_t ldf, const double* L, int64_t ldl, int k, int ell, int nt,
               const double* gamma, const double* tau, double* g, double* Wm, hipStream_t st) {
  int grid = std::max(1, std::min((k + 255) / 256, 1024));
  hipLaunchKernelGGL(k_gw, dim3(grid), dim3(256), 0, st, F, ldf, L, ldl, k, ell, nt, gamma, tau, g, Wm);
  LYAP_LAUNCHED("gw");
}

void launch_ctri_sum(const double* lam, const double* g, const double* Wm, int k, int ell, int nt, double* part,
                     unsigned* counter, CheckOut* out, hipStream_t st) {
  LYAP_REQUIRE(ell <= kMaxEll && nt <= kMaxEll, LYAP_E_UNSUPPORTED, "block size %d > %d", ell, kMaxEll);
  int grid = std::max(1, std::min(k, 2048));
  hipLaunchKernelGGL(k_ctri_sum, dim3(grid), dim3(kBlock), 0, st, lam, g, Wm, k, ell, nt, part, counter, out);
  LYAP_LAUNCHED("ctri_sum");
}

void launch_pchol(const double* lam, const double* g, int k, int ell, double delta, int tmax, double* d, double* Lc,
                  int* piv, int* tout, hipStream_t st) {
  hipLaunchKernelGGL(k_pchol, dim3(1), dim3(kPcThreads), 0, st, lam, g, k, ell, delta, tmax, d, Lc, piv, tout);
  LYAP_LAUNCHED("pchol");
}

void launch_gram_cols(const double* Lc, int k, int tp, double* G, hipStream_t st) {
  int64_t npair = (int64_t)tp * (tp + 1) / 2;
  int grid = (int)std::max<int64_t>(1, std::min<int64_t>(npair, 8192));
  hipLaunchKernelGGL(k_gram_cols, dim3(grid), dim3(kBlock), 0, st, Lc, k, tp, G);
  LYAP_LAUNCHED("gram_cols");
}

void launch_shift_solve(const double* band, int ldb, int ell, int k, const double* lam, const double* g,
                        const double* gamma, const int* piv, int tp, double* Lb, double* X, int* fail,
                        hipStream_t st) {
  int grid = (tp + 63) / 64;
  hipLaunchKernelGGL(k_shift_solve, dim3(grid), dim3(64), 0, st, band, ldb, ell, k, lam, g, gamma, piv, tp, Lb, X,
                     fail);
  LYAP_LAUNCHED("shift_solve");
}

void launch_assemble_M(const double* Lc, int k, const int* piv, int tp, const double* Qg, int t, const double* X,
                       double* V1, double* B, double* M, hipStream_t st) {
  int64_t tot = (int64_t)tp * t;
  int grid = (int)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 4096));
  hipLaunchKernelGGL(k_pick_top, dim3(grid), dim3(256), 0, st, Qg, tp, t, V1);
  hipLaunchKernelGGL(k_trsm_lt, dim3((t + 63) / 64), dim3(64), 0, st, Lc, k, piv, tp, V1, t, B);
  tot = (int64_t)k * t;
  grid = (int)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 8192));
  hipLaunchKernelGGL(k_gemm_xb, dim3(grid), dim3(256), 0, st, X, k, tp, B, t, M);
  LYAP_LAUNCHED("assemble_M");
}

}  // namespace lyap
