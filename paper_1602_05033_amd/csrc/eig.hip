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
#include <cstring>
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
// The same sweeps for n <= NN <= 32 with every lane of the wave busy: after
// the round's rotations are chosen, each index i carries (alpha_i, beta_i,
// partner i') with row i of J^T A = alpha_i row i + beta_i row i' (c and -s
// for the first of a pair, c and s for the second, 1 and 0 when not rotated),
// and the lanes form every entry of J^T A J at once from the four entries it
// depends on, into a second buffer (then the exact values of the rotated
// pairs), and every pair of Q's columns row by row.  Two barriers per round;
// the previous form had 16 lanes working through the rotations one after
// another in three phases.  Returns the sweeps; the result is in *Aout.
template <int NN>
__device__ int jacobi_core_wave(double* A, double* B, double* Q, int n, int max_sweeps, double** Aout) {
  static_assert(NN <= 32, "one wave, LDS double buffer");
  __shared__ double sal[NN], sbe[NN], sdn[NN];
  __shared__ int spa[NN], srot[NN];
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < n * n; e += 64) {
    const int r = e / n;
    Q[e] = (r == e - r * n) ? 1.0 : 0.0;
  }
  __syncthreads();
  *Aout = A;
  if (n == 1) return 0;
  const int np = (n + 1) & ~1;
  const int rot = np - 1;
  const int half = np / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    int nrot = 0;
    for (int round = 0; round < rot; ++round) {
      bool rotated = false;
      if (lane < half) {
        const int kp = lane;
        int p, q;
        if (kp == 0) { p = 0; q = 1 + round; }
        else {
          p = round + kp; if (p >= rot) p -= rot; p += 1;
          q = round - kp; if (q < 0) q += rot; q += 1;
        }
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, sn = 0.0, dp = 0.0, dq = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          const double app = A[p * n + p], aqq = A[q * n + q];
          if (fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(app) * fabs(aqq)) && fabs(apq) > 1e-300) {
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
            dp = app - t * apq;
            dq = aqq + t * apq;
            rotated = true;
          }
        }
        sal[p] = c; sbe[p] = -sn; spa[p] = rotated ? q : p; srot[p] = rotated; sdn[p] = dp;
        if (q < n) { sal[q] = c; sbe[q] = sn; spa[q] = rotated ? p : q; srot[q] = rotated; sdn[q] = dq; }
      }
      nrot += __popcll(__ballot(rotated));
      __syncthreads();
      for (int e = lane; e < n * n; e += 64) {
        const int i = e / n, j = e - i * n;
        const int pi = spa[i], pj = spa[j];
        double v;
        if (srot[i] && j == pi) {
          v = 0.0;  // the rotated pair's off-diagonal entry, set exactly
        } else if (srot[i] && i == j) {
          v = sdn[i];
        } else {
          const double ai = sal[i], bi = sbe[i], aj = sal[j], bj = sbe[j];
          const double r0 = ai * A[i * n + j] + bi * A[pi * n + j];    // row update at column j
          const double r1 = ai * A[i * n + pj] + bi * A[pi * n + pj];  // and at column j'
          v = aj * r0 + bj * r1;
        }
        B[e] = v;
      }
      for (int e = lane; e < n * half; e += 64) {  // Q <- Q J, a pair of columns per item
        const int row = e / half, kp = e - row * half;
        int p, q;
        if (kp == 0) { p = 0; q = 1 + round; }
        else {
          p = round + kp; if (p >= rot) p -= rot; p += 1;
          q = round - kp; if (q < 0) q += rot; q += 1;
        }
        if (p > q) { int t = p; p = q; q = t; }
        if (q >= n || !srot[p]) continue;
        const double c = sal[p], sn = sbe[q];
        const double qp = Q[row * n + p], qv = Q[row * n + q];
        Q[row * n + p] = c * qp - sn * qv;
        Q[row * n + q] = sn * qp + c * qv;
      }
      __syncthreads();
      double* t = A; A = B; B = t;
    }
    if (nrot == 0) { *Aout = A; return sweep + 1; }
  }
  *Aout = A;
  return max_sweeps;
}

// Matrix b of the batch: A + b*strideA (n x n, row-major, lda = n), eigenvector
// matrix Q + b*strideQ (row-major, eigenvector i in column i), eigenvalues
// lam + b*strideL, ascending.  On exit A is destroyed.
constexpr int kJacThreads = 256;
constexpr int kJacMaxN = 1024;
constexpr int kJacLds = 64;  // matrices up to this size are worked on in LDS

// One sweep rotates every pair with |a_pq| > eps*sqrt(|a_pp a_qq|); after the
// row/column updates the rotated pair is set exactly (a_pq = 0,
// a_pp - t a_pq, a_qq + t a_pq), so rounding does not re-create the entry just
// annihilated and the loop ends after a sweep that rotates nothing.
// NN > 0: the matrix (n <= NN <= 64) lives in LDS and each thread owns column
// (or row) threadIdx.x % 64 of the updates; NN == 0: global memory, any n.
template <int NN>
__device__ int jacobi_core(double* A, double* Q, int n, int max_sweeps, int* sp, int* sq, double* sc, double* ss,
                           double* st_, int* nrot) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n;
    Q[e] = (r == e - r * n) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (n == 1) return 0;
  const int np = (n + 1) & ~1;  // players (one dummy when n is odd)
  const int rot = np - 1;       // rotating players
  const int half = np / 2;
  const int lane = threadIdx.x & 63;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) *nrot = 0;
    __syncthreads();
    for (int round = 0; round < rot; ++round) {
      for (int kp = threadIdx.x; kp < half; kp += blockDim.x) {
        int p, q;
        if (kp == 0) { p = 0; q = 1 + round; }
        else {
          p = round + kp; if (p >= rot) p -= rot; p += 1;
          q = round - kp; if (q < 0) q += rot; q += 1;
        }
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          const double app = A[p * n + p], aqq = A[q * n + q];
          if (fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(app) * fabs(aqq)) && fabs(apq) > 1e-300) {
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
            st_[3 * kp + 0] = app - t * apq;
            st_[3 * kp + 1] = aqq + t * apq;
            atomicAdd(nrot, 1);
          }
        }
        sp[kp] = p; sq[kp] = q; sc[kp] = c; ss[kp] = s;
      }
      __syncthreads();
      if constexpr (NN > 0) {
        // one wave: lane owns column `lane` (row phase) then row `lane` (column phase)
        int pp[NN / 2], qq[NN / 2];
        double cc[NN / 2], sv[NN / 2];
#pragma unroll
        for (int kp = 0; kp < NN / 2; ++kp) {
          if (kp < half) { pp[kp] = sp[kp]; qq[kp] = sq[kp]; cc[kp] = sc[kp]; sv[kp] = ss[kp]; }
          else { pp[kp] = 0; qq[kp] = n; cc[kp] = 1.0; sv[kp] = 0.0; }
        }
        if (lane < n) {
#pragma unroll
          for (int kp = 0; kp < NN / 2; ++kp) {
            if (qq[kp] >= n || sv[kp] == 0.0) continue;
            const double ap = A[pp[kp] * n + lane], aq = A[qq[kp] * n + lane];
            A[pp[kp] * n + lane] = cc[kp] * ap - sv[kp] * aq;
            A[qq[kp] * n + lane] = sv[kp] * ap + cc[kp] * aq;
          }
        }
        __syncthreads();
        if (lane < n) {
#pragma unroll
          for (int kp = 0; kp < NN / 2; ++kp) {
            if (qq[kp] >= n || sv[kp] == 0.0) continue;
            const double ap = A[lane * n + pp[kp]], aq = A[lane * n + qq[kp]];
            A[lane * n + pp[kp]] = cc[kp] * ap - sv[kp] * aq;
            A[lane * n + qq[kp]] = sv[kp] * ap + cc[kp] * aq;
            const double qp = Q[lane * n + pp[kp]], qv = Q[lane * n + qq[kp]];
            Q[lane * n + pp[kp]] = cc[kp] * qp - sv[kp] * qv;
            Q[lane * n + qq[kp]] = sv[kp] * qp + cc[kp] * qv;
          }
        }
      } else {
        for (int e = threadIdx.x; e < half * n; e += blockDim.x) {  // rows: A <- J^T A
          const int kp = e / n, col = e - kp * n;
          const int p = sp[kp], q = sq[kp];
          if (q >= n || ss[kp] == 0.0) continue;
          const double c = sc[kp], s = ss[kp];
          const double ap = A[p * n + col], aq = A[q * n + col];
          A[p * n + col] = c * ap - s * aq;
          A[q * n + col] = s * ap + c * aq;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < half * n; e += blockDim.x) {  // columns: A <- A J, Q <- Q J
          const int kp = e / n, row = e - kp * n;
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
      }
      __syncthreads();
      for (int kp = threadIdx.x; kp < half; kp += blockDim.x) {
        const int p = sp[kp], q = sq[kp];
        if (q >= n || ss[kp] == 0.0) continue;
        A[p * n + q] = 0.0;
        A[q * n + p] = 0.0;
        A[p * n + p] = st_[3 * kp + 0];
        A[q * n + q] = st_[3 * kp + 1];
      }
      __syncthreads();
    }
    const int done = (*nrot == 0);
    __syncthreads();
    if (done) return sweep + 1;
  }
  return max_sweeps;
}

// Matrix b of the batch: A + b*strideA (n x n, row-major, lda = n), eigenvector
// matrix Q + b*strideQ (row-major, eigenvector i in column i), eigenvalues
// lam + b*strideL, ascending.  On exit A is destroyed.
// NN > 0: every matrix of the batch has n <= NN and is worked on in LDS by one
// wave; NN == 0: global memory, kJacThreads threads.
template <int NN>
__global__ __launch_bounds__(kJacThreads) void k_jacobi(double* Aall, int64_t strideA, double* Qall, int64_t strideQ,
                                                       double* lamall, int64_t strideL, const int* nlist, int nfixed,
                                                       int max_sweeps, int* sweeps_out) {
  constexpr int MAXN = NN > 0 ? NN : kJacMaxN;
  constexpr int LDSN = NN > 0 ? NN : 1;
  const int bidx = blockIdx.x;
  const int n = nlist ? nlist[bidx] : nfixed;
  double* Ag = Aall + bidx * strideA;
  double* Qg = Qall + bidx * strideQ;
  double* lam = lamall + bidx * strideL;
  __shared__ int sp[MAXN / 2 + 1], sq[MAXN / 2 + 1];
  __shared__ double sc[MAXN / 2 + 1], ss[MAXN / 2 + 1];
  __shared__ double As[LDSN * LDSN], Qs[LDSN * LDSN];
  __shared__ double Bs[(NN > 0 && NN <= 32) ? LDSN * LDSN : 1];
  __shared__ double stt[3 * (MAXN / 2 + 1)];
  __shared__ int nrot;
  __shared__ int rk[MAXN];
  if (n <= 0) return;
  constexpr bool lds = NN > 0;
  int nsw;
  double* Ares = As;
  if constexpr (lds) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) As[e] = Ag[e];
    __syncthreads();
    if constexpr (NN <= 32) nsw = jacobi_core_wave<NN>(As, Bs, Qs, n, max_sweeps, &Ares);
    else nsw = jacobi_core<NN>(As, Qs, n, max_sweeps, sp, sq, sc, ss, stt, &nrot);
  } else {
    nsw = jacobi_core<0>(Ag, Qg, n, max_sweeps, sp, sq, sc, ss, stt, &nrot);
  }
  if (sweeps_out && threadIdx.x == 0) sweeps_out[bidx] = nsw;
  const double* A = lds ? Ares : Ag;
  // sort ascending: rank of each eigenvalue (ties by index), permute columns
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double li = A[i * n + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j * n + j];
      rank += (lj < li) || (lj == li && j < i);
    }
    rk[i] = rank;
    lam[rank] = li;
  }
  __syncthreads();
  if (lds) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int r = e / n, i = e - r * n;
      Qg[r * n + rk[i]] = Qs[e];
    }
  } else {  // permute through A (its contents are no longer needed)
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int r = e / n, i = e - r * n;
      Ag[r * n + rk[i]] = Qg[e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) Qg[e] = Ag[e];
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
  __shared__ double red[pow2_at_least(kMaxEll) * kWaves];
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
// Y~_ij = -(g_i . g_j)/(lambda_i + lambda_j), generated on the fly.  One
// kernel per pivot: every workgroup first reduces the previous kernel's
// per-workgroup (max diagonal, index, trace) partials in a fixed order, takes
// the pivot, forms its column of the factor for its rows, updates the Schur
// diagonal and writes its own partials.  Stops (all later launches return at
// once) when the trace of the remaining Schur complement is <= delta.
constexpr int kPcThreads = 256;

struct PcState {
  int stop;    // set once the trace criterion is met
  int t;       // number of columns formed
  int pad[2];
};

__device__ __forceinline__ void pc_partials(const double* d, int k, double* pv, int* pi, double* ps) {
  __shared__ double rv[kPcThreads / 64], rs[kPcThreads / 64];
  __shared__ int ri[kPcThreads / 64];
  double best = -1.0, sum = 0.0;
  int bi = 0x7fffffff;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const double v = d[i];
    sum += v;
    if (v > best || (v == best && i < bi)) { best = v; bi = i; }
  }
  // butterfly over the wave: both lanes of a pair keep the same (value, index)
  auto merge = [&](double ob, int oi) {
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  };
  merge(lane_xor<1>(best), lane_xor<1>(bi));
  merge(lane_xor<2>(best), lane_xor<2>(bi));
  merge(lane_xor<7>(best), lane_xor<7>(bi));
  merge(lane_xor<15>(best), lane_xor<15>(bi));
  merge(lane_xor<16>(best), lane_xor<16>(bi));
  merge(lane_xor<32>(best), lane_xor<32>(bi));
  sum = wave_sum(sum);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { rv[wave] = best; ri[wave] = bi; rs[wave] = sum; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = rv[0], sm = rs[0];
    int ii = ri[0];
    for (int w = 1; w < kPcThreads / 64; ++w) {
      if (rv[w] > b || (rv[w] == b && ri[w] < ii)) { b = rv[w]; ii = ri[w]; }
      sm += rs[w];
    }
    pv[blockIdx.x] = b; pi[blockIdx.x] = ii; ps[blockIdx.x] = sm;
  }
}

__global__ __launch_bounds__(kPcThreads) void k_pchol_init(const double* lam, const double* g, int k, int ell,
                                                           double* d, double* pv, int* pi, double* ps, PcState* stt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    double nn = 0.0;
    for (int a = 0; a < ell; ++a) nn = fma(g[(size_t)i * ell + a], g[(size_t)i * ell + a], nn);
    d[i] = -nn / (2.0 * lam[i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) { stt->stop = 0; stt->t = 0; }
  // the partials below read d written by this same workgroup's threads only
  __syncthreads();
  pc_partials(d, k, pv, pi, ps);
}

__global__ __launch_bounds__(kPcThreads) void k_pchol_step(const double* lam, const double* g, int k, int ell,
                                                           double delta, int r, double* d, double* Lc, int* piv,
                                                           const double* pv_in, const int* pi_in,
                                                           const double* ps_in, int nparts, double* pv, int* pi,
                                                           double* ps, PcState* stt) {
  __shared__ int sp;
  __shared__ double spiv, strace;
  __shared__ double gp[kMaxEll];
  if (stt->stop) return;
  if (threadIdx.x == 0) {
    double b = -1.0, sm = 0.0;
    int ii = 0x7fffffff;
    for (int w = 0; w < nparts; ++w) {
      if (pv_in[w] > b || (pv_in[w] == b && pi_in[w] < ii)) { b = pv_in[w]; ii = pi_in[w]; }
      sm += ps_in[w];
    }
    sp = ii; spiv = b; strace = sm;
  }
  __syncthreads();
  if (!(strace > delta) || !(spiv > 0.0)) {
    // every workgroup sees the same totals; workgroup 0 records the stop
    if (blockIdx.x == 0 && threadIdx.x == 0) { stt->stop = 1; stt->t = r; }
    return;
  }
  const int p = sp;
  const double sq = sqrt(spiv);
  if (threadIdx.x < ell) gp[threadIdx.x] = g[(size_t)p * ell + threadIdx.x];
  __syncthreads();
  const double lp = lam[p];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    double v;
    const double di = d[i];
    if (i == p) {
      v = sq;
    } else if (di == 0.0) {
      v = 0.0;  // an earlier pivot (or a row already represented exactly)
    } else {
      double dot = 0.0;
      for (int a = 0; a < ell; ++a) dot = fma(g[(size_t)i * ell + a], gp[a], dot);
      double y = -dot / (lam[i] + lp);
      for (int q = 0; q < r; ++q) y = fma(-Lc[(size_t)q * k + i], Lc[(size_t)q * k + p], y);
      v = y / sq;
    }
    Lc[(size_t)r * k + i] = v;
    const double nd = (i == p) ? 0.0 : di - v * v;
    d[i] = nd > 0.0 ? nd : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) { piv[r] = p; stt->t = r + 1; }
  __syncthreads();
  pc_partials(d, k, pv, pi, ps);
}

// The whole factorisation in one workgroup, for k up to kPcOneMax rows: the
// pivot rule (largest remaining diagonal entry, the lowest index on ties),
// the stopping rule (remaining trace <= delta) and the column arithmetic of
// k_pchol_init / k_pchol_step, with the pivot search and the trace reduced
// inside the workgroup between pivots instead of one launch per pivot.  Each
// pivot costs a thread k / 1024 rows times r loads in sequence, so above
// about a thousand rows the one-launch-per-pivot kernels are faster (measured:
// 1.6 ms per factorisation on the 64-problem batch, k up to about 3000,
// against about 1 ms of step kernels; 22 against 14 ms at k = 5348, t = 131).
constexpr int kPcOneThreads = 1024;
constexpr int kPcOneMax = 1024;

__global__ __launch_bounds__(kPcOneThreads) void k_pchol_one(const double* lam, const double* g, int k, int ell,
                                                             double delta, int tmax, double* d, double* Lc, int* piv,
                                                             PcState* stt) {
  constexpr int NW = kPcOneThreads / 64;
  __shared__ double rv[NW], rs[NW];
  __shared__ int ri[NW];
  __shared__ int sp;
  __shared__ double spiv, strace;
  __shared__ double gp[kMaxEll];
  for (int i = threadIdx.x; i < k; i += kPcOneThreads) {
    double nn = 0.0;
    for (int a = 0; a < ell; ++a) nn = fma(g[(size_t)i * ell + a], g[(size_t)i * ell + a], nn);
    d[i] = -nn / (2.0 * lam[i]);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int t = 0;
  for (int r = 0; r < tmax; ++r) {
    double best = -1.0, sum = 0.0;
    int bi = 0x7fffffff;
    for (int i = threadIdx.x; i < k; i += kPcOneThreads) {
      const double v = d[i];
      sum += v;
      if (v > best || (v == best && i < bi)) { best = v; bi = i; }
    }
    auto merge = [&](double ob, int oi) {
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    };
    merge(lane_xor<1>(best), lane_xor<1>(bi));
    merge(lane_xor<2>(best), lane_xor<2>(bi));
    merge(lane_xor<7>(best), lane_xor<7>(bi));
    merge(lane_xor<15>(best), lane_xor<15>(bi));
    merge(lane_xor<16>(best), lane_xor<16>(bi));
    merge(lane_xor<32>(best), lane_xor<32>(bi));
    sum = wave_sum(sum);
    if (lane == 0) { rv[wave] = best; ri[wave] = bi; rs[wave] = sum; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = rv[0], sm = rs[0];
      int ii = ri[0];
      for (int w = 1; w < NW; ++w) {
        if (rv[w] > b || (rv[w] == b && ri[w] < ii)) { b = rv[w]; ii = ri[w]; }
        sm += rs[w];
      }
      sp = ii; spiv = b; strace = sm;
    }
    __syncthreads();
    if (!(strace > delta) || !(spiv > 0.0)) break;  // the same values in every thread
    const int p = sp;
    const double sq = sqrt(spiv);
    if (threadIdx.x < ell) gp[threadIdx.x] = g[(size_t)p * ell + threadIdx.x];
    __syncthreads();
    const double lp = lam[p];
    for (int i = threadIdx.x; i < k; i += kPcOneThreads) {
      double v;
      const double di = d[i];
      if (i == p) {
        v = sq;
      } else if (di == 0.0) {
        v = 0.0;
      } else {
        double dot = 0.0;
        for (int a = 0; a < ell; ++a) dot = fma(g[(size_t)i * ell + a], gp[a], dot);
        double y = -dot / (lam[i] + lp);
        for (int q = 0; q < r; ++q) y = fma(-Lc[(size_t)q * k + i], Lc[(size_t)q * k + p], y);
        v = y / sq;
      }
      Lc[(size_t)r * k + i] = v;
      const double nd = (i == p) ? 0.0 : di - v * v;
      d[i] = nd > 0.0 ? nd : 0.0;
    }
    if (threadIdx.x == 0) piv[r] = p;
    t = r + 1;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stt->stop = 1;
    stt->t = t;
  }
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

// Banded shifted solves: thread p factors S_p = -(T + lambda_{piv[p]} I) =
// L L^T (lower band, bandwidth ELL; S_p is positive definite since T is
// negative definite) row by row with the last ELL rows of L (and the
// reciprocals of their diagonal entries) kept in registers, solves
// L z = E_1 (gamma g_{piv[p]}^T) on the fly, stores the rows of L (interleaved
// by thread, the reciprocal of the diagonal in the diagonal's slot), then
// solves L^T x = z backwards.  x is Q Y~(:, piv[p]) = -(T + lambda I)^{-1} E_1
// gamma g^T written as S_p^{-1} E_1 gamma g^T.  X: k x tp column-major.
// The recurrences are sequential in the rows, so each thread keeps the loads
// of the next U rows (band entries forward, rows of L and z backward) in
// flight while it works on the current U rows: the chain per row is then a
// few FMAs, one square root and one division instead of a memory round trip
// and ELL + 2 divisions.
template <int ELL>
__global__ __launch_bounds__(64) void k_shift_solve(const double* band, int ldb, int k, const double* lam,
                                                    const double* g, const double* gamma, const int* piv, int tp,
                                                    double* Lb, double* X, int* fail) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= tp) return;
  constexpr int LB = ELL + 1;
  constexpr int U = ELL <= 4 ? 8 : (ELL <= 8 ? 4 : 2);
  const int ip = piv[p];
  const double sh = lam[ip];
  double rhs[ELL];
#pragma unroll
  for (int a = 0; a < ELL; ++a) {
    double acc = 0.0;
    for (int c = 0; c < ELL; ++c) acc = fma(gamma[a * ELL + c], g[(size_t)ip * ELL + c], acc);
    rhs[a] = acc;
  }
  // window: W[i][m] = L(j-ELL+i, j-ELL+i-ELL+m) for the previous ELL rows (m = 0..ELL, m == ELL is diagonal);
  // rd[i] = 1 / W[i][ELL]
  double W[ELL][LB], rd[ELL];
  double zw[ELL];  // z of the previous ELL rows
#pragma unroll
  for (int i = 0; i < ELL; ++i) {
    zw[i] = 0.0;
    rd[i] = 1.0;
#pragma unroll
    for (int m = 0; m < LB; ++m) W[i][m] = (m == ELL) ? 1.0 : 0.0;
  }
  double* x = X + (size_t)p * k;
  // B[u][m] = T(j-ELL+m, j) for m < ELL (0 above the first row), B[u][ELL] = T(j, j), j = j0 + u
  auto band_rows = [&](int j0, double (&B)[U][LB]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u;
#pragma unroll
      for (int m = 0; m < ELL; ++m) {
        const int i = j - ELL + m;
        B[u][m] = (i >= 0 && j < k) ? band[(size_t)i * ldb + (j - i)] : 0.0;
      }
      B[u][ELL] = j < k ? band[(size_t)j * ldb] : 0.0;
    }
  };
  double Bc[U][LB];
  band_rows(0, Bc);
  for (int j0 = 0; j0 < k; j0 += U) {
    double Bn[U][LB];
    band_rows(j0 + U, Bn);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u;
      if (j >= k) break;  // (the same j in every thread)
      // row j of L: Lj[m] = L(j, j-ELL+m), m = 0..ELL
      double Lj[LB];
#pragma unroll
      for (int m = 0; m < ELL; ++m) {
        const int i = j - ELL + m;  // column
        double v = 0.0;
        if (i >= 0) {
          v = -Bc[u][m];
          // subtract sum_{mm < m} L(j, j-ELL+mm) L(i, j-ELL+mm); row i is window slot m
#pragma unroll
          for (int mm = 0; mm < m; ++mm) v = fma(-Lj[mm], W[m][mm + ELL - m], v);
          v *= rd[m];
        }
        Lj[m] = v;
      }
      double djj = -(Bc[u][ELL] + sh);
#pragma unroll
      for (int m = 0; m < ELL; ++m) djj = fma(-Lj[m], Lj[m], djj);
      if (!(djj > 0.0)) { fail[0] = 1; djj = 1e-300; }
      Lj[ELL] = sqrt(djj);
      const double rj = 1.0 / Lj[ELL];
      // forward substitution
      double zj = j < ELL ? rhs[j < ELL ? j : 0] : 0.0;
#pragma unroll
      for (int m = 0; m < ELL; ++m) zj = fma(-Lj[m], zw[m], zj);
      zj *= rj;
      // store row j (the reciprocal in the diagonal's slot), slide the window
#pragma unroll
      for (int m = 0; m < ELL; ++m) Lb[((size_t)j * LB + m) * tp + p] = Lj[m];
      Lb[((size_t)j * LB + ELL) * tp + p] = rj;
      x[j] = zj;
#pragma unroll
      for (int i = 0; i < ELL - 1; ++i) {
        zw[i] = zw[i + 1];
        rd[i] = rd[i + 1];
#pragma unroll
        for (int m = 0; m < LB; ++m) W[i][m] = W[i + 1][m];
      }
      zw[ELL - 1] = zj;
      rd[ELL - 1] = rj;
#pragma unroll
      for (int m = 0; m < LB; ++m) W[ELL - 1][m] = Lj[m];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < LB; ++m) Bc[u][m] = Bn[u][m];
  }
  // backward: x_j = (z_j - sum_{r=j+1}^{j+ELL} L(r, j) x_r) / L(j, j); L(r, j) = row r slot j-r+ELL
  double xw[ELL];      // x of rows j+1..j+ELL
  double Rw[ELL][LB];  // rows j+1..j+ELL of L
#pragma unroll
  for (int i = 0; i < ELL; ++i) {
    xw[i] = 0.0;
#pragma unroll
    for (int m = 0; m < LB; ++m) Rw[i][m] = 0.0;
  }
  // R[u] = row j of L and Z[u] = z_j for j = j1 - u (descending)
  auto lrows = [&](int j1, double (&R)[U][LB], double (&Z)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j1 - u;
#pragma unroll
      for (int m = 0; m < LB; ++m) R[u][m] = j >= 0 ? Lb[((size_t)j * LB + m) * tp + p] : 0.0;
      Z[u] = j >= 0 ? x[j] : 0.0;
    }
  };
  double Rc[U][LB], Zc[U];
  lrows(k - 1, Rc, Zc);
  for (int j1 = k - 1; j1 >= 0; j1 -= U) {
    double Rn[U][LB], Zn[U];
    lrows(j1 - U, Rn, Zn);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j1 - u;
      if (j < 0) break;
      double v = Zc[u];
#pragma unroll
      for (int i = 0; i < ELL; ++i) v = fma(-Rw[i][ELL - 1 - i], xw[i], v);  // row j+1+i, column j: slot ELL-(1+i)
      v *= Rc[u][ELL];
      x[j] = v;
#pragma unroll
      for (int i = ELL - 1; i > 0; --i) {
        xw[i] = xw[i - 1];
#pragma unroll
        for (int m = 0; m < LB; ++m) Rw[i][m] = Rw[i - 1][m];
      }
      xw[0] = v;
#pragma unroll
      for (int m = 0; m < LB; ++m) Rw[0][m] = Rc[u][m];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      Zc[u] = Zn[u];
#pragma unroll
      for (int m = 0; m < LB; ++m) Rc[u][m] = Rn[u][m];
    }
  }
}

// B = L_PP^{-T} V1: L_PP[a][b] = Lc[b*k + piv[a]] (lower triangular);
// V1 given as tp x t row-major.  One thread per column.
__global__ void k_trsm_lt(const double* Lc, int k, const int* piv, int tp, const double* V1, int t, double* B) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= t) return;
  for (int a = tp - 1; a >= 0; --a) {
    double v = V1 ? V1[(size_t)a * t + c] : (a == c ? 1.0 : 0.0);
    for (int b = a + 1; b < tp; ++b) v -= Lc[(size_t)a * k + piv[b]] * B[(size_t)b * t + c];
    B[(size_t)a * t + c] = v / Lc[(size_t)a * k + piv[a]];
  }
}

// The same solve with one wave per column: the sum over b > a is split over
// the 64 lanes (a butterfly adds the parts; every lane ends with the same
// total), the solved entries of the column and the pivots are kept in LDS.
// tp <= kTrsmLds.
constexpr int kTrsmLds = 4096;
__global__ __launch_bounds__(64) void k_trsm_lt_wave(const double* Lc, int k, const int* piv, int tp,
                                                     const double* V1, int t, double* B) {
  __shared__ double sB[kTrsmLds];
  __shared__ int sp[kTrsmLds];
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  for (int b = lane; b < tp; b += 64) sp[b] = piv[b];
  __syncthreads();
  for (int a = tp - 1; a >= 0; --a) {
    const double* La = Lc + (size_t)a * k;
    double part = 0.0;
    for (int b = a + 1 + lane; b < tp; b += 64) part = fma(La[sp[b]], sB[b], part);
    const double tot = wave_sum(part);
    const double v = (V1 ? V1[(size_t)a * t + c] : (a == c ? 1.0 : 0.0)) - tot;
    const double x = v / La[sp[a]];
    if (lane == 0) {
      sB[a] = x;
      B[(size_t)a * t + c] = x;
    }
    __syncthreads();
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
                   const int* nlist, int nfixed, int batch, hipStream_t st, int* sweeps) {
  LYAP_REQUIRE(nfixed <= kJacMaxN, LYAP_E_UNSUPPORTED, "dense eigensolver limited to n <= %d (got %d)", kJacMaxN,
               nfixed);
  // nfixed is the largest n of the batch; LDS-sized matrices run on one wave,
  // with the rotation loops unrolled for the smallest size class that fits
  const dim3 g(batch);
  if (nfixed <= 8)
    hipLaunchKernelGGL(k_jacobi<8>, g, dim3(64), 0, st, A, strideA, Q, strideQ, lam, strideL, nlist, nfixed, 40, sweeps);
  else if (nfixed <= 16)
    hipLaunchKernelGGL(k_jacobi<16>, g, dim3(64), 0, st, A, strideA, Q, strideQ, lam, strideL, nlist, nfixed, 40, sweeps);
  else if (nfixed <= 32)
    hipLaunchKernelGGL(k_jacobi<32>, g, dim3(64), 0, st, A, strideA, Q, strideQ, lam, strideL, nlist, nfixed, 40, sweeps);
  else if (nfixed <= kJacLds)
    hipLaunchKernelGGL(k_jacobi<kJacLds>, g, dim3(64), 0, st, A, strideA, Q, strideQ, lam, strideL, nlist, nfixed, 40,
                       sweeps);
  else
    hipLaunchKernelGGL(k_jacobi<0>, g, dim3(kJacThreads), 0, st, A, strideA, Q, strideQ, lam, strideL, nlist, nfixed,
                       40, sweeps);
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

struct PcholRun::Impl {
  const double* lam;
  const double* g;
  int k, ell, tmax, grid, r = 0;
  double delta;
  double* d;
  double* Lc;
  int* piv;
  hipStream_t st;
  DevBuf pvA, pvB, psA, psB, piA, piB, stt;
  HostBuf hst;
  bool finished = false;
  bool one = false;  // k_pchol_one: the whole factorisation in one launch
  int t = 0;
};

PcholRun::PcholRun(const double* lam, const double* g, int k, int ell, double delta, int tmax, double* d, double* Lc,
                   int* piv, hipStream_t st)
    : w_(new Impl) {
  Impl& w = *w_;
  w.lam = lam;
  w.g = g;
  w.k = k;
  w.ell = ell;
  w.tmax = tmax;
  w.delta = delta;
  w.d = d;
  w.Lc = Lc;
  w.piv = piv;
  w.st = st;
  w.grid = std::max(1, std::min((k + kPcThreads - 1) / kPcThreads, 256));
  w.one = k <= kPcOneMax;
  w.stt.alloc(sizeof(PcState));
  w.hst.alloc(sizeof(PcState));
  std::memset(w.hst.p, 0, sizeof(PcState));
  if (tmax <= 0) w.finished = true;
  if (w.one) return;
  const int grid = w.grid;
  w.pvA.alloc(grid * sizeof(double));
  w.pvB.alloc(grid * sizeof(double));
  w.psA.alloc(grid * sizeof(double));
  w.psB.alloc(grid * sizeof(double));
  w.piA.alloc(grid * sizeof(int));
  w.piB.alloc(grid * sizeof(int));
  hipLaunchKernelGGL(k_pchol_init, dim3(grid), dim3(kPcThreads), 0, st, lam, g, k, ell, d, w.pvA.as<double>(),
                     w.piA.as<int>(), w.psA.as<double>(), w.stt.as<PcState>());
  LYAP_LAUNCHED("pchol init");
}

PcholRun::~PcholRun() { delete w_; }

bool PcholRun::launch_chunk() {
  Impl& w = *w_;
  if (w.finished) return false;
  if (w.one) {
    hipLaunchKernelGGL(k_pchol_one, dim3(1), dim3(kPcOneThreads), 0, w.st, w.lam, w.g, w.k, w.ell, w.delta, w.tmax,
                       w.d, w.Lc, w.piv, w.stt.as<PcState>());
    LYAP_LAUNCHED("pchol one");
    LYAP_HIP(hipMemcpyAsync(w.hst.p, w.stt.p, sizeof(PcState), hipMemcpyDeviceToHost, w.st));
    w.r = w.tmax;
    return true;
  }
  // pivot steps up to the next multiple of 32 (or tmax), then the state
  const int end = std::min(w.tmax, (w.r / 32 + 1) * 32);
  for (; w.r < end; ++w.r) {
    const bool even = (w.r % 2) == 0;
    hipLaunchKernelGGL(k_pchol_step, dim3(w.grid), dim3(kPcThreads), 0, w.st, w.lam, w.g, w.k, w.ell, w.delta, w.r, w.d,
                       w.Lc, w.piv, even ? w.pvA.as<double>() : w.pvB.as<double>(),
                       even ? w.piA.as<int>() : w.piB.as<int>(), even ? w.psA.as<double>() : w.psB.as<double>(),
                       w.grid, even ? w.pvB.as<double>() : w.pvA.as<double>(), even ? w.piB.as<int>() : w.piA.as<int>(),
                       even ? w.psB.as<double>() : w.psA.as<double>(), w.stt.as<PcState>());
  }
  LYAP_LAUNCHED("pchol");
  LYAP_HIP(hipMemcpyAsync(w.hst.p, w.stt.p, sizeof(PcState), hipMemcpyDeviceToHost, w.st));
  return true;
}

void PcholRun::read() {
  Impl& w = *w_;
  const PcState& h = *w.hst.as<PcState>();
  w.t = h.t;
  if (h.stop || w.r >= w.tmax) w.finished = true;
}

bool PcholRun::finished() const { return w_->finished; }
int PcholRun::t() const { return w_->t; }

int run_pchol(const double* lam, const double* g, int k, int ell, double delta, int tmax, double* d, double* Lc,
              int* piv, hipStream_t st) {
  PcholRun run(lam, g, k, ell, delta, tmax, d, Lc, piv, st);
  while (run.launch_chunk()) {
    LYAP_HIP(hipStreamSynchronize(st));
    run.read();
  }
  return run.t();
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
  const int grid = (tp + 63) / 64;
  switch (ell) {
#define LYAP_SS(E) case E: hipLaunchKernelGGL((k_shift_solve<E>), dim3(grid), dim3(64), 0, st, band, ldb, k, lam, g, gamma, piv, tp, Lb, X, fail); break;
    LYAP_SS(1) LYAP_SS(2) LYAP_SS(3) LYAP_SS(4) LYAP_SS(5) LYAP_SS(6) LYAP_SS(7) LYAP_SS(8)
    LYAP_SS(10) LYAP_SS(12) LYAP_SS(14) LYAP_SS(16)
#undef LYAP_SS
    default: LYAP_REQUIRE(false, LYAP_E_UNSUPPORTED, "shifted solve for ell=%d not built", ell);
  }
  LYAP_LAUNCHED("shift_solve");
}

void launch_gemm_xb(const double* X, int k, int tp, const double* B, int t, double* M, hipStream_t st) {
  const int64_t tot = (int64_t)k * t;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 8192));
  hipLaunchKernelGGL(k_gemm_xb, dim3(grid), dim3(256), 0, st, X, k, tp, B, t, M);
  LYAP_LAUNCHED("gemm_xb");
}

void launch_assemble_M(const double* Lc, int k, const int* piv, int tp, const double* Qg, int t, const double* X,
                       double* V1, double* B, double* M, hipStream_t st) {
  int64_t tot = (int64_t)tp * t;
  int grid = (int)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 4096));
  if (Qg) hipLaunchKernelGGL(k_pick_top, dim3(grid), dim3(256), 0, st, Qg, tp, t, V1);
  if (tp <= kTrsmLds)
    hipLaunchKernelGGL(k_trsm_lt_wave, dim3(t), dim3(64), 0, st, Lc, k, piv, tp, V1, t, B);
  else
    hipLaunchKernelGGL(k_trsm_lt, dim3((t + 63) / 64), dim3(64), 0, st, Lc, k, piv, tp, V1, t, B);
  tot = (int64_t)k * t;
  grid = (int)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 8192));
  hipLaunchKernelGGL(k_gemm_xb, dim3(grid), dim3(256), 0, st, X, k, tp, B, t, M);
  LYAP_LAUNCHED("assemble_M");
}

}  // namespace lyap
