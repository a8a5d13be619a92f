// Learned SPD preconditioner: forward (K, K^T), backward (weight gradients of
// the energy-norm loss), Adam, and the component entry points used by the
// tests.  See pcnet.hpp for the definition.
//
// Convolutions of the application z = M r: four tiled kernels (8 x 8 x 4
// output points per workgroup, input tile and halo staged in LDS), the input
// channels formed inside the first and the output z inside the last.  The
// training's convolutions keep their activations: the weights in LDS,
// neighbours read through the caches, four consecutive cells per thread with
// vector loads when nx is a multiple of 4, else one per thread.  Weight
// gradients: 8 x 8 x 4 cell tiles with a one-cell halo staged in LDS, each
// thread accumulating the three x taps of one (output, input, dz, dy) weight
// group over the tile; per-tile partials are summed in FP64 in a fixed order
// (two passes).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "pcnet.hpp"
#include "pcg.hpp"

namespace lyap {

constexpr int kPcThreads = 256;
constexpr int kTX = 8, kTY = 8, kTZ = 4;                    // weight-gradient tile
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;  // with halo
constexpr int kWSeg = 64;  // first-pass segments of the tile sums

__device__ __forceinline__ void offset_of(int t, int& dz, int& dy, int& dx) {
  dz = t / 9 - 1;
  dy = (t / 3) % 3 - 1;
  dx = t % 3 - 1;
}

// dinv = 1 / (-A_pp) (FP64), s = sqrt(dinv) (FP32), partial sums of log(-A_pp)
__global__ __launch_bounds__(kPcThreads) void k_pc_prep1(OpDev<double> op, int n, double* dinv, float* s,
                                                         double* part) {
  __shared__ double red[kPcThreads / 64];
  double acc[1] = {0.0};
  for (int p = blockIdx.x * kPcThreads + threadIdx.x; p < n; p += gridDim.x * kPcThreads) {
    const double d = -op_diag<double>(op, p);
    dinv[p] = 1.0 / d;
    s[p] = (float)sqrt(1.0 / d);
    acc[0] += log(d);
  }
  write_partial<1, kPcThreads>(acc, red, part);
}

// f = log(-A_pp) - mean
__global__ __launch_bounds__(kPcThreads) void k_pc_prep2(OpDev<double> op, int n, const double* part, int nparts,
                                                         float* f) {
  __shared__ double red[kPcThreads / 64];
  reduce_partials<1, kPcThreads>(part, nparts, red);
  const double mean = uniform_d(red[0]) / (double)n;
  for (int p = blockIdx.x * kPcThreads + threadIdx.x; p < n; p += gridDim.x * kPcThreads)
    f[p] = (float)(log(-op_diag<double>(op, p)) - mean);
}

// From a given diagonal part: s = sqrt(dinv) (FP32), partial sums of
// log(1 / dinv) and of the count over the points with dinv > 0.
__global__ __launch_bounds__(kPcThreads) void k_pc_prep_d1(const double* __restrict__ dinv, int n, float* s,
                                                           double* part) {
  __shared__ double red[2 * (kPcThreads / 64)];
  double acc[2] = {0.0, 0.0};
  for (int p = blockIdx.x * kPcThreads + threadIdx.x; p < n; p += gridDim.x * kPcThreads) {
    const double d = dinv[p];
    s[p] = (float)sqrt(d);
    if (d > 0.0) {
      acc[0] += -log(d);
      acc[1] += 1.0;
    }
  }
  write_partial<2, kPcThreads>(acc, red, part);
}

// f = log(1 / dinv) - mean over the points with dinv > 0, 0 elsewhere
__global__ __launch_bounds__(kPcThreads) void k_pc_prep_d2(const double* __restrict__ dinv, int n, const double* part,
                                                           int nparts, float* f) {
  __shared__ double red[2 * (kPcThreads / 64)];
  reduce_partials<2, kPcThreads>(part, nparts, red);
  const double mean = uniform_d(red[0]) / uniform_d(red[1]);
  for (int p = blockIdx.x * kPcThreads + threadIdx.x; p < n; p += gridDim.x * kPcThreads) {
    const double d = dinv[p];
    f[p] = d > 0.0 ? (float)(-log(d) - mean) : 0.0f;
  }
}

// dd = z - e (the network's error for the pair)
__global__ void k_pc_sub(const double* __restrict__ z, const double* __restrict__ e, int n, double* __restrict__ dd) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dd[p] = z[p] - e[p];
}

// with Kd = K dd given: gw = s * 2 Kd / eAe (FP32), partial dd.Kd
__global__ __launch_bounds__(kPcThreads) void k_pc_resid_k(const double* __restrict__ dd, const double* __restrict__ kd,
                                                           const float* __restrict__ s, double eAe, int n,
                                                           float* __restrict__ gw, double* part) {
  __shared__ double red[kPcThreads / 64];
  double acc[1] = {0.0};
  for (int p = blockIdx.x * kPcThreads + threadIdx.x; p < n; p += gridDim.x * kPcThreads) {
    acc[0] = fma(dd[p], kd[p], acc[0]);
    gw[p] = (float)((double)s[p] * 2.0 * kd[p] / eAe);
  }
  write_partial<1, kPcThreads>(acc, red, part);
}

// partial x.y
__global__ __launch_bounds__(kPcThreads) void k_pc_dot(const double* __restrict__ x, const double* __restrict__ y,
                                                       int n, double* part) {
  __shared__ double red[kPcThreads / 64];
  double acc[1] = {0.0};
  for (int p = blockIdx.x * kPcThreads + threadIdx.x; p < n; p += gridDim.x * kPcThreads) acc[0] = fma(x[p], y[p], acc[0]);
  write_partial<1, kPcThreads>(acc, red, part);
}

// x0 = [s r, f s r]
__global__ void k_pc_in_r(const double* __restrict__ r, const float* __restrict__ s, const float* __restrict__ f,
                          int n, float* __restrict__ x0) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float u = (float)((double)s[p] * r[p]);
  x0[p] = u;
  x0[(size_t)n + p] = f[p] * u;
}

// x0 = [g, f g]
__global__ void k_pc_in_g(const float* __restrict__ g, const float* __restrict__ f, int n, float* __restrict__ x0) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  x0[p] = g[p];
  x0[(size_t)n + p] = f[p] * g[p];
}

// out[o][p] = sum_i sum_t W[o][i][t] in[i][p + t]
template <int CI, int CO>
__global__ __launch_bounds__(kPcThreads) void k_pc_conv(const float* __restrict__ in, const float* __restrict__ W,
                                                        float* __restrict__ out, int nx, int ny, int nz) {
  const int n = nx * ny * nz;
  const int lb = xcd_block(blockIdx.x, (n + kPcThreads - 1) / kPcThreads);
  if (lb < 0) return;
  __shared__ float sW[CO * CI * 27];
  for (int e = threadIdx.x; e < CO * CI * 27; e += kPcThreads) sW[e] = W[e];
  __syncthreads();
  const int p = lb * kPcThreads + threadIdx.x;
  if (p >= n) return;
  const int nxy = nx * ny;
  const int z = p / nxy, y = (p / nx) % ny, x = p % nx;
  float acc[CO];
#pragma unroll
  for (int o = 0; o < CO; ++o) acc[o] = 0.f;
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    int dz, dy, dx;
    offset_of(t, dz, dy, dx);
    const int zz = z + dz, yy = y + dy, xx = x + dx;
    if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx) continue;
    const int q = p + dz * nxy + dy * nx + dx;
#pragma unroll
    for (int i = 0; i < CI; ++i) {
      const float v = in[(size_t)i * n + q];
#pragma unroll
      for (int o = 0; o < CO; ++o) acc[o] = fmaf(sW[(o * CI + i) * 27 + t], v, acc[o]);
    }
  }
#pragma unroll
  for (int o = 0; o < CO; ++o) out[(size_t)o * n + p] = acc[o];
}

// The adjoint: out[i][q] = sum_o sum_t W[o][i][t] in[o][q - t]
template <int CO, int CI>
__global__ __launch_bounds__(kPcThreads) void k_pc_convT(const float* __restrict__ in, const float* __restrict__ W,
                                                         float* __restrict__ out, int nx, int ny, int nz) {
  const int n = nx * ny * nz;
  const int lb = xcd_block(blockIdx.x, (n + kPcThreads - 1) / kPcThreads);
  if (lb < 0) return;
  __shared__ float sW[CO * CI * 27];
  for (int e = threadIdx.x; e < CO * CI * 27; e += kPcThreads) sW[e] = W[e];
  __syncthreads();
  const int p = lb * kPcThreads + threadIdx.x;
  if (p >= n) return;
  const int nxy = nx * ny;
  const int z = p / nxy, y = (p / nx) % ny, x = p % nx;
  float acc[CI];
#pragma unroll
  for (int i = 0; i < CI; ++i) acc[i] = 0.f;
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    int dz, dy, dx;
    offset_of(t, dz, dy, dx);
    const int zz = z - dz, yy = y - dy, xx = x - dx;
    if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx) continue;
    const int q = p - dz * nxy - dy * nx - dx;
#pragma unroll
    for (int o = 0; o < CO; ++o) {
      const float v = in[(size_t)o * n + q];
#pragma unroll
      for (int i = 0; i < CI; ++i) acc[i] = fmaf(sW[(o * CI + i) * 27 + t], v, acc[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < CI; ++i) out[(size_t)i * n + p] = acc[i];
}

// Both convolutions with four consecutive x cells per thread, for nx a
// multiple of 4: per (dz, dy) and input channel, one aligned float4 load and
// two edge loads give the six inputs x0-1 .. x0+4 that the three x taps of the
// four cells read, so a cell costs about a quarter of the loads of the kernels
// above.  TRANS = false: out[o][p] = sum_t sum_i W[o][i][t] in[i][p + t];
// TRANS = true (the adjoint): out[i][q] = sum_t sum_o W[o][i][t] in[o][q - t].
// The terms are added in the same order as in k_pc_conv / k_pc_convT; taps
// outside the grid in x add an exact zero instead of being skipped.
template <int CI, int CO, bool TRANS>
__global__ __launch_bounds__(kPcThreads) void k_pc_conv4(const float* __restrict__ in, const float* __restrict__ W,
                                                         float* __restrict__ out, int nx, int ny, int nz) {
  constexpr int NIN = TRANS ? CO : CI;
  constexpr int NOUT = TRANS ? CI : CO;
  constexpr int SG = TRANS ? -1 : 1;
  const int n = nx * ny * nz;
  const int nq = n / 4;
  const int lb = xcd_block(blockIdx.x, (nq + kPcThreads - 1) / kPcThreads);
  if (lb < 0) return;
  __shared__ float sW[CO * CI * 27];
  for (int e = threadIdx.x; e < CO * CI * 27; e += kPcThreads) sW[e] = W[e];
  __syncthreads();
  const int qd = lb * kPcThreads + threadIdx.x;
  if (qd >= nq) return;
  const int p0 = 4 * qd;
  const int nxy = nx * ny;
  const int z = p0 / nxy, y = (p0 / nx) % ny, x0 = p0 % nx;
  float acc[NOUT][4];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[o][k] = 0.f;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    const int zz = z + SG * dz;
    if (zz < 0 || zz >= nz) continue;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = y + SG * dy;
      if (yy < 0 || yy >= ny) continue;
      const size_t base = (size_t)zz * nxy + (size_t)yy * nx + x0;
      float v[NIN][6];
#pragma unroll
      for (int c = 0; c < NIN; ++c) {
        const float* row = in + (size_t)c * n + base;
        const float4 mid = *reinterpret_cast<const float4*>(row);
        v[c][0] = x0 > 0 ? row[-1] : 0.f;
        v[c][1] = mid.x;
        v[c][2] = mid.y;
        v[c][3] = mid.z;
        v[c][4] = mid.w;
        v[c][5] = x0 + 4 < nx ? row[4] : 0.f;
      }
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int t = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
        const int sh = SG * dx;
#pragma unroll
        for (int c = 0; c < NIN; ++c)
#pragma unroll
          for (int o = 0; o < NOUT; ++o) {
            const float w = TRANS ? sW[(c * CI + o) * 27 + t] : sW[(o * CI + c) * 27 + t];
            // a tap outside the grid in x reads the zero padding (adds 0)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[o][k] = fmaf(w, v[c][1 + k + sh], acc[o][k]);
          }
      }
    }
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    float4 r;
    r.x = acc[o][0];
    r.y = acc[o][1];
    r.z = acc[o][2];
    r.w = acc[o][3];
    *reinterpret_cast<float4*>(out + (size_t)o * n + p0) = r;
  }
}

// ------------------------------------------------------------------ tiled application
// The preconditioner's application z = M r as four tiled convolutions: one
// output point per thread over an 8 x 8 x 4 tile, the input channels of the
// tile and its one-point halo staged in LDS first (each input value is read
// from memory once per tile instead of once per tap through the caches; the
// channel counts are too small to keep a wave busy otherwise).  Tiles are
// dealt XCD by XCD (neighbouring tiles share halo rows in one L2).
//   MODE 0: FP32 channels in[c][n] -> out[o][n];
//   MODE 1: the input channels x0 = [u, f u], u = s r rounded to FP32, formed
//           from r, s, f while staging (the first convolution);
//   MODE 2: the output of the last transposed convolution (two channels d)
//           as z = dinv r + s (d0 + f d1) (FP64), with one partial z.q per tile;
//   MODE 3: as MODE 1 from r = r_in - alpha q, with the flexible CG update of
//           x and r at the tile's own points and one partial r.r per tile
//           (the PcUpd argument).
// TRANS = false: out[o][p] = sum_t sum_i W[o][i][t] in[i][p + t];
// TRANS = true (the adjoint): out[i][p] = sum_t sum_o W[o][i][t] in[o][p - t].
constexpr int kQX = 8, kQY = 8, kQZ = 4;
constexpr int kQHX = kQX + 2, kQHY = kQY + 2, kQHZ = kQZ + 2;
constexpr int kQH = kQHX * kQHY * kQHZ;

template <int CI, int CO, bool TRANS, int MODE>
__global__ __launch_bounds__(kPcThreads) void k_pc_tile(const float* __restrict__ in, const double* __restrict__ r,
                                                        const float* __restrict__ s, const float* __restrict__ f,
                                                        const double* __restrict__ dinv, const float* __restrict__ W,
                                                        float* __restrict__ out, double* __restrict__ z,
                                                        const double* __restrict__ q, double* part, int nx, int ny,
                                                        int nz, int tx, int ty, int tz, PcUpd u) {
  static_assert(kQX * kQY * kQZ == kPcThreads, "one output point per thread");
  constexpr int NIN = TRANS ? CO : CI;
  constexpr int NOUT = TRANS ? CI : CO;
  constexpr int SG = TRANS ? -1 : 1;
  static_assert((MODE != 1 && MODE != 3) || NIN == 2, "the formed input has two channels");
  static_assert(MODE != 2 || NOUT == 2, "the output is formed from two channels");
  const int lb = xcd_block(blockIdx.x, tx * ty * tz);
  if (lb < 0) return;
  __shared__ float sx[NIN * kQH];
  __shared__ double red[kPcThreads / 64];
  const int bx = lb % tx, by = (lb / tx) % ty, bz = lb / (tx * ty);
  const int x0 = bx * kQX, y0 = by * kQY, z0 = bz * kQZ;
  const int n = nx * ny * nz;
  double alpha = 0.0;
  if constexpr (MODE == 3) {
    // alpha = p.r / p.q, identical in every workgroup (fixed summation order)
    __shared__ double redu[2 * (kPcThreads / 64)];
    reduce_partials<2, kPcThreads>(u.pin, u.nparts, redu);
    const double pq = uniform_d(redu[0]), pr = uniform_d(redu[1]);
    __syncthreads();
    const bool active = uniform_d(u.log[u.it].rr[0]) > uniform_d(u.state[0]);
    alpha = (active && pq > 0.0) ? pr / pq : 0.0;
    if (lb == 0 && threadIdx.x == 0) {
      u.log[u.it].sigma[0] = pq;
      u.log[u.it].rho[0] = pr;
      u.log[u.it].alpha[0] = alpha;
      if (active && !(pq > 0.0)) u.flag[1] = u.it + 1;
    }
  }
  // every thread loads its (at most three) halo-tile points before storing
  // any, so that all loads are in flight together
  constexpr int NST = (kQH + kPcThreads - 1) / kPcThreads;
  float v0[NST], v1[NST][NIN > 1 ? NIN - 1 : 1];
#pragma unroll
  for (int k = 0; k < NST; ++k) {
    const int h = threadIdx.x + k * kPcThreads;
    const int hx = h % kQHX, hy = (h / kQHX) % kQHY, hz = h / (kQHX * kQHY);
    const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
    const bool inside = h < kQH && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
    const int p = inside ? gx + nx * (gy + ny * gz) : 0;
    if constexpr (MODE == 1 || MODE == 3) {
      float su = 0.f, fu = 0.f;
      if (inside) {
        const double rp = MODE == 3 ? fma(-alpha, u.q[p], u.r_in[p]) : r[p];
        su = (float)((double)s[p] * rp);
        fu = f[p] * su;
      }
      v0[k] = su;
      v1[k][0] = fu;
    } else {
      v0[k] = inside ? in[p] : 0.f;
#pragma unroll
      for (int c = 1; c < NIN; ++c) v1[k][c - 1] = inside ? in[(size_t)c * n + p] : 0.f;
    }
  }
#pragma unroll
  for (int k = 0; k < NST; ++k) {
    const int h = threadIdx.x + k * kPcThreads;
    if (h < kQH) {
      sx[h] = v0[k];
#pragma unroll
      for (int c = 1; c < NIN; ++c) sx[c * kQH + h] = v1[k][c - 1];
    }
  }
  __syncthreads();
  const int lx = threadIdx.x % kQX, ly = (threadIdx.x / kQX) % kQY, lz = threadIdx.x / (kQX * kQY);
  const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
  const bool own = gx < nx && gy < ny && gz < nz;
  float acc[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) acc[o] = 0.f;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int t = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
        const int idx = ((lz + 1 + SG * dz) * kQHY + (ly + 1 + SG * dy)) * kQHX + (lx + 1 + SG * dx);
#pragma unroll
        for (int c = 0; c < NIN; ++c) {
          const float v = sx[c * kQH + idx];
#pragma unroll
          for (int o = 0; o < NOUT; ++o) {
            // uniform address: a scalar load, the weight an SGPR operand of the FMA
            const float w = TRANS ? W[(c * CI + o) * 27 + t] : W[(o * CI + c) * 27 + t];
            acc[o] = fmaf(w, v, acc[o]);
          }
        }
      }
  const int p = gx + nx * (gy + ny * gz);
  if constexpr (MODE == 2) {
    double zq[1] = {0.0};
    if (own) {
      const double w = (double)acc[0] + (double)f[p] * (double)acc[1];
      const double zv = fma(dinv[p], r[p], (double)s[p] * w);
      z[p] = zv;
      if (q) zq[0] = zv * q[p];
    }
    if (part) write_partial_at<1, kPcThreads>(zq, red, part, lb);
  } else {
    if (own) {
#pragma unroll
      for (int o = 0; o < NOUT; ++o) out[(size_t)o * n + p] = acc[o];
    }
    if constexpr (MODE == 3) {
      double rr[1] = {0.0};
      if (own) {
        const double rq = fma(-alpha, u.q[p], u.r_in[p]);
        u.r_out[p] = rq;
        u.x[p] = fma(alpha, u.p[p], u.x[p]);
        rr[0] = rq * rq;
      }
      write_partial_at<1, kPcThreads>(rr, red, u.rr_part, lb);
    }
  }
}

// z = dinv r + s (d0 + f d1); optional partial z.q per workgroup
template <int NT>
__global__ __launch_bounds__(NT) void k_pc_out(const double* __restrict__ r, const double* __restrict__ dinv,
                                               const float* __restrict__ s, const float* __restrict__ f,
                                               const float* __restrict__ d, int n, double* __restrict__ z,
                                               const double* __restrict__ q, double* part) {
  __shared__ double red[NT / 64];
  double acc[1] = {0.0};
  for (int p = blockIdx.x * NT + threadIdx.x; p < n; p += gridDim.x * NT) {
    const double w = (double)d[p] + (double)f[p] * (double)d[(size_t)n + p];
    const double zp = fma(dinv[p], r[p], (double)s[p] * w);
    z[p] = zp;
    if (q) acc[0] = fma(zp, q[p], acc[0]);
  }
  if (part) write_partial<1, NT>(acc, red, part);
}

// dd = z - e, Ad = (-A) dd, gw = s * 2 Ad / eAe (FP32), partial dd.Ad
__global__ __launch_bounds__(kPcThreads) void k_pc_resid(OpDev<double> op, const double* __restrict__ z,
                                                         const double* __restrict__ e, const float* __restrict__ s,
                                                         double eAe, int n, float* __restrict__ gw, double* part) {
  __shared__ double red[kPcThreads / 64];
  double acc[1] = {0.0};
  for (int p = blockIdx.x * kPcThreads + threadIdx.x; p < n; p += gridDim.x * kPcThreads) {
    double w[1];
    op_row_fn<double, 1>(op, p, [&](int i, double (&v)[1]) { v[0] = z[i] - e[i]; }, w);
    const double Ad = -w[0];
    const double dd = z[p] - e[p];
    acc[0] = fma(dd, Ad, acc[0]);
    gw[p] = (float)((double)s[p] * 2.0 * Ad / eAe);
  }
  write_partial<1, kPcThreads>(acc, red, part);
}

// e^T (-A) e partials
__global__ __launch_bounds__(kPcThreads) void k_pc_energy(OpDev<double> op, const double* __restrict__ e, int n,
                                                          double* part) {
  __shared__ double red[kPcThreads / 64];
  double acc[1] = {0.0};
  for (int p = blockIdx.x * kPcThreads + threadIdx.x; p < n; p += gridDim.x * kPcThreads) {
    double w[1];
    op_row<double, 1>(op, e, p, w);
    acc[0] = fma(e[p], -w[0], acc[0]);
  }
  write_partial<1, kPcThreads>(acc, red, part);
}

// Weight gradient of <g, conv(x, W)> over one 8x8x4 tile: part[tile][(o*CI+i)*27+t]
template <int CI, int CO>
__global__ __launch_bounds__(kPcThreads) void k_pc_wgrad(const float* __restrict__ x, const float* __restrict__ g,
                                                         float* __restrict__ part, int nx, int ny, int nz) {
  __shared__ float xs[CI][kHZ * kHY * kHX];
  __shared__ float gs[CO][kTZ * kTY * kTX];
  const int n = nx * ny * nz;
  const int nxy = nx * ny;
  const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
  for (int h = threadIdx.x; h < kHZ * kHY * kHX; h += kPcThreads) {
    const int hz = h / (kHY * kHX), hy = (h / kHX) % kHY, hx = h % kHX;
    const int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
    const bool in = zz >= 0 && zz < nz && yy >= 0 && yy < ny && xx >= 0 && xx < nx;
    const size_t q = in ? (size_t)zz * nxy + (size_t)yy * nx + xx : 0;
#pragma unroll
    for (int i = 0; i < CI; ++i) xs[i][h] = in ? x[(size_t)i * n + q] : 0.f;
  }
  {
    const int c = threadIdx.x;  // kTZ*kTY*kTX == kPcThreads
    const int cz = c / (kTY * kTX), cy = (c / kTX) % kTY, cx = c % kTX;
    const int zz = z0 + cz, yy = y0 + cy, xx = x0 + cx;
    const bool in = zz < nz && yy < ny && xx < nx;
    const size_t q = in ? (size_t)zz * nxy + (size_t)yy * nx + xx : 0;
#pragma unroll
    for (int o = 0; o < CO; ++o) gs[o][c] = in ? g[(size_t)o * n + q] : 0.f;
  }
  __syncthreads();
  constexpr int E = CO * CI * 27;
  const size_t tile = blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
  // one thread per (o, i, dz, dy): its three dx taps read the same g row and
  // overlapping x rows (kTX + 2 values), so the row is read from LDS once;
  // each weight still sums over cz, cy, cx in that order
  for (int grp = threadIdx.x; grp < CO * CI * 9; grp += kPcThreads) {
    const int o = grp / (CI * 9), i = (grp / 9) % CI, dzy = grp % 9;
    const int dz = dzy / 3 - 1, dy = dzy % 3 - 1;
    float acc[3] = {0.f, 0.f, 0.f};
    for (int cz = 0; cz < kTZ; ++cz)
      for (int cy = 0; cy < kTY; ++cy) {
        const float* gr = &gs[o][(cz * kTY + cy) * kTX];
        const float* xr = &xs[i][((cz + 1 + dz) * kHY + (cy + 1 + dy)) * kHX];
        float xv[kTX + 2];
#pragma unroll
        for (int j = 0; j < kTX + 2; ++j) xv[j] = xr[j];
#pragma unroll
        for (int cx = 0; cx < kTX; ++cx) {
          const float gv = gr[cx];
#pragma unroll
          for (int k = 0; k < 3; ++k) acc[k] = fmaf(gv, xv[cx + k], acc[k]);
        }
      }
    const int e0 = (o * CI + i) * 27 + 3 * dzy;  // tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1)
#pragma unroll
    for (int k = 0; k < 3; ++k) part[tile * E + e0 + k] = acc[k];
  }
}

// tmp[seg][e] = sum over the tiles of segment seg (FP64).  A workgroup takes
// 64 weights (one per lane) of one segment; its four waves sum the tiles
// t = b + w, b + w + 4, ... (w = wave), and the four wave sums are added in
// wave order: a fixed order, with four independent load streams per weight.
__global__ __launch_bounds__(256) void k_pc_wreduce1(const float* __restrict__ part, int ntiles, int E, int per,
                                                     double* __restrict__ tmp) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int sgm = blockIdx.y;
  const int b = sgm * per, end = min(ntiles, b + per);
  double acc = 0.0;
  if (e < E)
    for (int t = b + w; t < end; t += 4) acc += (double)part[(size_t)t * E + e];
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && e < E) tmp[(size_t)sgm * E + e] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// out[e] (+)= sum_seg tmp[seg][e], split over the four waves as in
// k_pc_wreduce1 (segments w, w + 4, ...; wave sums added in wave order)
__global__ __launch_bounds__(256) void k_pc_wreduce2(const double* __restrict__ tmp, int nseg, int E,
                                                     double* __restrict__ out, int accumulate) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (e < E)
    for (int sgm = w; sgm < nseg; sgm += 4) acc += tmp[(size_t)sgm * E + e];
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && e < E) {
    const double sum = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    out[e] = accumulate ? out[e] + sum : sum;
  }
}

__global__ void k_pc_loss(const double* part, int nparts, double eAe, double* loss) {
  __shared__ double red[kPcThreads / 64];
  reduce_partials<1, kPcThreads>(part, nparts, red);
  if (threadIdx.x == 0) loss[0] = red[0] / eAe;
}

__global__ void k_pc_sum1(const double* part, int nparts, double* out) {
  __shared__ double red[kPcThreads / 64];
  reduce_partials<1, kPcThreads>(part, nparts, red);
  if (threadIdx.x == 0) out[0] = red[0];
}

// Adam (FP32 parameters and moments, FP64 gradient)
__global__ void k_pc_adam(float* W, const double* g, float* m, float* v, int P, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = (float)g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  W[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ host
void pcnet_init_weights(int C, uint64_t seed, double scale, float* W) {
  uint64_t state = seed;
  const int P = pcnet_param_count(C);
  for (int i = 0; i < P; ++i) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double u = (double)(z >> 11) / 9007199254740992.0;  // 2^53
    W[i] = (float)(scale * (2.0 * u - 1.0));
  }
}

PcNetGpu::PcNetGpu(const OpDev<double>& op, int C, hipStream_t st) : op_(op), C_(C), st_(st) {
  LYAP_REQUIRE(op.kind == LYAP_OP_STENCIL5 || op.kind == LYAP_OP_STENCIL7, LYAP_E_UNSUPPORTED,
               "the learned preconditioner needs a stencil operator (a grid)");
  LYAP_REQUIRE(C == 2 || C == 4 || C == 8, LYAP_E_UNSUPPORTED, "network width C=%d not built (2, 4, 8)", C);
  nx_ = op.nx;
  ny_ = op.ny;
  nz_ = op.kind == LYAP_OP_STENCIL5 ? 1 : op.nz;
  n_ = op.n;
  alloc_common();
  const int g = grid_for(n_, 1, 1024);
  hipLaunchKernelGGL(k_pc_prep1, dim3(g), dim3(kPcThreads), 0, st_, op_, n_, dinv_.as<double>(), s_.as<float>(),
                     part_.as<double>());
  hipLaunchKernelGGL(k_pc_prep2, dim3(g), dim3(kPcThreads), 0, st_, op_, n_, part_.as<double>(), g, f_.as<float>());
  LYAP_LAUNCHED("pcnet prep");
}

PcNetGpu::PcNetGpu(int nx, int ny, int nz, const double* dinv, SpdApply kapply, int C, hipStream_t st)
    : op_{}, kapply_(std::move(kapply)), C_(C), st_(st) {
  LYAP_REQUIRE(C == 2 || C == 4 || C == 8, LYAP_E_UNSUPPORTED, "network width C=%d not built (2, 4, 8)", C);
  LYAP_REQUIRE(nx > 0 && ny > 0 && nz > 0 && dinv && kapply_, LYAP_E_ARG, "bad network grid");
  nx_ = nx;
  ny_ = ny;
  nz_ = nz;
  n_ = nx * ny * nz;
  alloc_common();
  LYAP_HIP(hipMemcpyAsync(dinv_.p, dinv, (size_t)n_ * sizeof(double), hipMemcpyDeviceToDevice, st_));
  const int g = grid_for(n_, 1, 1024);
  hipLaunchKernelGGL(k_pc_prep_d1, dim3(g), dim3(kPcThreads), 0, st_, dinv_.as<double>(), n_, s_.as<float>(),
                     part_.as<double>());
  hipLaunchKernelGGL(k_pc_prep_d2, dim3(g), dim3(kPcThreads), 0, st_, dinv_.as<double>(), n_, part_.as<double>(), g,
                     f_.as<float>());
  LYAP_LAUNCHED("pcnet prep");
}

void PcNetGpu::alloc_common() {
  P_ = pcnet_param_count(C_);
  const size_t n = (size_t)n_;
  W_.alloc(P_ * sizeof(float));
  m_.alloc(P_ * sizeof(float));
  v_.alloc(P_ * sizeof(float));
  grad_.alloc(P_ * sizeof(double));
  LYAP_HIP(hipMemsetAsync(W_.p, 0, P_ * sizeof(float), st_));
  LYAP_HIP(hipMemsetAsync(m_.p, 0, P_ * sizeof(float), st_));
  LYAP_HIP(hipMemsetAsync(v_.p, 0, P_ * sizeof(float), st_));
  dinv_.alloc(n * sizeof(double));
  s_.alloc(n * sizeof(float));
  f_.alloc(n * sizeof(float));
  x0_.alloc(2 * n * sizeof(float));
  a1_.alloc(C_ * n * sizeof(float));
  k_.alloc(C_ * n * sizeof(float));
  t1_.alloc(C_ * n * sizeof(float));
  d_.alloc(2 * n * sizeof(float));
  part_.alloc((size_t)kWSeg * kPcMaxC * kPcMaxC * 27 * sizeof(double));
  loss_.alloc(64);
}

void PcNetGpu::set_weights(const float* host) {
  LYAP_HIP(hipMemcpyAsync(W_.p, host, P_ * sizeof(float), hipMemcpyHostToDevice, st_));
  LYAP_HIP(hipMemsetAsync(m_.p, 0, P_ * sizeof(float), st_));
  LYAP_HIP(hipMemsetAsync(v_.p, 0, P_ * sizeof(float), st_));
  LYAP_HIP(hipStreamSynchronize(st_));
  adam_t_ = 0;
}

void PcNetGpu::get_weights(float* host) const {
  LYAP_HIP(hipMemcpyAsync(host, W_.p, P_ * sizeof(float), hipMemcpyDeviceToHost, st_));
  LYAP_HIP(hipStreamSynchronize(st_));
}

template <int CI, int CO>
void PcNetGpu::conv(const float* in, const float* W, float* out) {
  if (nx_ % 4 == 0) {
    hipLaunchKernelGGL((k_pc_conv4<CI, CO, false>), dim3(xcd_grid((n_ / 4 + kPcThreads - 1) / kPcThreads)),
                       dim3(kPcThreads), 0, st_, in, W, out, nx_, ny_, nz_);
  } else {
    hipLaunchKernelGGL((k_pc_conv<CI, CO>), dim3(xcd_grid((n_ + kPcThreads - 1) / kPcThreads)), dim3(kPcThreads), 0,
                       st_, in, W, out, nx_, ny_, nz_);
  }
  LYAP_LAUNCHED("k_pc_conv");
}

template <int CO, int CI>
void PcNetGpu::convT(const float* in, const float* W, float* out) {
  if (nx_ % 4 == 0) {
    hipLaunchKernelGGL((k_pc_conv4<CI, CO, true>), dim3(xcd_grid((n_ / 4 + kPcThreads - 1) / kPcThreads)),
                       dim3(kPcThreads), 0, st_, in, W, out, nx_, ny_, nz_);
  } else {
    hipLaunchKernelGGL((k_pc_convT<CO, CI>), dim3(xcd_grid((n_ + kPcThreads - 1) / kPcThreads)), dim3(kPcThreads), 0,
                       st_, in, W, out, nx_, ny_, nz_);
  }
  LYAP_LAUNCHED("k_pc_convT");
}

template <int CI, int CO>
void PcNetGpu::wgrad(const float* x, const float* g, double* gradW, bool accumulate) {
  constexpr int E = CO * CI * 27;
  const dim3 grid((nx_ + kTX - 1) / kTX, (ny_ + kTY - 1) / kTY, (nz_ + kTZ - 1) / kTZ);
  const size_t ntiles = (size_t)grid.x * grid.y * grid.z;
  const size_t need = std::max(ntiles * E * sizeof(float), (size_t)kWSeg * E * sizeof(double));
  if (wpart_cap_ < need) {
    LYAP_HIP(hipStreamSynchronize(st_));
    wpart_.alloc(need);
    wpart_cap_ = need;
  }
  hipLaunchKernelGGL((k_pc_wgrad<CI, CO>), grid, dim3(kPcThreads), 0, st_, x, g, wpart_.as<float>(), nx_, ny_, nz_);
  // tile sums in two fixed-order passes (the first pass's output reuses the part_ scratch)
  const int per = (int)((ntiles + kWSeg - 1) / kWSeg);
  DevBuf& tmp = part_;
  LYAP_REQUIRE(tmp.bytes >= (size_t)kWSeg * E * sizeof(double), LYAP_E_UNSUPPORTED, "scratch too small");
  hipLaunchKernelGGL(k_pc_wreduce1, dim3((E + 63) / 64, kWSeg), dim3(256), 0, st_, wpart_.as<float>(),
                     (int)ntiles, E, per, tmp.as<double>());
  hipLaunchKernelGGL(k_pc_wreduce2, dim3((E + 63) / 64), dim3(256), 0, st_, tmp.as<double>(), kWSeg, E, gradW,
                     accumulate ? 1 : 0);
  LYAP_LAUNCHED("k_pc_wgrad");
}

#define LYAP_PC_SWITCH(...)                                   \
  switch (C_) {                                               \
    case 2: { constexpr int CC = 2; __VA_ARGS__; } break;     \
    case 4: { constexpr int CC = 4; __VA_ARGS__; } break;     \
    default: { constexpr int CC = 8; __VA_ARGS__; } break;    \
  }

void PcNetGpu::forward(const double* r) {
  const float* W1 = W_.as<float>();
  const float* W2 = W1 + C_ * 2 * 27;
  const int g = (n_ + kPcThreads - 1) / kPcThreads;
  hipLaunchKernelGGL(k_pc_in_r, dim3(g), dim3(kPcThreads), 0, st_, r, s_.as<float>(), f_.as<float>(), n_,
                     x0_.as<float>());
  LYAP_PC_SWITCH({
    conv<2, CC>(x0_.as<float>(), W1, a1_.as<float>());
    conv<CC, CC>(a1_.as<float>(), W2, k_.as<float>());
    convT<CC, CC>(k_.as<float>(), W2, t1_.as<float>());
    convT<CC, 2>(t1_.as<float>(), W1, d_.as<float>());
  });
}

int PcNetGpu::tiles() const {
  return ((nx_ + kQX - 1) / kQX) * ((ny_ + kQY - 1) / kQY) * ((nz_ + kQZ - 1) / kQZ);
}

int PcNetGpu::max_out_parts() const { return std::max(tiles(), stream_grid(n_)); }

int PcNetGpu::apply(const double* r, double* z, const double* q, double* part) {
  return launch_apply(r, nullptr, r, z, q, part);
}

int PcNetGpu::apply_upd(const PcUpd& u, double* z, const double* q, double* part) {
  LYAP_REQUIRE(u.r_out != u.r_in, LYAP_E_ARG, "fused update: r_out must not alias r_in");
  return launch_apply(nullptr, &u, u.r_out, z, q, part);
}

int PcNetGpu::launch_apply(const double* r_first, const PcUpd* up, const double* r_last, double* z, const double* q,
                           double* part) {
  const float* W1 = W_.as<float>();
  const float* W2 = W1 + C_ * 2 * 27;
  const int tx = (nx_ + kQX - 1) / kQX, ty = (ny_ + kQY - 1) / kQY, tz = (nz_ + kQZ - 1) / kQZ;
  const int G = tx * ty * tz;
  const dim3 grid(xcd_grid(G)), blk(kPcThreads);
  const float* fn = nullptr;
  float* fo = nullptr;
  const double* dn = nullptr;
  double* dno = nullptr;
  const PcUpd none{};
  LYAP_PC_SWITCH({
    if (up)
      hipLaunchKernelGGL((k_pc_tile<2, CC, false, 3>), grid, blk, 0, st_, fn, dn, s_.as<float>(), f_.as<float>(), dn,
                         W1, a1_.as<float>(), dno, dn, dno, nx_, ny_, nz_, tx, ty, tz, *up);
    else
      hipLaunchKernelGGL((k_pc_tile<2, CC, false, 1>), grid, blk, 0, st_, fn, r_first, s_.as<float>(), f_.as<float>(),
                         dn, W1, a1_.as<float>(), dno, dn, dno, nx_, ny_, nz_, tx, ty, tz, none);
    hipLaunchKernelGGL((k_pc_tile<CC, CC, false, 0>), grid, blk, 0, st_, a1_.as<float>(), dn, fn, fn, dn, W2,
                       k_.as<float>(), dno, dn, dno, nx_, ny_, nz_, tx, ty, tz, none);
    hipLaunchKernelGGL((k_pc_tile<CC, CC, true, 0>), grid, blk, 0, st_, k_.as<float>(), dn, fn, fn, dn, W2,
                       t1_.as<float>(), dno, dn, dno, nx_, ny_, nz_, tx, ty, tz, none);
    hipLaunchKernelGGL((k_pc_tile<2, CC, true, 2>), grid, blk, 0, st_, t1_.as<float>(), r_last, s_.as<float>(),
                       f_.as<float>(), dinv_.as<double>(), W1, fo, z, q, part, nx_, ny_, nz_, tx, ty, tz, none);
  });
  LYAP_LAUNCHED("pcnet apply");
  return G;
}

double PcNetGpu::energy(const double* e) {
  const int g = grid_for(n_, 1, 1024);
  if (kapply_) {
    if (!ky_.p) ky_.alloc((size_t)n_ * sizeof(double));
    kapply_(e, ky_.as<double>());
    hipLaunchKernelGGL(k_pc_dot, dim3(g), dim3(kPcThreads), 0, st_, e, ky_.as<double>(), n_, part_.as<double>());
  } else {
    hipLaunchKernelGGL(k_pc_energy, dim3(g), dim3(kPcThreads), 0, st_, op_, e, n_, part_.as<double>());
  }
  hipLaunchKernelGGL(k_pc_sum1, dim3(1), dim3(kPcThreads), 0, st_, part_.as<double>(), g, loss_.as<double>() + 1);
  double h = 0.0;
  LYAP_HIP(hipMemcpyAsync(&h, loss_.as<double>() + 1, sizeof(double), hipMemcpyDeviceToHost, st_));
  LYAP_HIP(hipStreamSynchronize(st_));
  return h;
}

double PcNetGpu::grad(const double* r, const double* e, double eAe, bool want_loss) {
  if (!z_.p) {
    const size_t n = (size_t)n_;
    z_.alloc(n * sizeof(double));
    gw_.alloc(n * sizeof(float));
    x0g_.alloc(2 * n * sizeof(float));
    a1g_.alloc(C_ * n * sizeof(float));
    kg_.alloc(C_ * n * sizeof(float));
    t2_.alloc(C_ * n * sizeof(float));
  }
  const float* W1 = W_.as<float>();
  const float* W2 = W1 + C_ * 2 * 27;
  double* g1 = grad_.as<double>();
  double* g2 = g1 + C_ * 2 * 27;
  forward(r);
  constexpr int NT = stream_threads(1);
  hipLaunchKernelGGL((k_pc_out<NT>), dim3(stream_grid(n_)), dim3(NT), 0, st_, r, dinv_.as<double>(), s_.as<float>(),
                     f_.as<float>(), d_.as<float>(), n_, z_.as<double>(), (const double*)nullptr, (double*)nullptr);
  const int gr = grid_for(n_, 1, 1024);
  if (kapply_) {
    if (!ky_.p) ky_.alloc((size_t)n_ * sizeof(double));
    if (!kd_.p) kd_.alloc((size_t)n_ * sizeof(double));
    hipLaunchKernelGGL(k_pc_sub, dim3((n_ + 255) / 256), dim3(256), 0, st_, z_.as<double>(), e, n_, kd_.as<double>());
    kapply_(kd_.as<double>(), ky_.as<double>());
    hipLaunchKernelGGL(k_pc_resid_k, dim3(gr), dim3(kPcThreads), 0, st_, kd_.as<double>(), ky_.as<double>(),
                       s_.as<float>(), eAe, n_, gw_.as<float>(), part_.as<double>());
  } else {
    hipLaunchKernelGGL(k_pc_resid, dim3(gr), dim3(kPcThreads), 0, st_, op_, z_.as<double>(), e, s_.as<float>(), eAe,
                       n_, gw_.as<float>(), part_.as<double>());
  }
  hipLaunchKernelGGL(k_pc_loss, dim3(1), dim3(kPcThreads), 0, st_, part_.as<double>(), gr, eAe, loss_.as<double>());
  const int g = (n_ + kPcThreads - 1) / kPcThreads;
  hipLaunchKernelGGL(k_pc_in_g, dim3(g), dim3(kPcThreads), 0, st_, gw_.as<float>(), f_.as<float>(), n_,
                     x0g_.as<float>());
  LYAP_LAUNCHED("pcnet loss");
  LYAP_PC_SWITCH({
    conv<2, CC>(x0g_.as<float>(), W1, a1g_.as<float>());
    conv<CC, CC>(a1g_.as<float>(), W2, kg_.as<float>());
    // dW2 = wgrad(a1, K gw) + wgrad(a1g, K u)
    wgrad<CC, CC>(a1_.as<float>(), kg_.as<float>(), g2, false);
    wgrad<CC, CC>(a1g_.as<float>(), k_.as<float>(), g2, true);
    // dW1 = wgrad(x0, conv2^T(K gw)) + wgrad(x0g, conv2^T(K u))  (conv2^T(K u) = t1 from forward)
    convT<CC, CC>(kg_.as<float>(), W2, t2_.as<float>());
    wgrad<2, CC>(x0_.as<float>(), t2_.as<float>(), g1, false);
    wgrad<2, CC>(x0g_.as<float>(), t1_.as<float>(), g1, true);
  });
  if (!want_loss) return 0.0;
  double h = 0.0;
  LYAP_HIP(hipMemcpyAsync(&h, loss_.p, sizeof(double), hipMemcpyDeviceToHost, st_));
  LYAP_HIP(hipStreamSynchronize(st_));
  return h;
}

void PcNetGpu::adam(double lr) {
  ++adam_t_;
  const float c1 = (float)(1.0 - std::pow(0.9, adam_t_));
  const float c2 = (float)(1.0 - std::pow(0.999, adam_t_));
  hipLaunchKernelGGL(k_pc_adam, dim3((P_ + 255) / 256), dim3(256), 0, st_, W_.as<float>(), grad_.as<double>(),
                     m_.as<float>(), v_.as<float>(), P_, (float)lr, c1, c2);
  LYAP_LAUNCHED("k_pc_adam");
}

}  // namespace lyap

// ------------------------------------------------------------------ C ABI (components)
extern "C" void lyap_pcnet_init(int32_t C, uint64_t seed, double scale, float* W) {
  if (!W || !(C == 2 || C == 4 || C == 8)) return;
  lyap::pcnet_init_weights(C, seed, scale, W);
}

extern "C" lyap_status lyap_pcnet_apply(const lyap_op* A, int32_t C, const float* W, const double* r, double* z,
                                        void* stream) {
  using namespace lyap;
  clear_error();
  try {
    validate_op(A);
    LYAP_REQUIRE(W && r && z, LYAP_E_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    OpHolder<double> op;
    make_op_f64(A, op, st);
    PcNetGpu net(op.dev, C, st);
    net.set_weights(W);
    net.apply(r, z, nullptr, nullptr);
    LYAP_HIP(hipStreamSynchronize(st));
    return LYAP_OK;
  } catch (const Error& e) {
    return e.st;
  }
}

extern "C" lyap_status lyap_pcnet_grad(const lyap_op* A, int32_t C, const float* W, const double* r, const double* e,
                                       double* loss, double* grad, void* stream) {
  using namespace lyap;
  clear_error();
  try {
    validate_op(A);
    LYAP_REQUIRE(W && r && e && loss && grad, LYAP_E_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    OpHolder<double> op;
    make_op_f64(A, op, st);
    PcNetGpu net(op.dev, C, st);
    net.set_weights(W);
    const double eAe = net.energy(e);
    LYAP_REQUIRE(eAe > 0.0, LYAP_E_ARG, "e^T (-A) e must be positive");
    *loss = net.grad(r, e, eAe, true);
    LYAP_HIP(hipMemcpyAsync(grad, net.grad_dev(), pcnet_param_count(C) * sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipStreamSynchronize(st));
    return LYAP_OK;
  } catch (const Error& e2) {
    return e2.st;
  }
}

extern "C" lyap_status lyap_pcnet_train(const lyap_op* A, int32_t C, float* W, int32_t npairs,
                                        const double* const* r, const double* const* e, int32_t steps, double lr,
                                        double* losses, void* stream) {
  using namespace lyap;
  clear_error();
  try {
    validate_op(A);
    LYAP_REQUIRE(W && r && e && npairs > 0 && steps >= 0, LYAP_E_ARG, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    OpHolder<double> op;
    make_op_f64(A, op, st);
    PcNetGpu net(op.dev, C, st);
    net.set_weights(W);
    std::vector<double> eAe(npairs);
    for (int i = 0; i < npairs; ++i) {
      eAe[i] = net.energy(e[i]);
      LYAP_REQUIRE(eAe[i] > 0.0, LYAP_E_ARG, "pair %d: e^T (-A) e must be positive", i);
    }
    for (int t = 0; t < steps; ++t) {
      const int i = t % npairs;
      const double L = net.grad(r[i], e[i], eAe[i], losses != nullptr);
      if (losses) losses[t] = L;
      net.adam(lr);
    }
    net.get_weights(W);
    return LYAP_OK;
  } catch (const Error& e2) {
    return e2.st;
  }
}

extern "C" lyap_status lyap_pcnet_fcg(const lyap_op* A, int32_t C, const float* W, const double* B, double* X,
                                      double eta, int32_t max_iter, int64_t* iters, double* relres, void* stream) {
  using namespace lyap;
  clear_error();
  try {
    validate_op(A);
    LYAP_REQUIRE(W && B && X, LYAP_E_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    OpHolder<double> op;
    make_op_f64(A, op, st);
    PcNetGpu net(op.dev, C, st);
    net.set_weights(W);
    InnerCG cg(op.dev, (int)A->n, 1, LYAP_PC_LEARNED, eta, max_iter, st);
    cg.set_net(&net);
    lyap_status status = LYAP_OK;
    try {
      cg.solve(B, X);
    } catch (const Error& e) {
      if (e.st != LYAP_E_INNER) throw;
      status = LYAP_E_INNER;
    }
    LYAP_HIP(hipStreamSynchronize(st));
    if (iters) *iters = cg.stats().iters;
    if (relres) *relres = cg.stats().worst_relres;
    return status;
  } catch (const Error& e2) {
    return e2.st;
  }
}

// ------------------------------------------------------------------ on the Schur complement
extern "C" lyap_status lyap_pcnet_schur_train(const lyap_op* A, int32_t C, float* W, const double* b, int32_t every,
                                              int32_t keep, int32_t steps, double lr, double* losses,
                                              int32_t* npairs, void* stream) {
  using namespace lyap;
  clear_error();
  try {
    validate_op(A);
    LYAP_REQUIRE(W && b && every > 0 && keep > 0 && steps >= 0, LYAP_E_ARG, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    OpHolder<double> op;
    make_op_f64(A, op, st);
    const int n = (int)A->n;
    InnerCG cg(op.dev, n, 1, LYAP_PC_LEARNED, 1e-12, 100000, st);
    auto net = cg.make_schur_net(C);
    net->set_weights(W);
    cg.harvest(every, keep);
    DevBuf x((size_t)n * sizeof(double));
    cg.solve(b, x.as<double>());
    std::vector<int> use;
    std::vector<double> eAe;
    for (int i = 0; i < cg.pairs(); ++i) {
      const double v = net->energy(cg.pair_e(i));
      if (v > 0.0) {
        use.push_back(i);
        eAe.push_back(v);
      }
    }
    LYAP_REQUIRE(!use.empty(), LYAP_E_INNER, "no training pairs");
    for (int t = 0; t < steps; ++t) {
      const int q = t % (int)use.size();
      const double L = net->grad(cg.pair_r(use[q]), cg.pair_e(use[q]), eAe[q], losses != nullptr);
      if (losses) losses[t] = L;
      net->adam(lr);
    }
    net->get_weights(W);
    if (npairs) *npairs = (int32_t)use.size();
    return LYAP_OK;
  } catch (const Error& e2) {
    return e2.st;
  }
}

extern "C" lyap_status lyap_pcnet_schur_fcg(const lyap_op* A, int32_t C, const float* W, const double* B, double* X,
                                            double eta, int32_t max_iter, int64_t* iters, double* relres,
                                            void* stream) {
  using namespace lyap;
  clear_error();
  try {
    validate_op(A);
    LYAP_REQUIRE(W && B && X, LYAP_E_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    OpHolder<double> op;
    make_op_f64(A, op, st);
    InnerCG cg(op.dev, (int)A->n, 1, LYAP_PC_LEARNED, eta, max_iter, st);
    auto net = cg.make_schur_net(C);
    net->set_weights(W);
    cg.set_net_schur(net.get());
    lyap_status status = LYAP_OK;
    try {
      cg.solve(B, X);
    } catch (const Error& e) {
      if (e.st != LYAP_E_INNER) throw;
      status = LYAP_E_INNER;
    }
    LYAP_HIP(hipStreamSynchronize(st));
    if (iters) *iters = cg.stats().iters;
    if (relres) *relres = cg.stats().worst_relres;
    return status;
  } catch (const Error& e2) {
    return e2.st;
  }
}

// ------------------------------------------------------------------ allocation-free apply
// Workspace of lyap_pcnet_apply_noalloc: one static device array per GPU (each
// device that loads this code object holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel: its device
// address, per device, comes from hipGetSymbolAddress on the first call made
// with that device current, and the buffers of the apply are slices of it.
namespace lyap {

constexpr size_t kNoAllocBytes = (size_t)32 << 20;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices] = {};

static char* scratch_base() {
  int dev = 0;
  LYAP_HIP(hipGetDevice(&dev));
  LYAP_REQUIRE(dev >= 0 && dev < kNoAllocMaxDevices, LYAP_E_DEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    LYAP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    LYAP_REQUIRE(p != nullptr, LYAP_E_DEVICE, "no device address for the workspace array");
    g_scratch_ptr[dev] = p;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

// Workspace bytes of one apply: the FP64 copies of a 7-point operator's four
// coefficient arrays (32 n), D^{-1} (8 n), s and f (8 n), the input channels
// and K^T's output (16 n), three C-channel activations (12 C n), and the
// weights, optimizer state and reduction partials (under 1 MiB), with the
// 256-byte alignment of every slice.
static size_t pcnet_noalloc_bytes(const lyap_op* A, int C) {
  const size_t n = (size_t)A->n;
  const size_t P = (size_t)pcnet_param_count(C);
  const size_t op = A->kind == LYAP_OP_STENCIL7 ? 32 * n : 0;
  const size_t fixed = 4 * P * sizeof(float) + P * sizeof(double) + (size_t)kWSeg * kPcMaxC * kPcMaxC * 27 *
                       sizeof(double) + 64 + 32 * 256;
  return op + (8 + 8 + 16) * n + 12 * (size_t)C * n + fixed;
}

}  // namespace lyap

extern "C" lyap_status lyap_pcnet_apply_noalloc(const lyap_op* A, int32_t C, const float* W, const double* r,
                                                double* z, void* stream) {
  using namespace lyap;
  clear_error();
  try {
    validate_op(A);
    LYAP_REQUIRE(W && r && z, LYAP_E_ARG, "NULL argument");
    LYAP_REQUIRE(A->kind == LYAP_OP_STENCIL5 || A->kind == LYAP_OP_STENCIL7, LYAP_E_UNSUPPORTED,
                 "the learned preconditioner needs a stencil operator (a grid)");
    LYAP_REQUIRE(C == 2 || C == 4 || C == 8, LYAP_E_UNSUPPORTED, "network width C=%d not built (2, 4, 8)", C);
    const size_t need = pcnet_noalloc_bytes(A, C);
    LYAP_REQUIRE(need <= kNoAllocBytes, LYAP_E_ARG,
                 "n=%lld with C=%d needs %zu bytes of workspace; the allocation-free apply has %zu",
                 (long long)A->n, C, need, kNoAllocBytes);
    hipStream_t st = (hipStream_t)stream;
    Arena arena{scratch_base(), kNoAllocBytes, 0};
    ArenaScope scope(&arena);
    OpHolder<double> op;
    make_op_f64(A, op, st);
    PcNetGpu net(op.dev, C, st);
    net.set_weights(W);
    net.apply(r, z, nullptr, nullptr);
    LYAP_HIP(hipStreamSynchronize(st));
    return LYAP_OK;
  } catch (const Error& e) {
    return e.st;
  }
}
