// Learned SPD preconditioner: forward (K, K^T), backward (weight gradients of
// the energy-norm loss), Adam, and the component entry points used by the
// tests.  See pcnet.hpp for the definition.
//
// Convolutions: the weights in LDS, neighbours read through the caches
// (channel counts are small: 2 -> C -> C, C <= 8); four consecutive cells per
// thread with vector loads when nx is a multiple of 4, else one per thread.  In
// the preconditioner's application (nx a multiple of 4) the input channels are
// formed inside the first convolution and the output z inside the last one,
// so the network costs four kernels.  Weight
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

// The first convolution with its two input channels x0 = [u, f u], u = s r
// (rounded to FP32), formed from r, s, f as they are read (k_pc_in_r and
// k_pc_conv4<2, CO, false> in one pass; the same values and order).
template <int CO>
__global__ __launch_bounds__(kPcThreads) void k_pc_conv4_r(const double* __restrict__ r, const float* __restrict__ s,
                                                           const float* __restrict__ f, const float* __restrict__ W,
                                                           float* __restrict__ out, int nx, int ny, int nz) {
  constexpr int CI = 2;
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
  float acc[CO][4];
#pragma unroll
  for (int o = 0; o < CO; ++o)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[o][k] = 0.f;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    const int zz = z + dz;
    if (zz < 0 || zz >= nz) continue;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = y + dy;
      if (yy < 0 || yy >= ny) continue;
      const size_t base = (size_t)zz * nxy + (size_t)yy * nx + x0;
      double rv[6];
      float sv[6], fv[6];
      {
        const double2 r01 = *reinterpret_cast<const double2*>(r + base);
        const double2 r23 = *reinterpret_cast<const double2*>(r + base + 2);
        const float4 s4 = *reinterpret_cast<const float4*>(s + base);
        const float4 f4 = *reinterpret_cast<const float4*>(f + base);
        rv[1] = r01.x; rv[2] = r01.y; rv[3] = r23.x; rv[4] = r23.y;
        sv[1] = s4.x; sv[2] = s4.y; sv[3] = s4.z; sv[4] = s4.w;
        fv[1] = f4.x; fv[2] = f4.y; fv[3] = f4.z; fv[4] = f4.w;
        const bool lo = x0 > 0, hi = x0 + 4 < nx;
        rv[0] = lo ? r[base - 1] : 0.0;
        sv[0] = lo ? s[base - 1] : 0.f;
        fv[0] = lo ? f[base - 1] : 0.f;
        rv[5] = hi ? r[base + 4] : 0.0;
        sv[5] = hi ? s[base + 4] : 0.f;
        fv[5] = hi ? f[base + 4] : 0.f;
      }
      float v[CI][6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const float u = (float)((double)sv[j] * rv[j]);
        v[0][j] = u;
        v[1][j] = fv[j] * u;
      }
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int t = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
#pragma unroll
        for (int c = 0; c < CI; ++c)
#pragma unroll
          for (int o = 0; o < CO; ++o) {
            const float w = sW[(o * CI + c) * 27 + t];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[o][k] = fmaf(w, v[c][1 + k + dx], acc[o][k]);
          }
      }
    }
  }
#pragma unroll
  for (int o = 0; o < CO; ++o) {
    float4 rr;
    rr.x = acc[o][0];
    rr.y = acc[o][1];
    rr.z = acc[o][2];
    rr.w = acc[o][3];
    *reinterpret_cast<float4*>(out + (size_t)o * n + p0) = rr;
  }
}

// The last transposed convolution (CO -> 2 channels, as k_pc_conv4<2, CO,
// true>) followed by the output of k_pc_out for the same four cells:
// z = dinv r + s (d0 + f d1), the two channels d kept in registers.  With q,
// one partial z.q per workgroup at index lb (pc_out_parts(n) partials).
template <int CO>
__global__ __launch_bounds__(kPcThreads) void k_pc_conv4_out(const float* __restrict__ in, const float* __restrict__ W,
                                                             const double* __restrict__ r,
                                                             const double* __restrict__ dinv,
                                                             const float* __restrict__ s, const float* __restrict__ f,
                                                             int nx, int ny, int nz, double* __restrict__ z,
                                                             const double* __restrict__ q, double* part) {
  constexpr int CI = 2;
  const int n = nx * ny * nz;
  const int nq = n / 4;
  const int lb = xcd_block(blockIdx.x, (nq + kPcThreads - 1) / kPcThreads);
  if (lb < 0) return;
  __shared__ float sW[CO * CI * 27];
  __shared__ double red[kPcThreads / 64];
  for (int e = threadIdx.x; e < CO * CI * 27; e += kPcThreads) sW[e] = W[e];
  __syncthreads();
  const int qd = lb * kPcThreads + threadIdx.x;
  double zq[1] = {0.0};
  if (qd < nq) {
    const int p0 = 4 * qd;
    const int nxy = nx * ny;
    const int zc = p0 / nxy, y = (p0 / nx) % ny, x0 = p0 % nx;
    float acc[CI][4];
#pragma unroll
    for (int i = 0; i < CI; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[i][k] = 0.f;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      const int zz = zc - dz;
      if (zz < 0 || zz >= nz) continue;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int yy = y - dy;
        if (yy < 0 || yy >= ny) continue;
        const size_t base = (size_t)zz * nxy + (size_t)yy * nx + x0;
        float v[CO][6];
#pragma unroll
        for (int c = 0; c < CO; ++c) {
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
#pragma unroll
          for (int c = 0; c < CO; ++c)
#pragma unroll
            for (int i = 0; i < CI; ++i) {
              const float w = sW[(c * CI + i) * 27 + t];
#pragma unroll
              for (int k = 0; k < 4; ++k) acc[i][k] = fmaf(w, v[c][1 + k - dx], acc[i][k]);
            }
        }
      }
    }
    const double2 r01 = *reinterpret_cast<const double2*>(r + p0);
    const double2 r23 = *reinterpret_cast<const double2*>(r + p0 + 2);
    const double2 d01 = *reinterpret_cast<const double2*>(dinv + p0);
    const double2 d23 = *reinterpret_cast<const double2*>(dinv + p0 + 2);
    const float4 s4 = *reinterpret_cast<const float4*>(s + p0);
    const float4 f4 = *reinterpret_cast<const float4*>(f + p0);
    const double rv[4] = {r01.x, r01.y, r23.x, r23.y};
    const double dv[4] = {d01.x, d01.y, d23.x, d23.y};
    const float sv[4] = {s4.x, s4.y, s4.z, s4.w};
    const float fv[4] = {f4.x, f4.y, f4.z, f4.w};
    double zv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double w = (double)acc[0][k] + (double)fv[k] * (double)acc[1][k];
      zv[k] = fma(dv[k], rv[k], (double)sv[k] * w);
    }
    *reinterpret_cast<double2*>(z + p0) = make_double2(zv[0], zv[1]);
    *reinterpret_cast<double2*>(z + p0 + 2) = make_double2(zv[2], zv[3]);
    if (q) {
      const double2 q01 = *reinterpret_cast<const double2*>(q + p0);
      const double2 q23 = *reinterpret_cast<const double2*>(q + p0 + 2);
      zq[0] = fma(zv[0], q01.x, zq[0]);
      zq[0] = fma(zv[1], q01.y, zq[0]);
      zq[0] = fma(zv[2], q23.x, zq[0]);
      zq[0] = fma(zv[3], q23.y, zq[0]);
    }
  }
  if (part) write_partial_at<1, kPcThreads>(zq, red, part, lb);
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
  P_ = pcnet_param_count(C);
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
  a1_.alloc(C * n * sizeof(float));
  k_.alloc(C * n * sizeof(float));
  t1_.alloc(C * n * sizeof(float));
  d_.alloc(2 * n * sizeof(float));
  part_.alloc((size_t)kWSeg * kPcMaxC * kPcMaxC * 27 * sizeof(double));
  loss_.alloc(64);
  const int g = grid_for(n_, 1, 1024);
  hipLaunchKernelGGL(k_pc_prep1, dim3(g), dim3(kPcThreads), 0, st_, op_, n_, dinv_.as<double>(), s_.as<float>(),
                     part_.as<double>());
  hipLaunchKernelGGL(k_pc_prep2, dim3(g), dim3(kPcThreads), 0, st_, op_, n_, part_.as<double>(), g, f_.as<float>());
  LYAP_LAUNCHED("pcnet prep");
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

void PcNetGpu::forward(const double* r, bool fused) {
  const float* W1 = W_.as<float>();
  const float* W2 = W1 + C_ * 2 * 27;
  const int g = (n_ + kPcThreads - 1) / kPcThreads;
  if (!fused) {
    hipLaunchKernelGGL(k_pc_in_r, dim3(g), dim3(kPcThreads), 0, st_, r, s_.as<float>(), f_.as<float>(), n_,
                       x0_.as<float>());
  }
  LYAP_PC_SWITCH({
    if (fused) {
      hipLaunchKernelGGL((k_pc_conv4_r<CC>), dim3(xcd_grid((n_ / 4 + kPcThreads - 1) / kPcThreads)),
                         dim3(kPcThreads), 0, st_, r, s_.as<float>(), f_.as<float>(), W1, a1_.as<float>(), nx_, ny_,
                         nz_);
      LYAP_LAUNCHED("k_pc_conv4_r");
    } else {
      conv<2, CC>(x0_.as<float>(), W1, a1_.as<float>());
    }
    conv<CC, CC>(a1_.as<float>(), W2, k_.as<float>());
    convT<CC, CC>(k_.as<float>(), W2, t1_.as<float>());
    if (!fused) convT<CC, 2>(t1_.as<float>(), W1, d_.as<float>());
  });
}

int PcNetGpu::max_out_parts() const { return std::max((n_ / 4 + kPcThreads - 1) / kPcThreads, stream_grid(n_)); }

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int PcNetGpu::apply(const double* r, double* z, const double* q, double* part) {
  const bool fused = nx_ % 4 == 0 && aligned16(r) && aligned16(z) && (!q || aligned16(q));
  forward(r, fused);
  if (fused) {
    // the last transposed convolution and the output in one kernel
    const float* W1 = W_.as<float>();
    LYAP_PC_SWITCH({
      hipLaunchKernelGGL((k_pc_conv4_out<CC>), dim3(xcd_grid((n_ / 4 + kPcThreads - 1) / kPcThreads)),
                         dim3(kPcThreads), 0, st_, t1_.as<float>(), W1, r, dinv_.as<double>(), s_.as<float>(),
                         f_.as<float>(), nx_, ny_, nz_, z, q, part);
    });
    LYAP_LAUNCHED("k_pc_conv4_out");
    return (n_ / 4 + kPcThreads - 1) / kPcThreads;
  }
  constexpr int NT = stream_threads(1);
  hipLaunchKernelGGL((k_pc_out<NT>), dim3(stream_grid(n_)), dim3(NT), 0, st_, r, dinv_.as<double>(), s_.as<float>(),
                     f_.as<float>(), d_.as<float>(), n_, z, q, part);
  LYAP_LAUNCHED("k_pc_out");
  return stream_grid(n_);
}

double PcNetGpu::energy(const double* e) {
  const int g = grid_for(n_, 1, 1024);
  hipLaunchKernelGGL(k_pc_energy, dim3(g), dim3(kPcThreads), 0, st_, op_, e, n_, part_.as<double>());
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
  forward(r, false);
  constexpr int NT = stream_threads(1);
  hipLaunchKernelGGL((k_pc_out<NT>), dim3(stream_grid(n_)), dim3(NT), 0, st_, r, dinv_.as<double>(), s_.as<float>(),
                     f_.as<float>(), d_.as<float>(), n_, z_.as<double>(), (const double*)nullptr, (double*)nullptr);
  const int gr = grid_for(n_, 1, 1024);
  hipLaunchKernelGGL(k_pc_resid, dim3(gr), dim3(kPcThreads), 0, st_, op_, z_.as<double>(), e, s_.as<float>(), eAe,
                     n_, gw_.as<float>(), part_.as<double>());
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
