// Sparse operator application for row-interleaved n x S blocks: row r of a
// block holds its S entries contiguously, so one row of V is one (or two)
// vector loads and a stencil reads each neighbour row once.
//
// The per-row arithmetic (op_row) is the single definition used by the first
// Lanczos pass, by the second pass that replays it and by lyap_op_apply, so
// that all three produce the same bits for the same input.
#pragma once

#include "common.hpp"

namespace lyap {

// Rows of workgroup wg_id in the kernels that apply the operator: one contiguous
// block of ceil(n / wg_cnt) rows, the blocks dealt so that the wg_cnt / 8
// workgroups the hardware places on one XCD (consecutive ids go round-robin
// over the 8 XCDs) hold adjacent blocks.  The rows r +- N a stencil reads then
// mostly come from the same XCD's L2 instead of being fetched again by another
// XCD (with rows dealt in a grid stride, each block was fetched about three
// times).
__device__ __forceinline__ void op_rows(int wg_id, int wg_cnt, int n, int& lo, int& hi) {
  const int blk = (wg_cnt % 8 == 0) ? (wg_id % 8) * (wg_cnt / 8) + wg_id / 8 : wg_id;
  const int64_t R = ((int64_t)n + wg_cnt - 1) / wg_cnt;
  lo = (int)min((int64_t)n, (int64_t)blk * R);
  hi = (int)min((int64_t)n, (int64_t)lo + R);
}

// One-dimensional launches of G workgroups of consecutive points: launched as
// 8 * ceil(G / 8) workgroups and renumbered so that the workgroups on one XCD
// take consecutive logical blocks (same reason as op_rows).  -1 for padding.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int per = (G + 7) / 8;
  const int lb = (b % 8) * per + b / 8;
  return lb < G ? lb : -1;
}
inline int xcd_grid(int G) { return (G + 7) / 8 * 8; }


// Device-side description of the operator; coefficient arrays are stored in the
// basis storage type T (converted once per solve).
template <typename T>
struct OpDev {
  int kind;            // LYAP_OP_*
  int nx, ny, nz;
  int n;
  T cc, co;            // stencil5 centre (shift included) / neighbour
  T shift;             // csr diagonal shift
  const T* diag;       // stencil7 (shift included)
  const T* tx;
  const T* ty;
  const T* tz;
  const int64_t* rowptr;
  const int32_t* col;
  const T* val;
};

// Rows are S*sizeof(T) bytes at a 256-byte aligned base: use 16- or 8-byte
// vector accesses when the row size allows it.
template <typename T, int S>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&v)[S]) {
  constexpr int B = S * (int)sizeof(T);
  if constexpr (B % 16 == 0) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
    for (int i = 0; i < B / 16; ++i) {
      uint4 x = q[i];
      __builtin_memcpy(reinterpret_cast<char*>(v) + 16 * i, &x, 16);
    }
  } else if constexpr (B % 8 == 0) {
    const uint2* q = reinterpret_cast<const uint2*>(p);
#pragma unroll
    for (int i = 0; i < B / 8; ++i) {
      uint2 x = q[i];
      __builtin_memcpy(reinterpret_cast<char*>(v) + 8 * i, &x, 8);
    }
  } else {
#pragma unroll
    for (int c = 0; c < S; ++c) v[c] = p[c];
  }
}

template <typename T, int S>
__device__ __forceinline__ void store_row(T* __restrict__ p, const T (&v)[S]) {
  constexpr int B = S * (int)sizeof(T);
  if constexpr (B % 16 == 0) {
    uint4* q = reinterpret_cast<uint4*>(p);
#pragma unroll
    for (int i = 0; i < B / 16; ++i) {
      uint4 x;
      __builtin_memcpy(&x, reinterpret_cast<const char*>(v) + 16 * i, 16);
      q[i] = x;
    }
  } else if constexpr (B % 8 == 0) {
    uint2* q = reinterpret_cast<uint2*>(p);
#pragma unroll
    for (int i = 0; i < B / 8; ++i) {
      uint2 x;
      __builtin_memcpy(&x, reinterpret_cast<const char*>(v) + 8 * i, 8);
      q[i] = x;
    }
  } else {
#pragma unroll
    for (int c = 0; c < S; ++c) p[c] = v[c];
  }
}

// store_row with non-temporal stores: for an output the same kernel never reads
// back (the standalone operator application), so it need not stay in L2.
template <typename T, int S>
__device__ __forceinline__ void store_row_nt(T* __restrict__ p, const T (&v)[S]) {
  constexpr int B = S * (int)sizeof(T);
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  if constexpr (B % 16 == 0) {
#pragma unroll
    for (int i = 0; i < B / 16; ++i) {
      u32x4 x;
      __builtin_memcpy(&x, reinterpret_cast<const char*>(v) + 16 * i, 16);
      __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(p) + i);
    }
  } else if constexpr (B % 8 == 0) {
#pragma unroll
    for (int i = 0; i < B / 8; ++i) {
      u32x2 x;
      __builtin_memcpy(&x, reinterpret_cast<const char*>(v) + 8 * i, 8);
      __builtin_nontemporal_store(x, reinterpret_cast<u32x2*>(p) + i);
    }
  } else {
#pragma unroll
    for (int c = 0; c < S; ++c) __builtin_nontemporal_store(v[c], p + c);
  }
}

template <typename T, int S>
__device__ __forceinline__ void axpy_row(T a, const T* __restrict__ p, T (&acc)[S]) {
  T v[S];
  load_row<T, S>(p, v);
#pragma unroll
  for (int c = 0; c < S; ++c) acc[c] = fma(a, v[c], acc[c]);
}

// w = (A v)_r, accumulated in T with a fixed order of terms; row i of the
// operand v is produced by ld(i, out) (a plain load for a stored block, or a
// value computed on the fly, e.g. a CG search direction).
template <typename T, int S, typename Load>
__device__ __forceinline__ void op_row_fn(const OpDev<T>& op, int r, Load&& ld, T (&w)[S]) {
  auto axpy = [&](T a, int i) {
    T v[S];
    ld(i, v);
#pragma unroll
    for (int c = 0; c < S; ++c) w[c] = fma(a, v[c], w[c]);
  };
  if (op.kind == LYAP_OP_STENCIL5) {
    const int nx = op.nx;
    const int j = r / nx;
    const int i = r - j * nx;
    T v[S];
    ld(r, v);
#pragma unroll
    for (int c = 0; c < S; ++c) w[c] = op.cc * v[c];
    if (j > 0) axpy(op.co, r - nx);
    if (i > 0) axpy(op.co, r - 1);
    if (i < nx - 1) axpy(op.co, r + 1);
    if (j < op.ny - 1) axpy(op.co, r + nx);
  } else if (op.kind == LYAP_OP_STENCIL7) {
    const int nx = op.nx, ny = op.ny;
    const int nxy = nx * ny;
    const int l = r / nxy;
    const int rem = r - l * nxy;
    const int j = rem / nx;
    const int i = rem - j * nx;
    T v[S];
    ld(r, v);
    const T d = op.diag[r];
#pragma unroll
    for (int c = 0; c < S; ++c) w[c] = d * v[c];
    if (l > 0) axpy(op.tz[r - nxy], r - nxy);
    if (j > 0) axpy(op.ty[r - nx], r - nx);
    if (i > 0) axpy(op.tx[r - 1], r - 1);
    if (i < nx - 1) axpy(op.tx[r], r + 1);
    if (j < ny - 1) axpy(op.ty[r], r + nx);
    if (l < op.nz - 1) axpy(op.tz[r], r + nxy);
  } else {  // CSR
    const int64_t b = op.rowptr[r];
    const int64_t e = op.rowptr[r + 1];
#pragma unroll
    for (int c = 0; c < S; ++c) w[c] = T(0);
    for (int64_t k = b; k < e; ++k) axpy(op.val[k], op.col[k]);
    if (op.shift != T(0)) axpy(op.shift, r);
  }
}

// w = (A V)_r for a stored row-interleaved block V.
template <typename T, int S>
__device__ __forceinline__ void op_row(const OpDev<T>& op, const T* __restrict__ V, int r, T (&w)[S]) {
  op_row_fn<T, S>(op, r, [&](int i, T (&v)[S]) { load_row<T, S>(V + (size_t)i * S, v); }, w);
}

// Diagonal entry A_rr (shift included).
template <typename T>
__device__ __forceinline__ T op_diag(const OpDev<T>& op, int r) {
  if (op.kind == LYAP_OP_STENCIL5) return op.cc;
  if (op.kind == LYAP_OP_STENCIL7) return op.diag[r];
  T d = op.shift;
  for (int64_t k = op.rowptr[r]; k < op.rowptr[r + 1]; ++k)
    if (op.col[k] == r) d += op.val[k];
  return d;
}

// Host side: an operator converted to storage type T on the device.
template <typename T>
struct OpHolder {
  OpDev<T> dev{};
  DevBuf diag, tx, ty, tz, val;
  int64_t nnz = 0;
  // Algorithmic bytes read per row for the coefficients (0 for stencil5).
  double coef_bytes_per_row() const {
    if (dev.kind == LYAP_OP_STENCIL7) return 4.0 * sizeof(T);
    if (dev.kind == LYAP_OP_CSR) return (double)nnz / dev.n * (sizeof(T) + 4) + 8;
    return 0.0;
  }
};

void make_op_f64(const lyap_op* A, OpHolder<double>& h, hipStream_t st);
void make_op_f32(const lyap_op* A, OpHolder<float>& h, hipStream_t st);
void validate_op(const lyap_op* A);

}  // namespace lyap
