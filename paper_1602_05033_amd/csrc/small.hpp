// Small dense FP64 helpers (S x S, row-major) used on the device by one
// thread: Cholesky with the positive-diagonal upper factor, triangular inverse
// and product.
#pragma once

#include "common.hpp"

namespace lyap {

// G = R^T R, R upper triangular with positive diagonal.  Returns the smallest
// pivot ratio d_i / G_ii (1 = orthogonal columns, 0 = dependent).
template <int S>
__device__ double chol_upper(const double* G, double* R) {
  double ratio = 1.0;
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) R[i * S + j] = 0.0;
  for (int i = 0; i < S; ++i) {
    double d = G[i * S + i];
    for (int k = 0; k < i; ++k) d -= R[k * S + i] * R[k * S + i];
    const double gi = G[i * S + i];
    const double r = gi > 0.0 ? d / gi : 0.0;
    if (!(r >= 0.0)) ratio = 0.0;
    else if (r < ratio) ratio = r;
    const double dd = d > 1e-300 ? d : 1e-300;
    const double rii = sqrt(dd);
    R[i * S + i] = rii;
    for (int j = i + 1; j < S; ++j) {
      double v = G[i * S + j];
      for (int k = 0; k < i; ++k) v -= R[k * S + i] * R[k * S + j];
      R[i * S + j] = v / rii;
    }
  }
  return ratio;
}

template <int S>
__device__ void inv_upper(const double* R, double* Ri) {
  for (int i = 0; i < S * S; ++i) Ri[i] = 0.0;
  for (int j = 0; j < S; ++j) {
    Ri[j * S + j] = 1.0 / R[j * S + j];
    for (int i = j - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int k = i; k < j; ++k) acc += Ri[i * S + k] * R[k * S + j];
      Ri[i * S + j] = -acc / R[j * S + j];
    }
  }
}

template <int S>
__device__ void mul_upper(const double* A, const double* B, double* C) {  // C = A B
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) {
      double acc = 0.0;
      for (int k = 0; k < S; ++k) acc += A[i * S + k] * B[k * S + j];
      C[i * S + j] = acc;
    }
}

// breakdown when a Cholesky pivot keeps less than this fraction of the
// squared column norm (the block is numerically rank deficient)
constexpr double kBreakdownRatio = 1e-14;

}  // namespace lyap
