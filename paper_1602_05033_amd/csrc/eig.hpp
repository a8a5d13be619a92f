// Launch interface of the FP64 eigen / residual / finalisation kernels.
#pragma once

#include "common.hpp"

namespace lyap {

// Result of one residual check, written by the device.
struct CheckOut {
  double res;      // ||R_m||_F (Proposition 1)
  double lam_max;  // largest Ritz value (>= 0 means A is not negative definite)
  double lam_min;
  double pad;
};

void launch_band_to_dense(const double* band, int ldb, int ell, int k, double* A, hipStream_t st);
void launch_jacobi(double* A, int64_t strideA, double* Q, int64_t strideQ, double* lam, int64_t strideL,
                   const int* nlist, int nfixed, int batch, hipStream_t st, int* sweeps = nullptr);
void launch_gw(const double* F, int64_t ldf, const double* L, int64_t ldl, int k, int ell, int nt,
               const double* gamma, const double* tau, double* g, double* Wm, hipStream_t st);
void launch_ctri_sum(const double* lam, const double* g, const double* Wm, int k, int ell, int nt, double* part,
                     unsigned* counter, CheckOut* out, hipStream_t st);
// Pivoted Cholesky of Y~ (k x k, generated from lambda and g); returns the
// number of columns formed (<= tmax).  Lc: k x tmax column-major, piv: tmax.
int run_pchol(const double* lam, const double* g, int k, int ell, double delta, int tmax, double* d, double* Lc,
              int* piv, hipStream_t st);
// The same factorisation driven step by step, so that the host can advance
// several of them (on different streams) in turn: launch_chunk() queues up to
// 32 pivot steps (for k <= 1024 the whole factorisation, one workgroup in one
// launch) and the copy of the state to host memory (false once finished);
// read() takes that state after the stream has passed the copy.
class PcholRun {
 public:
  PcholRun(const double* lam, const double* g, int k, int ell, double delta, int tmax, double* d, double* Lc,
           int* piv, hipStream_t st);
  ~PcholRun();
  PcholRun(const PcholRun&) = delete;
  PcholRun& operator=(const PcholRun&) = delete;
  bool launch_chunk();
  void read();
  bool finished() const;
  int t() const;

 private:
  struct Impl;
  Impl* w_;
};
void launch_gram_cols(const double* Lc, int k, int tp, double* G, hipStream_t st);
void launch_shift_solve(const double* band, int ldb, int ell, int k, const double* lam, const double* g,
                        const double* gamma, const int* piv, int tp, double* Lb, double* X, int* fail,
                        hipStream_t st);
// M (k x t, row-major) = X (k x tp, column-major) B (tp x t, row-major).
void launch_gemm_xb(const double* X, int k, int tp, const double* B, int t, double* M, hipStream_t st);
void launch_assemble_M(const double* Lc, int k, const int* piv, int tp, const double* Qg, int t, const double* X,
                       double* V1, double* B, double* M, hipStream_t st);

// Eigenvalues and first/last ell eigenvector rows of a symmetric band matrix
// (divide and conquer; see dc.hip).  F, L: ell x k row-major.
struct BandEig;

}  // namespace lyap
