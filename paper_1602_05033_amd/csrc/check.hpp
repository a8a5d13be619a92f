// Residual check engine: eigendecomposition of the banded T_m (FP64 on the
// GPU), then the Proposition 1 sum; keeps lambda and g of the latest check for
// the finalisation.
#pragma once

#include "eig.hpp"

namespace lyap {

class Checker {
 public:
  Checker(int ell, int nt, hipStream_t st) : ell_(ell), nt_(nt), st_(st) {}
  // band: device, (ell+1) x k lower band (ld = ell+1), gamma: device ell x ell
  // row-major, tau: device nt x ell row-major.  Result lands in *dev_out.
  void run(const double* band, int k, const double* gamma, const double* tau, CheckOut* dev_out);
  // Eigenvalues, g = (E_1^T Q)^T gamma and W_m = (E_m^T Q)^T tau^T only (the
  // inputs of the Sylvester residual, which couples two such spaces).
  void prepare(const double* band, int k, const double* gamma, const double* tau);
  const double* Wm() const { return Wm_.as<double>(); }
  int nt() const { return nt_; }
  const double* lam() const { return lam_.as<double>(); }
  const double* g() const { return g_.as<double>(); }
  int k() const { return k_; }
  int ell() const { return ell_; }

 private:
  void ensure(int k);
  void eig_jacobi(const double* band, int k);
  void eig_dc(const double* band, int k);
  int ell_, nt_;
  hipStream_t st_;
  int k_ = 0, cap_ = 0;
  DevBuf lam_, F_, L_, g_, Wm_, part_, counter_;
  DevBuf dense_, Q_;
  int dense_cap_ = 0;
  void* dc_ = nullptr;  // divide-and-conquer workspace
 public:
  ~Checker();
};

// Truncated factor M = Q_m Y-check (k x t, row-major, device) from the latest
// check: pivoted Cholesky of Y~, eigen-truncation of its Gram matrix at eps,
// banded shifted solves.  Returns t.
int finalise_factor(const Checker& ck, const double* band, const double* gamma, double eps, DevBuf& M,
                    hipStream_t st);

// The same finalisation in steps, so that several problems (each on its own
// stream) can be finalised in turn by one host thread: pchol_launch() /
// pchol_read() advance the pivoted Cholesky (false / finished when done),
// launch_tail() queues the shifted solves and the assembly of M and returns
// t, finish() checks the solves' failure flag once the stream has completed.
class FinaliseJob {
 public:
  FinaliseJob(const Checker& ck, const double* band, const double* gamma, double eps, hipStream_t st);
  ~FinaliseJob();
  FinaliseJob(const FinaliseJob&) = delete;
  FinaliseJob& operator=(const FinaliseJob&) = delete;
  bool pchol_launch();
  void pchol_read();
  bool pchol_finished() const;
  int launch_tail(DevBuf& M);
  void finish();

 private:
  struct Impl;
  Impl* w_;
};

}  // namespace lyap
