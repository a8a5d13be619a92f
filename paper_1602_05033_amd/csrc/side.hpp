// One standard block Krylov space K_m(A, C) driven on the GPU: the operator,
// the start block C = V_1 gamma, the block Lanczos steps with their
// coefficient log and T_m band, the breakdown / non-finite flags, and the
// second pass that regenerates the basis from the log (Section 3.3) or the
// stored basis to accumulate Z = V_m M.  lyap_solve drives one side,
// sylv_solve two (Section 5.1).
#pragma once

#include <memory>
#include <vector>

#include "lanczos.hpp"
#include "solver.hpp"

namespace lyap {

template <typename T>
class LanczosSide {
 public:
  LanczosSide(const lyap_op* A, const double* C, int S, int64_t ldc, int max_iter, bool two_pass, hipStream_t st,
              KernelTimer* kt);
  // QR of C; sets beta = ||C||_F.  Throws on NaN / zero / rank-deficient C.
  void init();
  // One block Lanczos step (asynchronous).
  void step();
  // Device flags: first breakdown step (+1) and first non-finite step (+1).
  void read_flags(int* breakdown, int* nonfinite);
  // Z (n x t, column-major, ldz) = V_m Mrows for the first m blocks (Mrows:
  // m*S x t, row-major, device); adds the algorithmic bytes to *bytes_out.
  void accumulate_Z(int m, const double* Mrows, int t, double* Z, int64_t ldz, double* bytes_out);

  const double* band() const { return band_.as<double>(); }
  const int* flags_dev() const { return flags_.as<int>(); }
  const double* gamma_dev() const { return glog_.as<double>() + L_R * S_ * S_; }
  const double* tau_dev(int mm) const { return logb_.as<double>() + (size_t)(mm - 1) * LS_ + L_R * S_ * S_; }
  const double* gamma_host() const { return hglog_.data() + L_R * S_ * S_; }
  int m() const { return m_; }
  int n() const { return n_; }
  int S() const { return S_; }
  double beta() const { return beta_; }
  const OpHolder<T>& op() const { return op_; }

 private:
  const double* C_;
  int64_t ldc_;
  int n_, S_, maxit_;
  bool two_pass_;
  hipStream_t st_;
  KernelTimer* kt_;
  OpHolder<T> op_;
  size_t blk_, LS_;
  int grid_;
  DevBuf Vb0_, Vb1_, Wb_, zero_, logb_, glog_, band_, partA_, partB_, flags_;
  HostBuf hflags_;
  std::vector<double> hglog_;
  std::vector<DevBuf> stored_;
  T* Vprev_ = nullptr;
  T* Vcur_ = nullptr;
  int m_ = 0;
  double beta_ = 0.0;
};

}  // namespace lyap
