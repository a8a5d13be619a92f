// Residual check and finalisation drivers (host side of eig.hip / dc.hip).
#include <algorithm>
#include <cmath>

#include "check.hpp"
#include "dc.hpp"

namespace lyap {

// dense Jacobi is used up to this size; larger T_m go through divide and conquer
constexpr int kDenseMax = 16;

Checker::~Checker() { delete static_cast<DcWork*>(dc_); }

void Checker::ensure(int k) {
  if (k <= cap_) return;
  int cap = std::max(k, cap_ * 3 / 2);
  cap = (cap + 255) / 256 * 256;
  lam_.alloc((size_t)cap * sizeof(double));
  F_.alloc((size_t)cap * ell_ * sizeof(double));
  L_.alloc((size_t)cap * ell_ * sizeof(double));
  g_.alloc((size_t)cap * ell_ * sizeof(double));
  Wm_.alloc((size_t)cap * nt_ * sizeof(double));
  if (!part_.p) {
    part_.alloc(4096 * sizeof(double));
    counter_.alloc(64);
    LYAP_HIP(hipMemsetAsync(counter_.p, 0, 64, st_));
  }
  cap_ = cap;
}

void Checker::eig_jacobi(const double* band, int k) {
  if (k > dense_cap_) {
    dense_.alloc((size_t)k * k * sizeof(double));
    Q_.alloc((size_t)k * k * sizeof(double));
    dense_cap_ = k;
  }
  launch_band_to_dense(band, ell_ + 1, ell_, k, dense_.as<double>(), st_);
  launch_jacobi(dense_.as<double>(), 0, Q_.as<double>(), 0, lam_.as<double>(), 0, nullptr, k, 1, st_);
  // first / last ell rows of Q (row-major, eigenvector i in column i)
  LYAP_HIP(hipMemcpyAsync(F_.p, Q_.p, (size_t)ell_ * k * sizeof(double), hipMemcpyDeviceToDevice, st_));
  LYAP_HIP(hipMemcpyAsync(L_.p, Q_.as<double>() + (size_t)(k - ell_) * k, (size_t)ell_ * k * sizeof(double),
                          hipMemcpyDeviceToDevice, st_));
}

void Checker::eig_dc(const double* band, int k) {
  if (!dc_) dc_ = new DcWork(ell_, st_);
  static_cast<DcWork*>(dc_)->run(band, ell_ + 1, k, lam_.as<double>(), F_.as<double>(), L_.as<double>());
}

void Checker::prepare(const double* band, int k, const double* gamma, const double* tau) {
  ensure(k);
  k_ = k;
  if (k <= kDenseMax) eig_jacobi(band, k);
  else eig_dc(band, k);
  launch_gw(F_.as<double>(), k, L_.as<double>(), k, k, ell_, nt_, gamma, tau, g_.as<double>(), Wm_.as<double>(), st_);
}

void Checker::run(const double* band, int k, const double* gamma, const double* tau, CheckOut* dev_out) {
  prepare(band, k, gamma, tau);
  launch_ctri_sum(lam_.as<double>(), g_.as<double>(), Wm_.as<double>(), k, ell_, nt_, part_.as<double>(),
                  counter_.as<unsigned>(), dev_out, st_);
}

int finalise_factor(const Checker& ck, const double* band, const double* gamma, double eps, DevBuf& M,
                    hipStream_t st) {
  const int k = ck.k();
  const int ell = ck.ell();
  const int tmax = std::min(k, 1024);
  DevBuf d((size_t)k * sizeof(double));
  DevBuf Lc((size_t)k * tmax * sizeof(double));
  DevBuf piv((size_t)tmax * sizeof(int));
  // Y~ ~= L L^T with trace(Y~ - L L^T) <= eps, hence ||Y~ - L L^T||_F <= eps
  // (the error bound of the paper's eigenvalue truncation, at a rank at most a
  // few columns above it)
  const int t = run_pchol(ck.lam(), ck.g(), k, ell, eps, tmax, d.as<double>(), Lc.as<double>(), piv.as<int>(), st);
  if (t <= 0) {
    M.alloc(8);
    return 0;
  }
  LYAP_REQUIRE(t < tmax || tmax == k, LYAP_E_UNSUPPORTED, "truncation rank exceeds %d", tmax);
  // Q L = Q Y~(:, P) L_PP^{-T}, with Q Y~(:, p) from a banded shifted solve
  DevBuf Lb((size_t)(ell + 1) * k * t * sizeof(double));
  DevBuf X((size_t)k * t * sizeof(double));
  DevBuf fail(sizeof(int) * 4);
  LYAP_HIP(hipMemsetAsync(fail.p, 0, sizeof(int) * 4, st));
  launch_shift_solve(band, ell + 1, ell, k, ck.lam(), ck.g(), gamma, piv.as<int>(), t, Lb.as<double>(),
                     X.as<double>(), fail.as<int>(), st);
  DevBuf B((size_t)t * t * sizeof(double));
  M.alloc((size_t)k * t * sizeof(double));
  launch_assemble_M(Lc.as<double>(), k, piv.as<int>(), t, nullptr, t, X.as<double>(), nullptr, B.as<double>(),
                    M.as<double>(), st);
  int hfail = 0;
  LYAP_HIP(hipMemcpyAsync(&hfail, fail.p, sizeof(int), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  LYAP_REQUIRE(hfail == 0, LYAP_E_INDEFINITE, "shifted operator -(T + lambda I) not positive definite");
  return t;
}

}  // namespace lyap
