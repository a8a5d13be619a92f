// Residual check and finalisation drivers (host side of eig.hip / dc.hip).
#include <algorithm>
#include <cmath>

#include <cstring>
#include <memory>

#include "check.hpp"
#include "dc.hpp"

namespace lyap {

// dense Jacobi is used up to this size; larger T_m go through divide and conquer
constexpr int kDenseMax = 16;

Checker::~Checker() { delete static_cast<DcWork*>(dc_); }

void Checker::ensure(int k) {
  if (k <= cap_) return;
  // geometric growth by 4 from 1024 rows: each reallocation frees the old
  // buffers, and a free waits for the device
  int cap = std::max({k, cap_ * 4, 1024});
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

struct FinaliseJob::Impl {
  const Checker& ck;
  const double* band;
  const double* gamma;
  hipStream_t st;
  int k, ell, tmax, t = 0;
  DevBuf d, Lc, piv, Lb, X, fail, B;
  HostBuf hfail;
  std::unique_ptr<PcholRun> pc;
  Impl(const Checker& c) : ck(c) {}
};

FinaliseJob::FinaliseJob(const Checker& ck, const double* band, const double* gamma, double eps, hipStream_t st)
    : w_(new Impl(ck)) {
  Impl& w = *w_;
  w.band = band;
  w.gamma = gamma;
  w.st = st;
  w.k = ck.k();
  w.ell = ck.ell();
  w.tmax = std::min(w.k, 1024);
  w.d.alloc((size_t)w.k * sizeof(double));
  w.Lc.alloc((size_t)w.k * w.tmax * sizeof(double));
  w.piv.alloc((size_t)w.tmax * sizeof(int));
  // Y~ ~= L L^T with trace(Y~ - L L^T) <= eps, hence ||Y~ - L L^T||_F <= eps
  // (the error bound of the paper's eigenvalue truncation, at a rank at most a
  // few columns above it)
  w.pc = std::make_unique<PcholRun>(ck.lam(), ck.g(), w.k, w.ell, eps, w.tmax, w.d.as<double>(), w.Lc.as<double>(),
                                    w.piv.as<int>(), st);
}

FinaliseJob::~FinaliseJob() { delete w_; }

bool FinaliseJob::pchol_launch() { return w_->pc->launch_chunk(); }
void FinaliseJob::pchol_read() { w_->pc->read(); }
bool FinaliseJob::pchol_finished() const { return w_->pc->finished(); }

int FinaliseJob::launch_tail(DevBuf& M) {
  Impl& w = *w_;
  const int t = w.pc->t();
  w.t = t;
  if (t <= 0) {
    M.alloc(8);
    return 0;
  }
  LYAP_REQUIRE(t < w.tmax || w.tmax == w.k, LYAP_E_UNSUPPORTED, "truncation rank exceeds %d", w.tmax);
  // Q L = Q Y~(:, P) L_PP^{-T}, with Q Y~(:, p) from a banded shifted solve
  const int k = w.k, ell = w.ell;
  w.Lb.alloc((size_t)(ell + 1) * k * t * sizeof(double));
  w.X.alloc((size_t)k * t * sizeof(double));
  w.fail.alloc(sizeof(int) * 4);
  w.hfail.alloc(sizeof(int) * 4);
  std::memset(w.hfail.p, 0, sizeof(int) * 4);
  LYAP_HIP(hipMemsetAsync(w.fail.p, 0, sizeof(int) * 4, w.st));
  launch_shift_solve(w.band, ell + 1, ell, k, w.ck.lam(), w.ck.g(), w.gamma, w.piv.as<int>(), t, w.Lb.as<double>(),
                     w.X.as<double>(), w.fail.as<int>(), w.st);
  w.B.alloc((size_t)t * t * sizeof(double));
  M.alloc((size_t)k * t * sizeof(double));
  launch_assemble_M(w.Lc.as<double>(), k, w.piv.as<int>(), t, nullptr, t, w.X.as<double>(), nullptr, w.B.as<double>(),
                    M.as<double>(), w.st);
  LYAP_HIP(hipMemcpyAsync(w.hfail.p, w.fail.p, sizeof(int), hipMemcpyDeviceToHost, w.st));
  return t;
}

void FinaliseJob::finish() {
  Impl& w = *w_;
  if (w.t <= 0) return;
  LYAP_REQUIRE(*w.hfail.as<int>() == 0, LYAP_E_INDEFINITE, "shifted operator -(T + lambda I) not positive definite");
}

int finalise_factor(const Checker& ck, const double* band, const double* gamma, double eps, DevBuf& M,
                    hipStream_t st) {
  FinaliseJob job(ck, band, gamma, eps, st);
  while (job.pchol_launch()) {
    LYAP_HIP(hipStreamSynchronize(st));
    job.pchol_read();
  }
  const int t = job.launch_tail(M);
  LYAP_HIP(hipStreamSynchronize(st));
  job.finish();
  return t;
}

}  // namespace lyap
