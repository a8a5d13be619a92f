// Inner solves with A for the extended Krylov method: preconditioned
// conjugate gradients in FP64 on -A (symmetric positive definite), s right-
// hand sides at once (independent scalars per column), accepted only when the
// true relative residual ||b - A x|| / ||b|| is at most eta.
#pragma once

#include "lanczos.hpp"
#include "solver.hpp"

namespace lyap {

// Per-iteration scalars (device), written by workgroup 0 of the kernels.
struct CgIter {
  double rho[4];    // r^T z at the start of the iteration
  double rr[4];     // r^T r at the start of the iteration
  double sigma[4];  // p^T (-A) p
  double alpha[4];
};

struct CgStats {
  int64_t iters = 0;   // iterations over all solves (restarts included)
  int solves = 0;
  int restarts = 0;
  double worst_relres = 0.0;
  double ms = 0.0;
};

class PcNetGpu;

class InnerCG {
 public:
  // op: FP64 operator; S: right-hand sides per solve (1, 2 or 4); pc:
  // LYAP_PC_NONE, LYAP_PC_JACOBI, or LYAP_PC_LEARNED (Jacobi until a network
  // is attached with set_net, flexible CG with it afterwards; S = 1).
  InnerCG(const OpDev<double>& op, int n, int S, int pc, double eta, int max_iter, hipStream_t st);
  // X = A^{-1} B for row-interleaved n x S blocks (device).  Throws
  // Error{LYAP_E_INNER} when a column does not reach eta.
  void solve(const double* B, double* X, KernelTimer* kt = nullptr);
  const CgStats& stats() const { return stats_; }
  // Later solves use flexible CG with z = M(r) from the network.
  void set_net(PcNetGpu* net) { net_ = net; }
  // The next (Jacobi) solve keeps (r, x) every `every` iterations, at most
  // `keep` times; after it, pair(i) gives r_i and e_i = x* - x_i ((-A) e_i = r_i).
  void harvest(int every, int keep) { harvest_every_ = every; harvest_keep_ = keep; }
  int pairs() const { return (int)hr_.size(); }
  const double* pair_r(int i) const { return hr_[i].as<double>(); }
  const double* pair_e(int i) const { return hx_[i].as<double>(); }

 private:
  void solve_fcg(const double* B, double* X, KernelTimer* kt);
  OpDev<double> op_;
  int n_, S_, pc_, max_iter_;
  double eta_;
  hipStream_t st_;
  int grid_, cgrid_;
  DevBuf dinv_, r_, p0_, p1_, q_, partA_, partB_, log_, state_, tot_, flag_;
  HostBuf hlog_, htot_;
  CgStats stats_;
  PcNetGpu* net_ = nullptr;
  DevBuf z_, partZ_;
  DevBuf r1_, w0_, w1_, s0_, s1_;  // double-buffered r, w = K M r, s = K p of the single-reduction CG
  int harvest_every_ = 0, harvest_keep_ = 0;
  std::vector<DevBuf> hr_, hx_;
};

}  // namespace lyap
