// Inner solves with A for the extended Krylov method: preconditioned
// conjugate gradients in FP64 on -A (symmetric positive definite), s right-
// hand sides at once (independent scalars per column), accepted only when the
// true relative residual ||b - A x|| / ||b|| is at most eta.
#pragma once
#include <algorithm>

#include <memory>

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
  // LYAP_PC_NONE, LYAP_PC_JACOBI, LYAP_PC_IC0 (red-black IC(0), run as CG on
  // the black Schur complement; stencil operators only, rbcg.hip), or
  // LYAP_PC_LEARNED (Jacobi until a network is attached with set_net,
  // flexible CG with it afterwards; S = 1).
  InnerCG(const OpDev<double>& op, int n, int S, int pc, double eta, int max_iter, hipStream_t st);
  // X = A^{-1} B for row-interleaved n x S blocks (device).  Throws
  // Error{LYAP_E_INNER} when a column does not reach eta.
  void solve(const double* B, double* X, KernelTimer* kt = nullptr);
  const CgStats& stats() const { return stats_; }
  // Algorithmic HBM bytes of one iteration kernel (LYAP_K_CG_DIR) of this
  // preconditioner's CG.
  double iter_bytes() const;
  // ... and of the second kernel (LYAP_K_CG_UPD) where an iteration has two
  // (IC(0): the Schur product sweep; the learned preconditioner's FCG update).
  double upd_bytes() const;
  // Later solves use flexible CG with z = M(r) from the network (on the
  // operator's whole grid, K = -A).
  void set_net(PcNetGpu* net) { net_ = net; net_schur_ = false; pred_ = marg_ = 0; }
  // Later solves use flexible CG on the black Schur complement of the
  // red-black split (IC(0)'s condensed system) with z = M(r) from a network
  // made by make_schur_net (LYAP_PC_LEARNED on a stencil operator, S = 1).
  void set_net_schur(PcNetGpu* net) { net_ = net; net_schur_ = true; pred_ = marg_ = 0; }
  // A network on the compact grid of the black cells whose diagonal part is
  // diag(Sigma)^{-1} (zero weights: IC(0) itself) and whose K is Sigma.
  std::unique_ptr<PcNetGpu> make_schur_net(int C);
  // y = Sigma x on the compact black slots (S = 1; IC(0) or LEARNED on a stencil).
  void schur_apply(const double* x, double* y);
  // The next solve keeps (r, x) every `every` iterations, at most `keep`
  // times; after it, pair(i) gives r_i and e_i = x* - x_i (K e_i = r_i) --
  // for the Jacobi iteration on the whole grid (K = -A), for IC(0) and
  // LEARNED on a stencil in compact black-slot layout (K = Sigma).
  void harvest(int every, int keep) { harvest_every_ = every; harvest_keep_ = keep; }
  int pairs() const { return (int)hr_.size(); }
  const double* pair_r(int i) const { return hr_[i].as<double>(); }
  const double* pair_e(int i) const { return hx_[i].as<double>(); }

 private:
  void solve_fcg(const double* B, double* X, KernelTimer* kt);
  void setup_rb();
  void solve_rb(const double* B, double* X, KernelTimer* kt);
  void solve_rb_fcg(const double* B, double* X, KernelTimer* kt);
  template <bool K7, int S>
  void rb_solve_templ(const double* B, double* X, int restarts, int chunk, KernelTimer* kt);
  // true residual of X = A^{-1} B into rt_ and its totals towards htotT_,
  // queued behind a chunk that is expected to end the solve
  void spec_true(const double* B, const double* X);
  double rb_iter_bytes() const;
  double rb_w_bytes() const;
  OpDev<double> op_;
  int n_, S_, pc_, max_iter_;
  double eta_;
  hipStream_t st_;
  int grid_, cgrid_;
  DevBuf dinv_, r_, p0_, p1_, q_, partA_, partB_, log_, state_, tot_, flag_;
  HostBuf hlog_, htot_;
  CgStats stats_;
  PcNetGpu* net_ = nullptr;
  DevBuf z_, partZ_, partRR_;
  // the speculative true residual (its own vector, partials and totals, so
  // that the iteration state is not touched)
  DevBuf rt_, partT_, totT_;
  HostBuf htotT_;
  DevBuf r1_, w0_, w1_, s0_, s1_;  // double-buffered r, w = K M r, s = K p of the single-reduction CG
  int harvest_every_ = 0, harvest_keep_ = 0;
  // iterations of the last solve that converged without a restart: the next
  // solve's first host check is placed just after it plus a margin (the
  // right-hand sides of consecutive solves are alike, and a host round trip
  // costs more than a few iterations), later checks every few iterations.
  // Iterations past convergence are masked (they leave x unchanged) but cost
  // as much as the others, so the margin adapts: one less after a first chunk
  // that sufficed with room to spare (down to one, the least that still sees
  // convergence at the predicted count), twice as many after one that did not
  // (at most `tail`).  The chunking changes no result.
  int pred_ = 0, marg_ = 0;
  int margin(int tail) const { return marg_ > 0 ? marg_ : std::max(1, tail / 2); }
  int chunk_len(int it, int nchk, int base, int tail) const {
    if (pred_ <= 0) return base;
    if (it == 0) return pred_ + margin(tail);
    return tail << std::min(nchk - 1, 3);
  }
  // after a solve without a restart that converged after `it` iterations in
  // `nchk` chunks (`chunked`: the chunks came from chunk_len)
  void learn_pred(int it, int nchk, int tail, bool chunked) {
    if (pred_ > 0 && chunked) {
      const int m = margin(tail);
      marg_ = nchk == 1 ? (pred_ + m - it > 1 ? std::max(1, m - 1) : m) : std::min(tail, 2 * m);
    }
    pred_ = it;
  }
  // red-black IC(0): 1 / D_r (red slots), D_b and 1 / Sigma_bb (black slots),
  // the condensed iteration's vectors (r, w, s double buffered), u at the
  // black slots and v = D_r^{-1} E^T u at the red slots
  DevBuf rb_rinv_, rb_db_, rb_sinv_, rb_x_, rb_p_, rb_r0_, rb_r1_, rb_w0_, rb_w1_, rb_s0_, rb_s1_, rb_u_, rb_v_;
  int rb_grid_ = 0;
  bool rb_ready_ = false, net_schur_ = false;
  std::vector<DevBuf> hr_, hx_;
};

// r = A x - B for row-interleaved n x S blocks; tot[0..S) = r^T r and
// tot[S..2S) = B^T B per column (part: grid * 2S partial sums).
void cg_true(const OpDev<double>& op, const double* B, const double* x, double* r, int n, int S, double* part,
             double* tot, int grid, hipStream_t st);

}  // namespace lyap
