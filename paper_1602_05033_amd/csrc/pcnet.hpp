// Learned preconditioner for the inner solves of the extended Krylov method:
//   M r = D^{-1} r + s * K^T(K(s * r)),  s = sqrt(D^{-1}),
//   K(u) = conv2(conv1([u, f u])),  f = log(-diag A) - mean,
// two 3x3x3 convolutions (2 -> C -> C channels, zero padding, no bias) on the
// operator's grid.  M is symmetric positive definite for any weights (zero
// weights give Jacobi).  Network tensors are FP32, channel-major [c][n]; the
// CG vectors stay FP64.  Trained with the energy-norm loss
// (M r - e)^T (-A) (M r - e) / e^T (-A) e on pairs harvested from the run's
// own Jacobi-PCG solve, by Adam, with this file's own forward, backward and
// optimizer kernels.
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

#include "lanczos.hpp"
#include "solver.hpp"

namespace lyap {

constexpr int kPcMaxC = 8;
inline int pcnet_param_count(int C) { return C * 2 * 27 + C * C * 27; }

// SplitMix64 initial weights, uniform in [-scale, scale): u = (top 53 bits) / 2^53.
void pcnet_init_weights(int C, uint64_t seed, double scale, float* W);

struct CgIter;

// The flexible CG update of one iteration fused into the first convolution of
// the next application: alpha = p.r / p.q from the partials pin (nparts
// pairs; 0 once r.r <= *state), x += alpha p, r_out = r_in - alpha q (r_in is
// read at every tile's halo, where the update is recomputed, so r_out must
// not alias it), the network applied to r_out, partial sums of
// r_out.r_out per tile into rr_part; log[it] receives p.q, p.r and alpha, and
// flag[1] = it + 1 when p.q <= 0 while active.
struct PcUpd {
  double* x;
  const double* r_in;
  double* r_out;
  const double* p;
  const double* q;
  CgIter* log;
  int it;
  const double* state;
  const double* pin;
  int nparts;
  double* rr_part;
  int* flag;
};

// y = K x for the symmetric positive definite matrix K of the system the
// network preconditions (device FP64 vectors on the network's grid, stream-ordered).
using SpdApply = std::function<void(const double* x, double* y)>;

class PcNetGpu {
 public:
  // op: FP64 stencil operator (5- or 7-point; its grid is the network's grid,
  // K = -A).
  PcNetGpu(const OpDev<double>& op, int C, hipStream_t st);
  // A network on an nx x ny x nz grid (x fastest) for a given K: dinv is the
  // diagonal part D^{-1} (device FP64, copied; 0 marks grid points outside
  // the system, which the network then leaves at zero) and kapply applies K
  // (used by energy() and grad()).
  PcNetGpu(int nx, int ny, int nz, const double* dinv, SpdApply kapply, int C, hipStream_t st);
  int C() const { return C_; }
  int n() const { return n_; }
  void set_weights(const float* host);
  void get_weights(float* host) const;
  // z = M r (device FP64 n-vectors).  With q != nullptr, also the partial
  // sums of z.q into part (at most max_out_parts() of them, in a fixed
  // order); returns how many were written.
  int apply(const double* r, double* z, const double* q, double* part);
  // The same with the flexible CG update fused in (see PcUpd): z = M r_out.
  // Returns the number of z.q partials, which equals that of the r.r partials.
  int apply_upd(const PcUpd& u, double* z, const double* q, double* part);
  int max_out_parts() const;
  int tiles() const;  // workgroups (and z.q partials) of one apply()
  // Algorithmic figures of one apply() (the four tiled kernels): FP32
  // multiply-adds x 2, and HBM bytes (r, s, f in; a1 out; a1 in, k out; k in,
  // t1 out; t1, r, D^{-1}, s, f, q in, z out).
  double apply_flops() const { return 2.0 * 27.0 * (4.0 * C_ + 2.0 * C_ * C_) * n_; }
  double apply_bytes() const { return (double)n_ * (56.0 + 24.0 * C_); }
  // Loss of the pair (r, e) (eAe = e^T (-A) e) and its gradient into the
  // device FP64 buffer grad (param_count values); the loss is left on the
  // device (loss_dev) and returned when want_loss (host sync).
  double grad(const double* r, const double* e, double eAe, bool want_loss);
  // One Adam step with the gradient of the last grad() call.
  void adam(double lr);
  // e^T K e on the device, returned to the host.
  double energy(const double* e);
  const double* dinv() const { return dinv_.as<double>(); }
  const double* grad_dev() const { return grad_.as<double>(); }

 private:
  template <int CI, int CO>
  void conv(const float* in, const float* W, float* out);
  template <int CO, int CI>
  void convT(const float* in, const float* W, float* out);
  template <int CI, int CO>
  void wgrad(const float* x, const float* g, double* gradW, bool accumulate);
  // x0 = [s r, f s r], a1, k = K(x0) and d = K^T k, kept for the weight gradients.
  void forward(const double* r);

  void alloc_common();
  int launch_apply(const double* r_first, const PcUpd* u, const double* r_last, double* z, const double* q,
                   double* part);
  OpDev<double> op_;
  SpdApply kapply_;   // set: K given by the caller (else K = -A of op_)
  int nx_, ny_, nz_, n_, C_, P_;
  hipStream_t st_;
  int adam_t_ = 0;
  DevBuf W_, m_, v_, grad_, dinv_, s_, f_;
  DevBuf x0_, a1_, k_, t1_, d_, x0g_, a1g_, kg_, t2_, z_, gw_;
  DevBuf part_, wpart_, loss_, ky_, kd_;
  size_t wpart_cap_ = 0;
};

}  // namespace lyap
