// Shared host-side pieces of the solvers.
#pragma once

#include <chrono>
#include <utility>
#include <vector>

#include "common.hpp"

namespace lyap {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0);

// When to evaluate the residual (Algorithm 1 step 6 is skipped in between).
// d > 0: every d steps (the paper's periodic check).  d == 0: adaptive —
// spaced checks growing geometrically (x1.5), then, once two checks give a
// log-linear trend, a jump to the predicted crossing of tol (never farther
// than the geometric step).
struct CheckSchedule {
  int d;
  int max_iter;
  // adaptive schedule (d = 0): the next check is at most grow * m steps
  // ahead, and aim times the predicted distance to the tolerance crossing
  double grow = 0.5;
  double aim = 1.0;
  std::vector<std::pair<int, double>> hist;
  int first() const;
  int next(int m, double res, double tol);
};

void store_history(lyap_result* out, const std::vector<int>& hm, const std::vector<double>& hr);
double* alloc_output(const lyap_opts& o, size_t bytes, bool* owned);
void rowmajor_to_colmajor(const double* rm, int rows, int cols, double* cm);
struct KernelTimer;
template <typename T>
void fill_kernel_bytes(int n, int S, double coef, const KernelTimer& kt, double zflush_bytes, double* kb);

template <typename T>
lyap_status solve_std(const lyap_op* A, const double* C, int S, int64_t ldc, const lyap_opts& o, lyap_result* out);
template <typename T>
lyap_status solve_ext(const lyap_op* A, const double* C, int S, int64_t ldc, const lyap_opts& o, lyap_result* out);

}  // namespace lyap
