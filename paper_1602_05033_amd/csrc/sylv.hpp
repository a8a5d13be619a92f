// Pieces of the two-sided Sylvester solver shared by its standard and
// extended Krylov drivers (Section 5.1).
#pragma once

#include "check.hpp"

namespace lyap {

// Corrected Algorithm 4 from two prepared checks (lambda, g, W of each space):
// ||R||_F into out->res.  ell: block size of T_m and J_m; nt: rows of the tau
// factors used (s for extended spaces, whose lower s rows vanish).
void launch_sylv_sum(const Checker& ca, const Checker& cb, int k, int ell, int nt, double* part, unsigned* counter,
                     CheckOut* out, hipStream_t st);

// Truncated factors of Y~ from the latest checks: Z1 = V_m M1, Z2 = U_m M2,
// M1, M2 k x t row-major (device).  Returns t.
int finalise_sylv(const Checker& ca, const Checker& cb, const double* bandA, const double* bandB,
                  const double* gamma1, const double* gamma2, int ell, double eps, DevBuf& M1, DevBuf& M2,
                  hipStream_t st);

// sylv_solve with method EXT: two extended Krylov spaces in lockstep.
lyap_status solve_sylv_ext(const lyap_op* A, const lyap_op* B, const double* C1, int64_t ldc1, const double* C2,
                           int64_t ldc2, int S, const lyap_opts& o, sylv_result* out);

}  // namespace lyap
