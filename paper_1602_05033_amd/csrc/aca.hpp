// Low-rank truncation by cross approximation with complete pivoting (the
// Sylvester finalisations): E ~= E(:, J) E(I, J)^{-1} E(I, :), pivots taken
// until the Frobenius norm of the remaining Schur complement, which is exactly
// the approximation error, is at most eps.
#pragma once

#include "common.hpp"

namespace lyap {

// E: device, rows x cols row-major, overwritten by the Schur complements.
// I, J: allocated here, t row / column pivots.  Returns t (<= tmax).
int aca_cross(double* E, int rows, int cols, double eps, int tmax, DevBuf& I, DevBuf& J, hipStream_t st);

// Core W = E0(I, J) (t x t, E0 row-major with leading dimension lde) = L U in
// the pivot order; B1 = U^{-1}, B2 = L^{-T}, both t x t row-major (device).
void core_lu_explicit(const double* E0, int64_t lde, const int* I, const int* J, int t, double* B1, double* B2,
                      hipStream_t st);

}  // namespace lyap
