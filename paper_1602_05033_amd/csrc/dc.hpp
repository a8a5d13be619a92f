// Divide-and-conquer eigensolver for a symmetric band (block tridiagonal)
// matrix that returns all eigenvalues and only the first and last ell rows of
// the eigenvector matrix (what Proposition 1 needs).
#pragma once

#include "eig.hpp"

namespace lyap {

class DcWork {
 public:
  DcWork(int ell, hipStream_t st);
  ~DcWork();
  // band: device lower band, ld = ldb; outputs lam (k, ascending), F and L
  // (ell x k row-major: rows 0..ell-1 and k-ell..k-1 of Q).
  void run(const double* band, int ldb, int k, double* lam, double* F, double* L);

 private:
  struct Impl;
  Impl* impl_;
};

}  // namespace lyap
