/*
 * lyap.h — C ABI of the MI355X (gfx950) projection solver for
 *
 *     A X + X A + C C^T = 0           (Lyapunov)
 *     A X + X B + C1 C2^T = 0         (Sylvester, symmetric A and B)
 *
 * with A, B large, sparse, symmetric negative definite and C tall (n x s,
 * s << n), following Palitta & Simoncini, "Computationally enhanced
 * projection methods for symmetric Sylvester and Lyapunov matrix equations":
 * Galerkin projection onto block Krylov spaces (Section 2, Algorithm 1),
 * block Lanczos with twice-applied block modified Gram-Schmidt
 * (Algorithm 2), the residual norm of Proposition 1 / Algorithm 3 computed
 * from the eigendecomposition of the block tridiagonal T_m without solving
 * the reduced equation, the two-pass reconstruction of the low-rank factor
 * Z (Section 3.3, eq. (twopasseq)), the extended Krylov variant (Section 4)
 * and the two-sided Sylvester variant (Section 5.1, Algorithm 4).
 *
 * Conventions
 *  - All pointers named "device" are HIP device pointers on the current
 *    device; the library never dereferences them on the host.
 *  - Dense n x s inputs are column-major FP64 with leading dimension ld >= n.
 *  - Every entry point returns a lyap_status and never aborts; on error
 *    lyap_last_error() gives a thread-local, human-readable message.
 *  - Inputs are borrowed for the duration of a call.  The library keeps no
 *    state between calls.
 *  - Work is enqueued on opts->stream (a hipStream_t; NULL = the null
 *    stream); solver entry points synchronise that stream before returning.
 */
#ifndef LYAP_H
#define LYAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef enum lyap_status {
  LYAP_OK = 0,               /* converged: ||R||_F / beta^2 <= tol            */
  LYAP_NOT_CONVERGED = 1,    /* max_iter reached; Z is from the last check     */
  LYAP_E_ARG = -1,           /* invalid argument (message says which)          */
  LYAP_E_BREAKDOWN = -2,     /* a block W loses rank with the residual still
                                above tol (C itself is deflated by lyap_solve) */
  LYAP_E_INDEFINITE = -3,    /* a Ritz value >= 0: A is not negative definite  */
  LYAP_E_NUMERIC = -4,       /* NaN/Inf met (input or arithmetic)              */
  LYAP_E_INNER = -5,         /* an inner solve (extended Krylov) failed        */
  LYAP_E_NOMEM = -6,         /* device allocation failed                       */
  LYAP_E_DEVICE = -7,        /* a HIP runtime call failed                      */
  LYAP_E_UNSUPPORTED = -8    /* combination of options not built               */
} lyap_status;

/* ------------------------------------------------------------------ operator */
enum {
  LYAP_OP_CSR = 0,       /* general sparse symmetric matrix in CSR          */
  LYAP_OP_STENCIL5 = 1,  /* constant 5-point operator on an nx x ny grid    */
  LYAP_OP_STENCIL7 = 2   /* variable 7-point operator on nx x ny x nz cells */
};

/*
 * A sparse symmetric negative definite operator.  Grid rows are ordered
 * lexicographically with x fastest: row = i + nx*(j + ny*l).
 *
 * STENCIL5: (A v)_r = cc v_r + co (v_{r-1} + v_{r+1} + v_{r-nx} + v_{r+nx}),
 *           neighbours outside the grid omitted (zero Dirichlet boundary).
 *           n = nx*ny.
 * STENCIL7: per-cell device arrays diag, tx, ty, tz (length n, FP64):
 *           (A v)_r = diag_r v_r + tx_r v_{r+1} + tx_{r-1} v_{r-1}
 *                   + ty_r v_{r+nx} + ty_{r-nx} v_{r-nx}
 *                   + tz_r v_{r+nx*ny} + tz_{r-nx*ny} v_{r-nx*ny};
 *           the coupling arrays are zero on the last cell of a line.
 *           n = nx*ny*nz (nz = 1 for a 2-D grid).
 * CSR:      device rowptr (int64, n+1), colind (int32, nnz, ascending within
 *           a row), val (FP64, nnz).  The matrix must be symmetric.
 * shift:    added to the diagonal of every kind (A + shift I).
 */
typedef struct lyap_op {
  int32_t kind;
  int32_t nx, ny, nz;
  int64_t n;
  double cc, co;
  const double* diag;
  const double* tx;
  const double* ty;
  const double* tz;
  const int64_t* rowptr;
  const int32_t* colind;
  const double* val;
  int64_t nnz;
  double shift;
} lyap_op;

/* ------------------------------------------------------------------ options */
enum { LYAP_STORE_F64 = 0, LYAP_STORE_F32 = 1 };
enum { LYAP_METHOD_STD = 0, LYAP_METHOD_EXT = 1 };
enum { LYAP_PC_NONE = 0, LYAP_PC_JACOBI = 1, LYAP_PC_IC0 = 2, LYAP_PC_LEARNED = 3 };

typedef void* (*lyap_alloc_fn)(size_t bytes, void* ctx);
typedef void (*lyap_free_fn)(void* ptr, void* ctx);

typedef struct lyap_opts {
  double tol;           /* stop when ||R_m||_F / ||C||_F^2 <= tol (Alg. 1 step 6.3) */
  int32_t max_iter;     /* maximum number of basis blocks m                          */
  int32_t method;       /* LYAP_METHOD_STD (block Lanczos) or LYAP_METHOD_EXT          */
  int32_t check_every;  /* d > 0: check every d steps (the paper's d); 0: adaptive      */
  int32_t storage;      /* LYAP_STORE_F64 or LYAP_STORE_F32 (basis and SpMM storage;
                           coefficients, T_m, eigen and residual are always FP64)      */
  int32_t two_pass;     /* 1: regenerate the basis in a second pass (Section 3.3);
                           0: store the whole basis (memory s*m vectors)               */
  double trunc_eps;     /* < 0: default truncation threshold (see lyap_solve);
                           >= 0: absolute threshold on ||Sigma_2||_F               */
  int32_t inner_pc;     /* extended Krylov inner CG preconditioner: LYAP_PC_NONE,
                           LYAP_PC_JACOBI, LYAP_PC_IC0 (zero fill-in incomplete
                           Cholesky in red-black order; stencil operators only,
                           see lyap_inner_solve) or LYAP_PC_LEARNED (see below) */
  double inner_tol;     /* inner solves accepted when true ||b-Ax||/||b|| <= this  */
  int32_t inner_max_iter;
  int32_t flush_blocks; /* second pass: blocks buffered per Z update (0 = default)  */
  void* stream;         /* hipStream_t                                              */
  lyap_alloc_fn alloc;  /* device allocator for returned buffers (NULL: hipMalloc)  */
  lyap_free_fn release; /* matching release (NULL: hipFree)                         */
  void* alloc_ctx;
  int32_t want_T;       /* 1: return T_m band and gamma/tau on the host            */
  int32_t verbose;
  int32_t profile;      /* 1: time every kernel of the two passes with HIP events on
                           the stream (small overhead); see lyap_result.kern_ms */
} lyap_opts;

/* Fills *o with: tol 1e-8, max_iter 5000, STD, adaptive checks, F64 storage,
 * two_pass 1, default truncation, inner PC Jacobi, inner_tol 1e-12,
 * inner_max_iter 5000, hipMalloc allocation, null stream. */
void lyap_opts_default(lyap_opts* o);

/* ------------------------------------------------------------------ result */
enum {
  LYAP_T_PASS1 = 0,    /* basis generation (first pass), ms               */
  LYAP_T_CHECKS = 1,   /* residual checks (eigen + Prop. 1 sum), ms        */
  LYAP_T_FINAL = 2,    /* truncation and Q Y-check, ms                      */
  LYAP_T_PASS2 = 3,    /* second pass and Z accumulation, ms               */
  LYAP_T_INNER = 4,    /* inner solves (extended Krylov), ms               */
  LYAP_T_TRAIN = 5,    /* preconditioner training, ms                      */
  LYAP_T_TOTAL = 6,    /* whole call, ms                                   */
  LYAP_T_TO_TOL = 7    /* entry to the first passing check, ms            */
};

/* kernel kinds of lyap_result.kern_ms */
enum {
  LYAP_K_SPMM_GRAM = 0,  /* W = A V_j fused with the first block Gram product  */
  LYAP_K_UPD_GRAM = 1,   /* block MGS update fused with the next Gram product  */
  LYAP_K_CHOL_GRAM = 2,  /* Cholesky of W^T W and the second Gram product      */
  LYAP_K_CHOL_STORE = 3, /* second Cholesky, V_{j+1} = W R^{-1}                */
  LYAP_K_REPLAY = 4,     /* second pass: one whole step from the log            */
  LYAP_K_ZFLUSH = 5,     /* Z += V_i M_i for a group of buffered blocks         */
  LYAP_K_CHECK = 6,      /* one residual check (all its kernels)                */
  LYAP_K_FINAL = 7,      /* truncation and Q Y-check (all its kernels)          */
  LYAP_K_INIT = 8,       /* QR of C                                             */
  LYAP_K_CG_DIR = 9,     /* inner CG: new direction fused with q = -A p         */
  LYAP_K_CG_UPD = 10,    /* inner CG: x, r update and the next dot products     */
  LYAP_K_EXT_ORTH = 11,  /* extended Krylov: full reorthogonalisation + QR + T  */
  LYAP_K_PCNET = 12,     /* inner CG: one application of the learned network    */
  LYAP_K_COUNT = 16      /* size of the per-kind arrays (kinds 13..15 unused)   */
};

typedef struct lyap_result {
  int32_t status;
  int32_t s;           /* block width of C                                 */
  int32_t ell;         /* block size of T_m: s (standard) or 2s (extended) */
  int32_t m;           /* number of basis blocks (dim = ell*m)             */
  int32_t t;           /* columns of Z                                     */
  int64_t n;
  double* Z;           /* device, n x t column-major FP64, owned by caller
                          (allocated with opts->alloc, else hipMalloc)     */
  int32_t n_hist;
  int32_t* hist_m;     /* host: m at each check                            */
  double* hist_res;    /* host: ||R_m||_F / beta^2 at each check            */
  double beta;         /* ||C||_F                                          */
  double res;          /* last checked ||R_m||_F / beta^2                  */
  double trunc_eps;    /* truncation threshold used                        */
  double times_ms[8];
  int64_t inner_iters; /* total inner iterations (extended Krylov)         */
  int32_t n_inner;     /* number of inner solves                           */
  int32_t n_checks;    /* residual checks whose results were read           */
  double* T_band;      /* host, (ell+1) x (ell*m) lower band of T_m (want_T) */
  double* gamma;       /* host, ell x ell, column-major (want_T)            */
  double* tau;         /* host, ell x ell tau_{m+1,m}, column-major (want_T) */
  int64_t bytes_pass1; /* algorithmic HBM bytes of the first pass          */
  int64_t bytes_spmm;  /* algorithmic HBM bytes of the SpMM calls           */
  double ms_spmm;      /* measured device time of SpMM calls, ms (0 if off) */
  int32_t owns_Z;      /* 1: Z came from hipMalloc and lyap_result_free frees it */
  /* opts->profile: device time and launch count per kernel kind (LYAP_K_*) */
  double kern_ms[LYAP_K_COUNT];
  int32_t kern_n[LYAP_K_COUNT];
  double kern_bytes[LYAP_K_COUNT]; /* algorithmic HBM bytes per launch of each kind */
} lyap_result;


/*
 * lyap_solve — AX + XA + CC^T = 0 by Algorithm 1.
 *
 *  A     operator (device arrays), symmetric negative definite.
 *  C     device, n x s column-major FP64, leading dimension ldc >= n.
 *  s     1 <= s <= 8 (standard, method STD); s = 1, 2 or 4 (extended,
 *        method EXT, ell = 2s; other s give LYAP_E_UNSUPPORTED).
 *        method EXT also needs FP64 storage and solves with A by the inner
 *        CG of lyap_inner_solve (opts->inner_pc, inner_tol, inner_max_iter).
 *  opts  may be NULL (defaults).
 *  out   filled on return (also on error, with status and history so far);
 *        out->s is the block width used (the numerical rank of C, below).
 *
 * A rank-deficient C is deflated (the paper takes a full-rank start block and
 * leaves deflation to the customary practice of block methods): r is the
 * number of eigenvalues of C^T C above 10 n eps lambda_max (eps = 2^-52; the
 * Gram matrix is formed on the device in FP64, its eigenvalues on the host),
 * and for r < s the method runs on C W_r, n x r, with W_r the eigenvectors of
 * the r largest; (C W_r)(C W_r)^T is C C^T without the dropped eigenvalues.
 * C = 0 gives LYAP_E_ARG (the solution is X = 0), NaN/Inf LYAP_E_NUMERIC; with
 * method EXT an r other than 1, 2 or 4 gives LYAP_E_UNSUPPORTED.  The C passed
 * in is only read; the deflated copy is freed on return.
 *
 * The residual is checked after m blocks when the schedule asks for it
 * (every d steps, or adaptively: spaced checks that tighten near the
 * predicted crossing) by Proposition 1 with T_m's eigendecomposition on the
 * GPU in FP64.  At the first passing check, Y~ of eq. (lyap2sol) is truncated
 * (eigenvalues with ||Sigma_2||_F <= eps are dropped; default
 * eps = min(1e-12, 0.05 tol / nu) ||C||_F^2 with nu = max|lambda(T_m)| +
 * ||tau_{m+1,m}||_F, so truncation moves the residual by at most 0.1 tol), and
 * Z = V_m (Q_m Y-check) is formed in a second Lanczos pass (two_pass = 1) or
 * from the stored basis.  Z Z^T approximates X.
 */
lyap_status lyap_solve(const lyap_op* A, const double* C, int32_t s, int64_t ldc,
                       const lyap_opts* opts, lyap_result* out);

typedef struct sylv_result {
  int32_t status;
  int32_t m, t;        /* blocks per space, rank of Z1 Z2^T                */
  int32_t s, ell;
  int32_t owns_Z;      /* 1: Z1/Z2 from hipMalloc, freed by sylv_result_free */
  int64_t n1, n2;
  double* Z1;          /* device, n1 x t column-major */
  double* Z2;          /* device, n2 x t column-major */
  int32_t n_hist;
  int32_t* hist_m;
  double* hist_res;    /* ||R_m||_F / (||C1||_F ||C2||_F) */
  double res;
  double beta1, beta2; /* ||C1||_F, ||C2||_F */
  double trunc_eps;    /* absolute threshold used for ||Y~ - Y1 Y2^T||_F */
  double times_ms[8];
  int32_t n_checks;
  /* opts->want_T: host copies (band layout and column-major as in lyap_result) */
  double* T_band;      /* (ell+1) x k, T_m = V_m^T A V_m */
  double* J_band;      /* (ell+1) x k, J_m = U_m^T B U_m */
  double* gamma1;      /* ell x ell */
  double* gamma2;
  double* tau;         /* tau_{m+1,m} */
  double* iota;        /* iota_{m+1,m} */
  double kern_ms[LYAP_K_COUNT];
  int32_t kern_n[LYAP_K_COUNT];
  double kern_bytes[LYAP_K_COUNT];
} sylv_result;

/*
 * sylv_solve — AX + XB + C1 C2^T = 0 with two standard block Krylov spaces
 * K_m(A, C1), K_m(B, C2) of equal dimension (Section 5.1).  The residual uses
 * eq. (resSylv) evaluated without Y_m (Algorithm 4, with the shifts of the
 * two diagonal matrices D'_i, D''_i taken as lambda_i I + Upsilon and
 * upsilon_j I + Lambda so that it agrees with eq. (resSylv)).  Z1 Z2^T
 * approximates X.  C1 is n1 x s, C2 is n2 x s (device, column-major FP64).
 * opts->method = LYAP_METHOD_EXT builds the two extended spaces EK_m(A, C1),
 * EK_m(B, C2) instead (Section 4's spaces in Section 5.1's method; ell = 2s,
 * Algorithm 4 with the first s rows of tau and iota, factors from the stored
 * bases): s = 1, 2 or 4, FP64 storage, inner CG with inner_pc NONE, JACOBI
 * or IC0 on each operator (E_UNSUPPORTED otherwise).
 */
lyap_status sylv_solve(const lyap_op* A, const lyap_op* B, const double* C1, int64_t ldc1,
                       const double* C2, int64_t ldc2, int32_t s, const lyap_opts* opts,
                       sylv_result* out);

/*
 * lyap_solve_gen — the generalized equation A X E + E X A + C C^T = 0 with E
 * symmetric positive definite, treated as the standard equation of
 * L^{-1} A L^{-T} and L^{-1} C (E = L L^T; Section 6, Example 3) without
 * forming L: block Lanczos for E^{-1} A in the E inner product (basis W with
 * W^T E W = I), one FP64 conjugate-gradient solve with E per step (inner_pc
 * LYAP_PC_JACOBI or LYAP_PC_NONE, others E_UNSUPPORTED; accepted on the true
 * relative residual <= inner_tol), Proposition 1 on T_m, truncation and Z = W_m M as in
 * lyap_solve, so Z Z^T approximates X.
 *  A     operator, symmetric negative definite; E operator (any kind),
 *        symmetric positive definite, same n.
 *  C     device, n x s column-major FP64 (ldc >= n); s = 1, 2 or 4.
 *  opts  method STD, storage F64 only (E_UNSUPPORTED otherwise); two_pass = 1
 *        repeats the steps (inner solves included) to form Z, two_pass = 0
 *        keeps every block.  tol applies to the transformed residual
 *        ||L^{-1} R L^{-T}||_F / ||L^{-1} C||_F^2, R = A X E + E X A + C C^T
 *        (out->beta = ||L^{-1} C||_F, out->hist_res the same ratio).
 *  out   as lyap_solve, with inner_iters / n_inner counting the E solves
 *        of the accepted steps (not those of steps run beside the last check).
 * Errors: E_ARG, E_INNER (an E solve missed inner_tol), E_INDEFINITE (a Ritz
 * value >= 0 or a diagonal entry of E <= 0), E_BREAKDOWN, E_NUMERIC.
 */
lyap_status lyap_solve_gen(const lyap_op* A, const lyap_op* E, const double* C, int32_t s, int64_t ldc,
                           const lyap_opts* opts, lyap_result* out);

/*
 * sylv_solve_small_b — AX + XB + C1 C2^T = 0 with A large and sparse and B
 * small and dense (Section 5.2, "Large A and small B").  Only A is projected:
 * X_m = V_m Y_m with V_m a basis of K_m(A, C1) and the one-sided Galerkin
 * condition V_m^T R_m = 0 (eq. (orthLargeAsmallB)), so Y_m solves the k x n2
 * equation T_m Y + Y B + E_1 gamma_1 C2^T = 0 (eq. (reducedLargeASmallB)).
 * B = P Upsilon P^T is computed once, before the iteration (lyap_sym_eig);
 * the residual at a check is Algorithm 5 (no Y_m formed); at the first
 * passing check Y_m = Q Y~ P^T (eq. (formulaLargeAsmallB)) is truncated to
 * ||Y~ - Y1 Y2^T||_F <= eps (cross approximation with complete pivoting; the
 * error bound of the paper's truncated SVD at a possibly larger rank) and
 * Z1 = V_m Q Y1 (second Lanczos pass when two_pass = 1), Z2 = P Y2.
 *  A      operator, symmetric negative definite, n1 = A->n rows.
 *  B      device, n2 x n2 column-major FP64 (ldb >= n2), symmetric negative
 *         definite, 1 <= n2 <= 2048; only its lower triangle is read.
 *  C1     device, n1 x s column-major FP64 (ldc1 >= n1); C2 device, n2 x s
 *         column-major FP64 (ldc2 >= n2); 1 <= s <= 8.
 *  opts   as for sylv_solve (method STD); tol applies to
 *         ||R_m||_F / (||C1||_F ||C2||_F); trunc_eps < 0 selects
 *         eps = min(1e-12, 0.05 tol / nu) ||C1||_F ||C2||_F with
 *         nu = max|lambda(T_m)| + ||tau_{m+1,m}||_F + max|upsilon|.
 *  out    sylv_result: Z1 (n1 x t), Z2 (n2 x t), history; with want_T the
 *         host T_band, gamma1 and tau (J_band, gamma2, iota stay NULL).
 * Errors: E_ARG (sizes), E_INDEFINITE (B or a Ritz value of A not negative),
 * E_NUMERIC (non-finite B, or Jacobi not converged in 60 sweeps), E_BREAKDOWN.
 */
lyap_status sylv_solve_small_b(const lyap_op* A, const double* B, int64_t n2, int64_t ldb, const double* C1,
                               int64_t ldc1, const double* C2, int64_t ldc2, int32_t s, const lyap_opts* opts,
                               sylv_result* out);

/*
 * lyap_sym_eig — B = P diag(w) P^T for a dense symmetric n x n matrix, the
 * decomposition of the small B that Section 5.2 computes once; parallel
 * cyclic Jacobi in FP64 on the GPU (round-robin pairs, n/2 commuting
 * rotations per launch) until every |b_pq| <= 2^-52 sqrt(|b_pp b_qq|) (or the
 * off-diagonal norm is below 2^-55 ||B||_F).
 *  B      device, column-major (ldb >= n), lower triangle read; 1 <= n <= 2048.
 *  w      device, n eigenvalues ascending.
 *  P      device, n x n column-major (ldp >= n), orthonormal eigenvectors.
 *  stream hipStream_t (NULL = null stream); synchronised before returning.
 *  sweeps optional output: Jacobi sweeps taken.
 */
lyap_status lyap_sym_eig(const double* B, int64_t n, int64_t ldb, double* w, double* P, int64_t ldp, void* stream,
                         int32_t* sweeps);

/* Releases host arrays of a result and, when the library allocated Z with
 * hipMalloc (opts->alloc == NULL), Z itself.  Safe on a zeroed struct. */
void lyap_result_free(lyap_result* r);
void sylv_result_free(sylv_result* r);

/* Thread-local message describing the last error (empty if none). */
const char* lyap_last_error(void);

/* ------------------------------------------------------------------ components
 * Single steps of the path, used by the tests and the benchmark.  Blocks are
 * n x s row-interleaved (row r holds its s entries contiguously) in the
 * storage type (double for LYAP_STORE_F64, float for LYAP_STORE_F32).
 */

/* W = A V for an n x s block (the sparse product of Algorithm 2's input
 * W = A V_{m-1}).  V and W are device pointers, not aliased. */
lyap_status lyap_op_apply(const lyap_op* A, int32_t storage, const void* V, void* W,
                          int32_t s, void* stream);

/* Same as lyap_op_apply repeated `reps` times back to back, returning the
 * average device time per call in *ms (HIP events on `stream`). */
lyap_status lyap_op_apply_timed(const lyap_op* A, int32_t storage, const void* V, void* W,
                                int32_t s, int32_t reps, void* stream, double* ms);

/*
 * Residual of Proposition 1 (Algorithm 3) for a given block tridiagonal T.
 *  T_band  host, (ell+1) x k lower band, column-major: T_band[c*(ell+1)+d] = T(c+d, c).
 *  gamma   host, ell x ell column-major.
 *  tau     host, ell x ell column-major (tau_{m+1,m}).
 *  res     output ||R||_F.
 *  lam     optional host output, k eigenvalues of T ascending (may be NULL).
 * Everything runs on the GPU in FP64.
 */
lyap_status lyap_ctri(const double* T_band, int32_t ell, int32_t k, const double* gamma,
                      const double* tau, double* res, double* lam, void* stream);

/*
 * Inner solve of the extended Krylov method (Section 4 applies A^{-1} to a
 * block at every step): X = A^{-1} B by preconditioned conjugate gradients on
 * -A (symmetric positive definite), FP64, the s columns advanced together
 * with their own scalars.
 *  A        operator (device arrays), symmetric negative definite.
 *  B, X     device, n x s column-major FP64, leading dimensions ldb, ldx >= n;
 *           X is overwritten (B is not modified).
 *  s        1, 2 or 4.
 *  opts     inner_pc, inner_tol (bound on the true ||b - A x|| / ||b|| of
 *           every column), inner_max_iter and stream are used; NULL means
 *           defaults.  inner_pc: LYAP_PC_NONE; LYAP_PC_JACOBI; LYAP_PC_IC0,
 *           zero fill-in incomplete Cholesky of -A with the grid cells in
 *           red-black order (i + j + l even first), for 5- and 7-point
 *           stencil operators (E_UNSUPPORTED for CSR): since a stencil couples
 *           only cells of different colours, the factor is explicit and PCG
 *           with it is run as CG on the black Schur complement
 *           D_b - E D_r^{-1} E^T preconditioned by its diagonal (the same
 *           iterates up to one iteration), then the red cells are solved for;
 *           the true residual still certifies the whole solution.
 *           LYAP_PC_LEARNED: E_UNSUPPORTED (trained inside lyap_solve).
 *  iters    optional output: CG iterations, restarts included.
 *  relres   optional output: largest true relative residual over the columns.
 * Returns LYAP_E_INNER when a column does not reach inner_tol (X then holds
 * the last iterate), LYAP_E_INDEFINITE when a diagonal entry of A is >= 0.
 */
lyap_status lyap_inner_solve(const lyap_op* A, const double* B, int64_t ldb, double* X, int64_t ldx, int32_t s,
                             const lyap_opts* opts, int64_t* iters, double* relres);

/* flag of lyap_solve_batched's tune argument */
#define LYAP_BATCH_GRAPHS 4

/*
 * lyap_solve_batched -- `count` independent equations A_i X + X A_i + C_i C_i^T = 0
 * advanced together: the block Lanczos steps of all unconverged problems of
 * one block width run in the same grouped launches (a work map assigns each
 * workgroup to a problem and a row range), each problem keeps its own check
 * schedule (Algorithm 1 step 6) and leaves the group when it converges, and
 * the second pass (Section 3.3) is grouped the same way.
 *  A      host array of `count` operators (device arrays inside).
 *  C      host array of `count` device pointers, n_i x s_i column-major FP64.
 *  s      host array, 1 <= s_i <= 8;  ldc: host array, ldc_i >= n_i.
 *  opts   shared by all problems (tol, max_iter, check_every, storage,
 *         allocator, stream, profile); method must be STD and two_pass 1.
 *  tune   0: the fixed tile shape (the single-problem kernels' workgroup
 *         size, 2048 rows per workgroup; reproducible bits); 1: tile shapes
 *         from the autotuner -- per (device, storage, block width, size
 *         bucket) and workgroup size (256 or 1024 threads, 256 only above 4
 *         columns) the fastest of 2048..16384 rows per workgroup, found by
 *         timing grouped steps on scratch data; each block width's launches
 *         take the workgroup size whose tuned step times sum lowest over its
 *         problems.  Results are kept in the process and in a text file that
 *         persists across processes ($LYAP_TUNE_CACHE, else
 *         $XDG_CACHE_HOME/lyap_tune.txt, else $HOME/.cache/lyap_tune.txt;
 *         a file that cannot be read or written is ignored); 2: as 1 but
 *         timing again and replacing what the caches hold.  Autotuned runs
 *         are reproducible when the same shapes are chosen.
 *         Or-ed with LYAP_BATCH_GRAPHS: the first pass issues every step of
 *         all problems as one replay of a captured HIP graph (the grouped
 *         step kernels of every block width, the step index read from device
 *         memory), captured again whenever a work map changes; the work runs
 *         on a stream of the solver's own, ordered after opts->stream, and
 *         the results are bit-identical to direct launches.  Not combined
 *         with opts->profile (LYAP_E_ARG).
 *  out    array of `count` results, filled like lyap_solve's; phase times are
 *         those of the whole batch (times_ms[LYAP_T_TO_TOL] is per problem);
 *         kern_ms / kern_n of out[0] cover the whole batch.
 * Returns LYAP_OK when every problem converged, else the first error status
 * (or LYAP_NOT_CONVERGED); each out[i].status has the problem's own status.
 */
lyap_status lyap_solve_batched(int32_t count, const lyap_op* A, const double* const* C, const int32_t* s,
                               const int64_t* ldc, const lyap_opts* opts, int32_t tune, lyap_result* out);

/* ------------------------------------------------------------------ learned preconditioner
 * The network, on an operator's whole grid (the entry points below; the
 * solver's inner solves use it on IC(0)'s Schur complement, see the next
 * block): trained for 200 Adam steps (learning rate 2e-3) on pairs harvested
 * from a CG solve, then applied in flexible CG with z = M(r):
 *   M r = D^{-1} r + s (K^T K)(s r),  s = sqrt(D^{-1}),  D = diag(-A),
 *   K(u) = conv2(conv1([u, f u])),  f = log(-diag A) - mean,
 * two 3x3x3 convolutions (2 -> C -> C channels, C = 2, 4 or 8, zero padding,
 * no bias) on the operator's grid, FP32 weights (SplitMix64 seed 0x5eed, uniform in
 * [-0.05, 0.05)).  M is symmetric positive definite for any weights.  The loss
 * of a pair (r, e), (-A) e = r, is (M r - e)^T (-A) (M r - e) / e^T (-A) e.
 * The entry points below expose the pieces for testing; W holds C*2*27 + C*C*27
 * floats, W1[o][i][t] then W2[o][i][t], t = 9 (dz+1) + 3 (dy+1) + (dx+1).
 * Vectors are device FP64, length n.
 */
void lyap_pcnet_init(int32_t C, uint64_t seed, double scale, float* W);
lyap_status lyap_pcnet_apply(const lyap_op* A, int32_t C, const float* W, const double* r, double* z, void* stream);
/*
 * lyap_pcnet_apply_noalloc -- lyap_pcnet_apply for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same result, with
 * every intermediate buffer (the operator's FP64 coefficient copies, D^{-1},
 * the network's activations, weights and partial sums) carved from one static
 * 32 MiB device array per GPU instead of hipMalloc.  No device or pinned host
 * memory is allocated; the array's address is looked up once per device, on
 * the first call made with that device current.
 *  Limit: n (64 + 12 C) bytes plus about 1 MiB must fit in 32 MiB for a
 *  7-point operator (n (32 + 12 C) for a 5-point one): n <= 262144 at C = 4.
 *  Larger inputs return LYAP_E_ARG with the bytes needed in the message.
 *  A, C, W, r, z, stream as for lyap_pcnet_apply (stencil operators only).
 *  Every call on one GPU uses that GPU's single array and returns only after
 *  its work on `stream` has finished; calls that overlap on one GPU (from
 *  several host threads, or on several streams at once) race on the array.
 */
lyap_status lyap_pcnet_apply_noalloc(const lyap_op* A, int32_t C, const float* W, const double* r, double* z,
                                     void* stream);
/* loss of (r, e) and its gradient (host, FP64, same layout as W) */
lyap_status lyap_pcnet_grad(const lyap_op* A, int32_t C, const float* W, const double* r, const double* e,
                            double* loss, double* grad, void* stream);
/* `steps` Adam steps over the pairs in order (pair t mod npairs at step t);
 * W (host) in/out; losses (host, optional) gets the loss before each step. */
lyap_status lyap_pcnet_train(const lyap_op* A, int32_t C, float* W, int32_t npairs, const double* const* r,
                             const double* const* e, int32_t steps, double lr, double* losses, void* stream);
/* X = A^{-1} B (one column) by flexible CG with M; certified like lyap_inner_solve. */
lyap_status lyap_pcnet_fcg(const lyap_op* A, int32_t C, const float* W, const double* B, double* X, double eta,
                           int32_t max_iter, int64_t* iters, double* relres, void* stream);

/* ------------------------------------------------------------------ learned correction of IC(0)
 * The inner solves of lyap_solve / sylv_solve with inner_pc = LYAP_PC_LEARNED
 * use the same network as a correction of red-black IC(0) (stencil operators,
 * one column): the solve runs on the black Schur complement
 * Sigma = D_b - E D_r^{-1} E^T of the red-black split (see lyap_inner_solve)
 * with
 *   M r = D_S^{-1} r + s K^T K (s r),  D_S = diag(Sigma),  s = sqrt(D_S^{-1}),
 *   f = log D_S - mean,
 * the network acting on the compact grid of the black cells: an array of
 * hx x ny x nz points, hx = ceil(nx / 2) rounded up to a multiple of 4, the
 * black cell (i, j, l) at point (i / 2, j, l), the remaining points held at
 * zero (D_S^{-1} = s = 0 there).  Zero weights give IC(0) itself.  Training
 * pairs (r_i, e_i), Sigma e_i = r_i, come from the first inner solve (the
 * condensed IC(0) CG, every 16 iterations, at most 16); the loss is
 * (M r - e)^T Sigma (M r - e) / e^T Sigma e; 50 Adam steps at learning rate
 * 1e-2 inside lyap_solve (the entry points below take steps and rate); later
 * solves run flexible CG on Sigma with M, then the red cells are solved for,
 * and the whole-grid true residual certifies each solve.  C = 2 in the solver.
 * The two entry points below expose this for testing (W as above, b, B, X
 * device FP64 of length n):
 *  lyap_pcnet_schur_train  solves A x = b by the condensed IC(0) CG to a true
 *      relative residual 1e-12, keeping (r_i, e_i) every `every` iterations
 *      (at most `keep`), then takes `steps` Adam steps over the pairs with
 *      e^T Sigma e > 0, in order; W in/out (host), losses (host, optional) the
 *      loss before each step, *npairs the pairs used.
 *  lyap_pcnet_schur_fcg    X = A^{-1} B by flexible CG on Sigma with M and W,
 *      certified like lyap_inner_solve.
 * E_UNSUPPORTED for a CSR operator. */
lyap_status lyap_pcnet_schur_train(const lyap_op* A, int32_t C, float* W, const double* b, int32_t every,
                                   int32_t keep, int32_t steps, double lr, double* losses, int32_t* npairs,
                                   void* stream);
lyap_status lyap_pcnet_schur_fcg(const lyap_op* A, int32_t C, const float* W, const double* B, double* X,
                                 double eta, int32_t max_iter, int64_t* iters, double* relres, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LYAP_H */
