// Operator validation, conversion to the storage type, and the SpMM component
// entry points (lyap_op_apply, lyap_op_apply_timed).
#include <cstdarg>

#include "lanczos.hpp"

namespace lyap {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

void validate_op(const lyap_op* A) {
  LYAP_REQUIRE(A != nullptr, LYAP_E_ARG, "operator is NULL");
  LYAP_REQUIRE(A->n > 0 && A->n < (int64_t)1 << 31, LYAP_E_ARG, "operator size n=%lld out of range",
               (long long)A->n);
  if (A->kind == LYAP_OP_STENCIL5) {
    LYAP_REQUIRE(A->nx > 0 && A->ny > 0 && (int64_t)A->nx * A->ny == A->n, LYAP_E_ARG,
                 "stencil5: nx*ny (%d*%d) != n (%lld)", A->nx, A->ny, (long long)A->n);
  } else if (A->kind == LYAP_OP_STENCIL7) {
    const int nz = A->nz > 0 ? A->nz : 1;
    LYAP_REQUIRE(A->nx > 0 && A->ny > 0 && (int64_t)A->nx * A->ny * nz == A->n, LYAP_E_ARG,
                 "stencil7: nx*ny*nz != n");
    LYAP_REQUIRE(A->diag && A->tx && A->ty && (nz == 1 || A->tz), LYAP_E_ARG,
                 "stencil7: coefficient arrays missing");
  } else if (A->kind == LYAP_OP_CSR) {
    LYAP_REQUIRE(A->rowptr && A->colind && A->val && A->nnz >= 0, LYAP_E_ARG, "csr: arrays missing");
  } else {
    LYAP_REQUIRE(false, LYAP_E_ARG, "unknown operator kind %d", A->kind);
  }
}

template <typename T>
__global__ void k_convert(const double* src, T* dst, int64_t n, double add) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (T)(src[i] + add);
}

template <typename T>
static void convert(const double* src, DevBuf& dst, int64_t n, double add, hipStream_t st) {
  dst.alloc((size_t)n * sizeof(T));
  if (n == 0) return;
  int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL((k_convert<T>), dim3(grid), dim3(256), 0, st, src, dst.as<T>(), n, add);
  LYAP_LAUNCHED("convert");
}

template <typename T>
static void make_op(const lyap_op* A, OpHolder<T>& h, hipStream_t st) {
  validate_op(A);
  OpDev<T>& d = h.dev;
  d = OpDev<T>{};
  d.kind = A->kind;
  d.nx = A->nx;
  d.ny = A->ny;
  d.nz = A->nz > 0 ? A->nz : 1;
  d.n = (int)A->n;
  if (A->kind == LYAP_OP_STENCIL5) {
    d.cc = (T)(A->cc + A->shift);
    d.co = (T)A->co;
  } else if (A->kind == LYAP_OP_STENCIL7) {
    convert<T>(A->diag, h.diag, A->n, A->shift, st);
    convert<T>(A->tx, h.tx, A->n, 0.0, st);
    convert<T>(A->ty, h.ty, A->n, 0.0, st);
    if (d.nz > 1) convert<T>(A->tz, h.tz, A->n, 0.0, st);
    else {
      h.tz.alloc(sizeof(T));
    }
    d.diag = static_cast<T*>(h.diag.p);
    d.tx = static_cast<T*>(h.tx.p);
    d.ty = static_cast<T*>(h.ty.p);
    d.tz = static_cast<T*>(h.tz.p);
  } else {
    convert<T>(A->val, h.val, A->nnz, 0.0, st);
    d.rowptr = A->rowptr;
    d.col = A->colind;
    d.val = static_cast<T*>(h.val.p);
    d.shift = (T)A->shift;
    h.nnz = A->nnz;
  }
}

void make_op_f64(const lyap_op* A, OpHolder<double>& h, hipStream_t st) { make_op<double>(A, h, st); }
void make_op_f32(const lyap_op* A, OpHolder<float>& h, hipStream_t st) { make_op<float>(A, h, st); }

template <typename T>
static double apply_impl(const lyap_op* A, const void* V, void* W, int s, int reps, hipStream_t st) {
  OpHolder<T> h;
  make_op<T>(A, h, st);
  const int grid = xcd_grid(grid_for(A->n, 2, 4096));  // two rows per thread
  if (reps <= 0) {
    launch_apply<T>(h.dev, s, (const T*)V, (T*)W, grid, st);
    LYAP_HIP(hipStreamSynchronize(st));
    return 0.0;
  }
  launch_apply<T>(h.dev, s, (const T*)V, (T*)W, grid, st);  // warm-up
  hipEvent_t e0, e1;
  LYAP_HIP(hipEventCreate(&e0));
  LYAP_HIP(hipEventCreate(&e1));
  LYAP_HIP(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) launch_apply<T>(h.dev, s, (const T*)V, (T*)W, grid, st);
  LYAP_HIP(hipEventRecord(e1, st));
  LYAP_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  LYAP_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)ms / reps;
}

}  // namespace lyap

using namespace lyap;

extern "C" const char* lyap_last_error(void) { return last_error(); }

extern "C" lyap_status lyap_op_apply(const lyap_op* A, int32_t storage, const void* V, void* W, int32_t s,
                                     void* stream) {
  clear_error();
  try {
    LYAP_REQUIRE(V && W, LYAP_E_ARG, "V or W is NULL");
    LYAP_REQUIRE(s >= 1 && s <= 8, LYAP_E_ARG, "s=%d out of range 1..8", s);
    hipStream_t st = (hipStream_t)stream;
    if (storage == LYAP_STORE_F64) apply_impl<double>(A, V, W, s, 0, st);
    else if (storage == LYAP_STORE_F32) apply_impl<float>(A, V, W, s, 0, st);
    else LYAP_REQUIRE(false, LYAP_E_ARG, "unknown storage %d", storage);
    return LYAP_OK;
  } catch (const Error& e) {
    return e.st;
  }
}

extern "C" lyap_status lyap_op_apply_timed(const lyap_op* A, int32_t storage, const void* V, void* W, int32_t s,
                                           int32_t reps, void* stream, double* ms) {
  clear_error();
  try {
    LYAP_REQUIRE(V && W && ms, LYAP_E_ARG, "NULL argument");
    LYAP_REQUIRE(s >= 1 && s <= 8, LYAP_E_ARG, "s=%d out of range 1..8", s);
    LYAP_REQUIRE(reps >= 1, LYAP_E_ARG, "reps must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    if (storage == LYAP_STORE_F64) *ms = apply_impl<double>(A, V, W, s, reps, st);
    else if (storage == LYAP_STORE_F32) *ms = apply_impl<float>(A, V, W, s, reps, st);
    else LYAP_REQUIRE(false, LYAP_E_ARG, "unknown storage %d", storage);
    return LYAP_OK;
  } catch (const Error& e) {
    return e.st;
  }
}
