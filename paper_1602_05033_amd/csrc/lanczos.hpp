// Launch interface of the block Lanczos kernels (see lanczos.hip).
#pragma once

#include <algorithm>

#include "op.hpp"

namespace lyap {

// Per-step coefficient log: 11 slots of S x S FP64 (row-major [a][b]) followed
// by 4 scalars (log_stride(S) doubles per step).
enum LogSlot {
  L_A1 = 0,  // alpha applied against V_{j-1}, first sweep
  L_A2 = 1,  // alpha against V_j, first sweep
  L_A3 = 2,  // alpha against V_{j-1}, second sweep
  L_A4 = 3,  // alpha against V_j, second sweep
  L_G1 = 4,  // W^T W before the QR
  L_R1 = 5,  // chol(G1)
  L_R1I = 6, // R1^{-1}
  L_G2 = 7,  // (W R1^{-1})^T (W R1^{-1})
  L_R2 = 8,  // chol(G2)
  L_R = 9,   // tau_{j+1,j} = R2 R1
  L_RI = 10, // R1^{-1} R2^{-1}
  L_FLAG = 11,  // scalars at 11*S*S: [0] smallest pivot ratio of chol(G1), [1] trace(G1)
  L_NSLOT = 12
};
constexpr size_t log_stride(int S) { return (size_t)11 * S * S + 4; }

template <typename T>
struct StepArgs {
  OpDev<T> op;
  int n;
  const T* Vprev;
  const T* Vcur;
  T* W;
  T* Vnext;
  double* log;       // this step's log
  double* band;      // T_m lower band, ld = S+1
  int j;             // step index (0-based)
  const double* pin; // partial Gram matrices of the previous kernel
  double* pout;      // partial Gram matrices of this kernel (one per workgroup)
  int nparts;        // number of workgroups (= partials)
  int* flags;        // [0] first breakdown step+1, [1] first non-finite step+1
};

// Workgroups of the streaming kernels for an n-row block: one per CU (256)
// from n = 65536 up; below that one per 256 rows, so that a small block still
// spreads over many CUs (these kernels wait on memory latency, not bandwidth,
// at such sizes) instead of filling a few workgroups of 1024 threads.
inline int stream_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kSGrid));
}

// Optional per-kernel timing with HIP events on the solver's stream: the time
// between one mark and the next is attributed to the kind given at the first.
struct KernelTimer {
  hipStream_t st = nullptr;
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;
  size_t used = 0;
  double ms[LYAP_K_COUNT] = {0};
  int n[LYAP_K_COUNT] = {0};
  void mark(int k) {
    if (!on) return;
    if (used == ev.size()) {
      hipEvent_t e;
      LYAP_HIP(hipEventCreate(&e));
      ev.push_back(e);
      kind.push_back(-1);
    }
    LYAP_HIP(hipEventRecord(ev[used], st));
    kind[used] = k;
    ++used;
  }
  // Closes the open interval and accumulates everything recorded so far.
  void collect() {
    if (!on || used == 0) return;
    mark(-1);
    LYAP_HIP(hipEventSynchronize(ev[used - 1]));
    for (size_t i = 0; i + 1 < used; ++i) {
      if (kind[i] < 0) continue;
      float t = 0.f;
      LYAP_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
      ms[kind[i]] += t;
      n[kind[i]] += 1;
    }
    used = 0;
  }
  ~KernelTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

template <typename T>
void launch_step(const StepArgs<T>& a, int S, int grid, double* partA, double* partB, hipStream_t st,
                 KernelTimer* kt = nullptr);
template <typename T>
void launch_replay(const OpDev<T>& op, int S, const T* Vprev, const T* Vcur, T* Vnext, const double* log, int grid,
                   hipStream_t st);
template <typename T>
void launch_init(const double* C, int64_t ldc, int n, int S, double* glog, double* partA, double* partB, int* flags,
                 T* V1, int grid, hipStream_t st);
template <typename T>
void launch_init_store(const double* C, int64_t ldc, int n, int S, const double* glog, T* V1, int grid, hipStream_t st);
// Up to 64 block pointers per flush launch (64/S blocks are used at a time).
struct BlockList {
  const void* p[64];
};
template <typename T>
void launch_zflush(const void* const* blocks, int nb, int n, int S, const double* Mrows, int t, double* Z,
                   int64_t ldz, int grid, hipStream_t st);
template <typename T> void launch_apply(const OpDev<T>& op, int S, const T* V, T* W, int grid, hipStream_t st);
int zflush_max_blocks(int S);

// ------------------------------------------------------------------ grouped launches
// Per-problem state of a grouped (batched) launch: every problem advances by
// the same step j, so the step's blocks and log entry follow from j (V_{j+1}
// overwrites V_{j-1}; V_j is Vb1 for even j, Vb0 for odd j).
template <typename T>
struct BatchDesc {
  OpDev<T> op;
  int n;
  int nparts;        // workgroups of this problem in every grouped launch
  T* Vb0;
  T* Vb1;
  T* W;
  double* log;       // step 0 of the coefficient log
  double* band;
  double* partA;
  double* partB;
  int* flags;
  T* ring;           // second pass: R blocks of n x S
  int R;
  const T* zero;     // an n x S block of zeros
};

// map[w] = (problem, workgroup index within the problem) for every workgroup
// of a grouped launch over the problems of one block width S; nt threads per
// workgroup (256, or 1024 for S <= 4; batch_default_threads(S) is the size
// the single-problem kernels use).  With jp set the kernels read the step
// index from *jp (device memory) instead of j, so that one captured graph of a
// step can be replayed for successive steps.
int batch_default_threads(int S);
template <typename T>
void launch_batch_step(const BatchDesc<T>* d, const int2* map, int nwg, int S, int nt, int j, hipStream_t st,
                       KernelTimer* kt = nullptr, const int* jp = nullptr);
template <typename T>
void launch_batch_replay(const BatchDesc<T>* d, const int2* map, int nwg, int S, int nt, int i, hipStream_t st);

}  // namespace lyap
