// lyap_solve_batched: many independent Lyapunov equations (different n, s and
// iteration counts) advanced together by grouped launches.  Every active
// problem of one block width takes its next block Lanczos step in the same
// seven kernels -- each workgroup looks up its (problem, workgroup-in-problem)
// pair in a work map -- so a batch of small problems fills the GPU and costs
// seven launches per step instead of seven per problem.  Residual checks run
// on each problem's own schedule; converged problems leave the work map.  The
// second pass is grouped the same way (one replay launch per step for all
// problems still replaying), with per-problem Z accumulation.
//
// Workgroups per problem ("nparts") are chosen per (block width, size
// bucket): a fixed rule, or an autotuner that times one grouped step on
// scratch problems for each candidate and keeps the fastest for the process.
// The choice sets the order of the partial sums, so autotuned runs are
// reproducible within a process (and across processes when the timings pick
// the same candidates); the fixed rule is reproducible always.
#include <sys/stat.h>

#include <algorithm>
#include <deque>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "check.hpp"
#include "lanczos.hpp"
#include "solver.hpp"

namespace lyap {

namespace {

constexpr int kChunkCandidates[] = {2048, 4096, 8192, 16384};

int nparts_for(int64_t n, int chunk) {
  const int64_t p = (n + chunk - 1) / chunk;
  return (int)std::max<int64_t>(1, std::min<int64_t>(p, kSGrid));
}

int size_bucket(int64_t n) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= n) ++b;
  return b;
}

// ------------------------------------------------------------------ tile autotuner
// A tile shape of the grouped step is (threads per workgroup, rows per
// workgroup).  For each (device, storage, block width, size bucket) and each
// workgroup size the autotuner times a grouped step on a scratch problem of
// the bucket's size for every row count and keeps the fastest with its time.
// Results live in the process and in a text file that persists across
// processes: $LYAP_TUNE_CACHE, else $XDG_CACHE_HOME/lyap_tune.txt, else
// $HOME/.cache/lyap_tune.txt (one line per entry: "lyap-tune-1 arch cus
// storage S bucket threads rows ms"; unreadable or unwritable files are
// ignored).
struct TuneEntry {
  int chunk;
  float ms;
};
using TuneKey = std::tuple<std::string, int, int, int, int>;  // (device, storage, S, bucket, threads)

std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string device_tag() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  static std::mutex mu;
  static std::map<int, std::string> tags;
  std::lock_guard<std::mutex> g(mu);
  auto it = tags.find(dev);
  if (it != tags.end()) return it->second;
  hipDeviceProp_t prop;
  std::string tag = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    std::string arch = prop.gcnArchName;
    for (char& c : arch)
      if (c == ' ' || c == '\t') c = '_';
    tag = arch + ":" + std::to_string(prop.multiProcessorCount);
  }
  tags[dev] = tag;
  return tag;
}

std::string tune_cache_path() {
  if (const char* p = std::getenv("LYAP_TUNE_CACHE")) return p;
  if (const char* x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/lyap_tune.txt";
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/lyap_tune.txt";
  return "";
}

// caller holds g_tune_mu
void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char tag[16], dev[128];
  int storage, S, bucket, nt, chunk;
  float ms;
  while (std::fscanf(f, "%15s %127s %d %d %d %d %d %f", tag, dev, &storage, &S, &bucket, &nt, &chunk, &ms) == 8) {
    if (std::string(tag) != "lyap-tune-1" || chunk <= 0 || !(ms > 0.f)) continue;
    g_tune[TuneKey(dev, storage, S, bucket, nt)] = TuneEntry{chunk, ms};
  }
  std::fclose(f);
}

void tune_store_locked(const TuneKey& k, const TuneEntry& e) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) {  // a missing ~/.cache: create that one directory
    const size_t sl = path.rfind('/');
    if (sl != std::string::npos && mkdir(path.substr(0, sl).c_str(), 0755) == 0) f = std::fopen(path.c_str(), "a");
  }
  if (!f) return;
  std::fprintf(f, "lyap-tune-1 %s %d %d %d %d %d %.6g\n", std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k),
               std::get<3>(k), std::get<4>(k), e.chunk, e.ms);
  std::fclose(f);
}

std::vector<int> thread_candidates(int S) {
  return S <= 4 ? std::vector<int>{256, 1024} : std::vector<int>{256};
}

template <typename T>
struct Problem {
  int id;
  int n, S;
  const double* C;
  int64_t ldc;
  OpHolder<T> op;
  DevBuf Vb0, Vb1, W, zero, log, glog, band, partA, partB, ring;
  std::vector<double> hglog;
  double beta = 0.0;
  int m = 0;           // steps taken
  int m_final = 0;     // blocks of the accepted basis
  bool active = true;
  lyap_status status = LYAP_NOT_CONVERGED;
  std::unique_ptr<Checker> ck;
  CheckSchedule sched{0, 0};
  int next_check = 0;
  int checked_m = 0;
  double lam_absmax = 0.0;
  double last_res = INFINITY;
  double t_to_tol = 0.0;
  std::vector<int> hm;
  std::vector<double> hr;
  int nparts = 1;
  std::vector<std::pair<int, TuneEntry>> shapes;  // per workgroup size: best rows per workgroup, step time
  DevBuf M;
  int t = 0;
};

// Times one grouped step on a scratch problem (a fixed pseudo-random block,
// the 5-point operator of the bucket's size) with nt threads per workgroup for
// every row count; returns the fastest (from the caches when known, unless
// refresh is set).
template <typename T>
TuneEntry autotune_shape(int S, int64_t n, int nt, bool refresh, hipStream_t st) {
  const int storage = std::is_same_v<T, double> ? LYAP_STORE_F64 : LYAP_STORE_F32;
  const TuneKey key(device_tag(), storage, S, size_bucket(n), nt);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end() && !refresh) return it->second;
  }
  const int N = (int)std::max<int64_t>(8, (int64_t)std::sqrt((double)n));
  const int nn = N * N;
  const size_t blk = (size_t)nn * S * sizeof(T);
  DevBuf Vb0(blk), Vb1(blk), W(blk), zero(blk), log(4 * log_stride(S) * sizeof(double)),
      band((size_t)(S + 1) * S * 8 * sizeof(double)), pA((size_t)kSGrid * 2 * S * S * sizeof(double)),
      pB((size_t)kSGrid * 2 * S * S * sizeof(double)), flags(64), dd(sizeof(BatchDesc<T>));
  LYAP_HIP(hipMemsetAsync(Vb0.p, 0, blk, st));
  LYAP_HIP(hipMemsetAsync(W.p, 0, blk, st));
  LYAP_HIP(hipMemsetAsync(flags.p, 0, 64, st));
  {
    std::vector<T> h((size_t)nn * S);
    for (size_t i = 0; i < h.size(); ++i) h[i] = (T)(((i * 2654435761u) % 1000) * 1e-3 - 0.5);
    LYAP_HIP(hipMemcpyAsync(Vb1.p, h.data(), blk, hipMemcpyHostToDevice, st));
    LYAP_HIP(hipStreamSynchronize(st));
  }
  BatchDesc<T> d{};
  d.op.kind = LYAP_OP_STENCIL5;
  d.op.nx = N;
  d.op.ny = N;
  d.op.nz = 1;
  d.op.n = nn;
  d.op.cc = (T)-4;
  d.op.co = (T)1;
  d.n = nn;
  d.Vb0 = Vb0.template as<T>();
  d.Vb1 = Vb1.template as<T>();
  d.W = W.template as<T>();
  d.log = log.template as<double>();
  d.band = band.template as<double>();
  d.partA = pA.template as<double>();
  d.partB = pB.template as<double>();
  d.flags = flags.template as<int>();
  hipEvent_t e0, e1;
  LYAP_HIP(hipEventCreate(&e0));
  LYAP_HIP(hipEventCreate(&e1));
  TuneEntry best{kChunkCandidates[0], 1e30f};
  DevBuf dm((size_t)kSGrid * sizeof(int2));
  for (int chunk : kChunkCandidates) {
    d.nparts = nparts_for(nn, chunk);
    std::vector<int2> map(d.nparts);
    for (int w = 0; w < d.nparts; ++w) map[w] = make_int2(0, w);
    LYAP_HIP(hipMemcpyAsync(dd.p, &d, sizeof(d), hipMemcpyHostToDevice, st));
    LYAP_HIP(hipMemcpyAsync(dm.p, map.data(), map.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    // step 0 twice (the same inputs every time), then timed
    for (int r = 0; r < 2; ++r)
      launch_batch_step<T>(dd.template as<BatchDesc<T>>(), dm.template as<int2>(), d.nparts, S, nt, 0, st);
    LYAP_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 5; ++r)
      launch_batch_step<T>(dd.template as<BatchDesc<T>>(), dm.template as<int2>(), d.nparts, S, nt, 0, st);
    LYAP_HIP(hipEventRecord(e1, st));
    LYAP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    LYAP_HIP(hipEventElapsedTime(&ms, e0, e1));
    const float per_step = ms / 5.0f;
    if (per_step < best.ms) best = TuneEntry{chunk, per_step};
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = best;
  tune_store_locked(key, best);
  return best;
}

// The step index of replayed step graphs, on the device: set when a graph is
// captured, advanced by the last node of every replay.
__global__ void k_step_set(int* jp, int j) {
  if (threadIdx.x == 0) *jp = j;
}
__global__ void k_step_next(int* jp) {
  if (threadIdx.x == 0) *jp += 1;
}

template <typename T>
lyap_status batched_impl(int count, const lyap_op* A, const double* const* C, const int32_t* s, const int64_t* ldc,
                         const lyap_opts& o, int tune, lyap_result* out) {
  const auto t_entry = Clock::now();
  // LYAP_BATCH_GRAPHS: pass 1 replays one captured graph per step (all
  // groups' step kernels) instead of launching them one by one; capture needs
  // a stream of its own, ordered after the caller's
  const bool graphs = (tune & LYAP_BATCH_GRAPHS) != 0;
  tune &= 3;
  struct OwnStream {
    hipStream_t s = nullptr;
    ~OwnStream() { if (s) (void)hipStreamDestroy(s); }
  } own;
  hipStream_t st = (hipStream_t)o.stream;
  if (graphs) {
    LYAP_HIP(hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking));
    hipEvent_t e;
    LYAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    LYAP_HIP(hipEventRecord(e, st));
    LYAP_HIP(hipStreamWaitEvent(own.s, e, 0));
    LYAP_HIP(hipEventDestroy(e));
    st = own.s;
  }
  const int maxit = o.max_iter;
  KernelTimer kt;
  kt.st = st;
  kt.on = o.profile != 0;

  // residual checks run on kCS extra streams (problem i on stream i mod kCS)
  // while the grouped steps continue; with opts->profile on the solver's
  // stream.  Three check streams and the solver's stream fill the four
  // hardware queues a process gets by default.
  constexpr int kCS = 3;
  const bool overlap = o.profile == 0;
  struct Streams {
    hipStream_t s[kCS] = {nullptr, nullptr, nullptr};
    ~Streams() { for (auto x : s) if (x) (void)hipStreamDestroy(x); }
  } cs;
  for (int i = 0; i < kCS; ++i) {
    if (overlap) LYAP_HIP(hipStreamCreateWithFlags(&cs.s[i], hipStreamNonBlocking));
  }
  auto cstream = [&](int id) { return overlap ? cs.s[id % kCS] : st; };
  // second-pass ring of V blocks per problem: with the checks overlapping,
  // the Z accumulation runs on the problem's check stream and its blocks stay
  // in the ring for kFlushSlack more replay steps while the replays go on
  constexpr int kFlushSlack = 16;
  auto ring_blocks = [&](int S) { return zflush_max_blocks(S) + 2 + (overlap ? kFlushSlack : 0); };

  std::vector<std::unique_ptr<Problem<T>>> P;
  DevBuf flags_all((size_t)count * 16 * sizeof(int));
  LYAP_HIP(hipMemsetAsync(flags_all.p, 0, flags_all.bytes, st));
  HostBuf hflags((size_t)count * 16 * sizeof(int));
  for (int i = 0; i < count; ++i) {
    auto p = std::make_unique<Problem<T>>();
    p->id = i;
    p->n = (int)A[i].n;
    p->S = s[i];
    p->C = C[i];
    p->ldc = ldc[i];
    if constexpr (std::is_same_v<T, double>) make_op_f64(&A[i], p->op, st);
    else make_op_f32(&A[i], p->op, st);
    const size_t blk = (size_t)p->n * p->S * sizeof(T);
    const size_t LS = log_stride(p->S);
    p->Vb0.alloc(blk);
    p->Vb1.alloc(blk);
    p->W.alloc(blk);
    p->zero.alloc(blk);
    p->log.alloc(((size_t)maxit + 1) * LS * sizeof(double));
    p->glog.alloc(LS * sizeof(double));
    p->band.alloc((size_t)(p->S + 1) * p->S * (maxit + 2) * sizeof(double));
    p->partA.alloc((size_t)kSGrid * 2 * p->S * p->S * sizeof(double));
    p->partB.alloc((size_t)kSGrid * 2 * p->S * p->S * sizeof(double));
    LYAP_HIP(hipMemsetAsync(p->zero.p, 0, blk, st));
    LYAP_HIP(hipMemsetAsync(p->Vb0.p, 0, blk, st));
    LYAP_HIP(hipMemsetAsync(p->band.p, 0, p->band.bytes, st));
    // tile shapes: the fixed rule (the single-problem kernels' workgroup size,
    // 2048 rows per workgroup) or the autotuner's table for this size
    if (tune)
      for (int nt : thread_candidates(p->S)) p->shapes.emplace_back(nt, autotune_shape<T>(p->S, p->n, nt, tune == 2, st));
    p->nparts = nparts_for(p->n, 2048);
    p->ck = std::make_unique<Checker>(p->S, p->S, cstream(i));
    p->sched = CheckSchedule{o.check_every, maxit};
    // a check costs the host about 170 launches (the first pass is bound by
    // the host's launch rate), a grouped step a handful for all problems
    // together: the batch checks less often (the next check at most 3 m steps
    // ahead, aimed at 0.9 of the predicted crossing; measured on the 64-problem
    // batch against at most m ahead: 1.7% more steps, pass 1 518 -> 391 ms)
    p->sched.grow = 3.0;
    p->sched.aim = 0.9;
    p->next_check = p->sched.first();
    out[i].n = p->n;
    out[i].s = p->S;
    out[i].ell = p->S;
    P.push_back(std::move(p));
  }
  // QR of every C
  kt.mark(LYAP_K_INIT);
  for (auto& p : P) {
    launch_init<T>(p->C, p->ldc, p->n, p->S, p->glog.template as<double>(), p->partA.template as<double>(), p->partB.template as<double>(),
                   flags_all.template as<int>() + 16 * p->id, p->Vb1.template as<T>(), stream_grid(p->n), st);
    p->hglog.assign(log_stride(p->S), 0.0);
    LYAP_HIP(hipMemcpyAsync(p->hglog.data(), p->glog.p, p->hglog.size() * sizeof(double), hipMemcpyDeviceToHost,
                            st));
  }
  LYAP_HIP(hipMemcpyAsync(hflags.p, flags_all.p, flags_all.bytes, hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  kt.collect();
  for (auto& p : P) {
    const int* f = hflags.template as<int>() + 16 * p->id;
    const double trC = p->hglog[L_FLAG * p->S * p->S + 1];
    LYAP_REQUIRE(f[1] == 0 && std::isfinite(trC), LYAP_E_NUMERIC, "problem %d: C contains NaN or Inf", p->id);
    LYAP_REQUIRE(trC > 0.0, LYAP_E_ARG, "problem %d: C is zero", p->id);
    LYAP_REQUIRE(f[0] == 0, LYAP_E_BREAKDOWN, "problem %d: C is numerically rank deficient", p->id);
    p->beta = std::sqrt(trC);
    out[p->id].beta = p->beta;
  }

  // block widths present, descriptors and work maps per width
  std::vector<int> widths;
  for (auto& p : P)
    if (std::find(widths.begin(), widths.end(), p->S) == widths.end()) widths.push_back(p->S);
  std::sort(widths.begin(), widths.end());
  // descriptors and work map of one block width; updated in stream order
  // from pinned staging (two slots, each reused once its previous copy has
  // executed), so the host never waits for the steps in flight
  struct Group {
    int S;
    std::vector<Problem<T>*> probs;
    DevBuf desc, map;
    HostBuf hdesc[2], hmap[2];
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ev_used[2] = {false, false};
    int slot = 0;
    int nwg = 0;
    int nt = 256;  // threads per workgroup of the group's launches
    Group() = default;
    Group(const Group&) = delete;
    Group& operator=(const Group&) = delete;
    ~Group() {
      for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    }
  };
  std::vector<Group> groups(widths.size());
  for (size_t g = 0; g < widths.size(); ++g) {
    groups[g].S = widths[g];
    groups[g].nt = batch_default_threads(widths[g]);
    for (auto& p : P)
      if (p->S == widths[g]) groups[g].probs.push_back(p.get());
    if (!tune) continue;
    // one workgroup size per group (a template parameter of its launches):
    // the one whose tuned step times sum lowest over the group's problems;
    // then every problem takes its own tuned row count for that size
    double best = 1e300;
    for (int nt : thread_candidates(widths[g])) {
      double tot = 0.0;
      for (Problem<T>* p : groups[g].probs)
        for (auto& sh : p->shapes)
          if (sh.first == nt) tot += sh.second.ms;
      if (tot < best) {
        best = tot;
        groups[g].nt = nt;
      }
    }
    for (Problem<T>* p : groups[g].probs)
      for (auto& sh : p->shapes)
        if (sh.first == groups[g].nt) p->nparts = nparts_for(p->n, sh.second.chunk);
    if (o.verbose)
      std::fprintf(stderr, "[batch] width %d: %d threads per workgroup\n", widths[g], groups[g].nt);
  }
  DevBuf dstep(64);  // the step index of the replayed graphs
  // captured step graphs, one per stretch of steps whose work maps do not
  // change (an upload ends the stretch); destroyed once the stream is idle
  struct StepGraphs {
    hipStream_t st = nullptr;
    std::vector<hipGraph_t> g;
    std::vector<hipGraphExec_t> x;
    ~StepGraphs() {
      if (st) (void)hipStreamSynchronize(st);
      for (auto e : x) (void)hipGraphExecDestroy(e);
      for (auto h : g) (void)hipGraphDestroy(h);
    }
  } sgs;
  sgs.st = st;
  bool sg_valid = false;
  auto upload = [&](Group& g, bool replay, int step) {
    sg_valid = false;
    if (!g.desc.p) {  // sized once: every problem of the group, every workgroup of each
      size_t wgs = 0;
      for (Problem<T>* p : g.probs) wgs += p->nparts;
      wgs = std::max<size_t>(wgs, 1);
      g.desc.alloc(g.probs.size() * sizeof(BatchDesc<T>));
      g.map.alloc(wgs * sizeof(int2));
      for (int sl = 0; sl < 2; ++sl) {
        g.hdesc[sl].alloc(g.probs.size() * sizeof(BatchDesc<T>));
        g.hmap[sl].alloc(wgs * sizeof(int2));
        LYAP_HIP(hipEventCreateWithFlags(&g.ev[sl], hipEventDisableTiming));
      }
    }
    const int sl = g.slot;
    g.slot ^= 1;
    if (g.ev_used[sl]) LYAP_HIP(hipEventSynchronize(g.ev[sl]));  // its previous copies have executed
    BatchDesc<T>* d = g.hdesc[sl].template as<BatchDesc<T>>();
    int2* map = g.hmap[sl].template as<int2>();
    int nmap = 0;
    for (size_t q = 0; q < g.probs.size(); ++q) {
      Problem<T>* p = g.probs[q];
      BatchDesc<T>& b = d[q];
      b = BatchDesc<T>{};
      b.op = p->op.dev;
      b.n = p->n;
      b.nparts = p->nparts;
      b.Vb0 = p->Vb0.template as<T>();
      b.Vb1 = p->Vb1.template as<T>();
      b.W = p->W.template as<T>();
      b.log = p->log.template as<double>();
      b.band = p->band.template as<double>();
      b.partA = p->partA.template as<double>();
      b.partB = p->partB.template as<double>();
      b.flags = flags_all.template as<int>() + 16 * p->id;
      b.ring = p->ring.p ? p->ring.template as<T>() : nullptr;
      b.R = ring_blocks(p->S);
      b.zero = p->zero.template as<T>();
      const bool take = replay ? (step + 1 < p->m_final) : p->active;
      if (take)
        for (int w = 0; w < p->nparts; ++w) map[nmap++] = make_int2((int)q, w);
    }
    // in stream order: the steps launched before read the previous contents
    LYAP_HIP(hipMemcpyAsync(g.desc.p, d, g.probs.size() * sizeof(BatchDesc<T>), hipMemcpyHostToDevice, st));
    if (nmap > 0) LYAP_HIP(hipMemcpyAsync(g.map.p, map, nmap * sizeof(int2), hipMemcpyHostToDevice, st));
    LYAP_HIP(hipEventRecord(g.ev[sl], st));
    g.ev_used[sl] = true;
    g.nwg = nmap;
  };
  for (auto& g : groups) upload(g, false, 0);

  DevBuf chk((size_t)count * sizeof(CheckOut));
  HostBuf hchk((size_t)count * sizeof(CheckOut));
  double check_ms = 0.0;
  constexpr int kAhead = 24;
  // events: kAhead for the step throttle, one for "steps launched so far",
  // one per problem for its check in flight
  struct EventRing {
    std::vector<hipEvent_t> ev;
    ~EventRing() { for (auto e : ev) (void)hipEventDestroy(e); }
  } er;
  er.ev.resize(kAhead + 1 + 2 * count);
  for (auto& e : er.ev) LYAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipEvent_t ev_step = er.ev[kAhead];
  hipEvent_t* ev_chk = &er.ev[kAhead + 1];
  hipEvent_t* ev_start = &er.ev[kAhead + 1 + count];
  // a problem's check is launched as soon as it is due (its stream waits for
  // the steps launched so far) and processed as soon as its own event has
  // completed, independently of the other problems' checks
  std::vector<char> chk_pending(count, 0);
  std::vector<int> chk_mm(count, 0);
  int n_pending = 0;
  int n_active = count;
  auto launch_check = [&](Problem<T>* p, int j) {
    // the check reads T_m's band and the log up to step mm, written by the
    // steps launched so far on the solver's stream
    hipStream_t cq = cstream(p->id);
    if (overlap) LYAP_HIP(hipEventRecord(ev_start[p->id], st));
    kt.mark(LYAP_K_CHECK);
    const int mm = std::min(p->next_check, j);
    if (overlap) LYAP_HIP(hipStreamWaitEvent(cq, ev_start[p->id], 0));
    const size_t LS = log_stride(p->S);
    p->ck->run(p->band.template as<double>(), mm * p->S, p->glog.template as<double>() + L_R * p->S * p->S,
               p->log.template as<double>() + (size_t)(mm - 1) * LS + L_R * p->S * p->S,
               chk.template as<CheckOut>() + p->id);
    LYAP_HIP(hipMemcpyAsync(hchk.template as<CheckOut>() + p->id, chk.template as<CheckOut>() + p->id,
                            sizeof(CheckOut), hipMemcpyDeviceToHost, cq));
    LYAP_HIP(hipMemcpyAsync(hflags.template as<int>() + 16 * p->id, flags_all.template as<int>() + 16 * p->id,
                            2 * sizeof(int), hipMemcpyDeviceToHost, cq));
    LYAP_HIP(hipEventRecord(ev_chk[p->id], cq));
    chk_pending[p->id] = 1;
    chk_mm[p->id] = mm;
    ++n_pending;
  };
  // a check at m on problem p's stream, waited for (breakdown re-checks)
  auto check_now = [&](Problem<T>* p, int mm) {
    LYAP_HIP(hipStreamSynchronize(st));
    const size_t LS = log_stride(p->S);
    hipStream_t cq = cstream(p->id);
    p->ck->run(p->band.template as<double>(), mm * p->S, p->glog.template as<double>() + L_R * p->S * p->S,
               p->log.template as<double>() + (size_t)(mm - 1) * LS + L_R * p->S * p->S,
               chk.template as<CheckOut>() + p->id);
    LYAP_HIP(hipMemcpyAsync(hchk.template as<CheckOut>() + p->id, chk.template as<CheckOut>() + p->id,
                            sizeof(CheckOut), hipMemcpyDeviceToHost, cq));
    LYAP_HIP(hipStreamSynchronize(cq));
  };
  // the result of p's completed check; returns true when p left the active set
  auto process_check = [&](Problem<T>* p) {
    chk_pending[p->id] = 0;
    --n_pending;
    int mm = chk_mm[p->id];
    const int* f = hflags.template as<int>() + 16 * p->id;
    LYAP_REQUIRE(!(f[1] > 0 && f[1] <= mm && (f[0] == 0 || f[1] <= f[0])), LYAP_E_NUMERIC,
                 "problem %d: non-finite values at step %d", p->id, f[1]);
    bool broke = false;
    if (f[0] > 0 && f[0] <= mm) {
      mm = f[0];
      broke = true;
      check_now(p, mm);
    }
    const CheckOut& c = hchk.template as<CheckOut>()[p->id];
    LYAP_REQUIRE(std::isfinite(c.res), LYAP_E_NUMERIC, "problem %d: residual not finite", p->id);
    LYAP_REQUIRE(c.lam_max < 0.0, LYAP_E_INDEFINITE, "problem %d: Ritz value %.3e >= 0", p->id, c.lam_max);
    const double rel = c.res / (p->beta * p->beta);
    p->hm.push_back(mm);
    p->hr.push_back(rel);
    p->last_res = rel;
    p->checked_m = mm;
    p->lam_absmax = std::max(std::fabs(c.lam_min), std::fabs(c.lam_max));
    out[p->id].n_checks++;
    if (o.verbose) std::fprintf(stderr, "[batch] problem %d m=%d res=%.3e\n", p->id, mm, rel);
    if (rel <= o.tol) {
      p->status = LYAP_OK;
      p->m_final = mm;
      p->active = false;
      p->t_to_tol = ms_since(t_entry);
    } else if (broke) {
      p->status = LYAP_E_BREAKDOWN;
      p->m_final = mm;
      p->active = false;
    } else if (mm >= maxit) {
      p->m_final = mm;
      p->active = false;
    } else {
      p->next_check = p->sched.next(mm, rel, o.tol);
    }
    if (!p->active) {
      --n_active;
      return true;
    }
    return false;
  };
  // process every completed check (all pending ones when wait is set)
  auto poll_checks = [&](bool wait) {
    bool changed = false;
    for (auto& p : P) {
      if (!chk_pending[p->id]) continue;
      if (wait) {
        const auto t0 = Clock::now();
        LYAP_HIP(hipEventSynchronize(ev_chk[p->id]));
        check_ms += ms_since(t0);
      } else {
        const hipError_t q = hipEventQuery(ev_chk[p->id]);
        if (q == hipErrorNotReady) continue;
        LYAP_HIP(q);
      }
      changed = process_check(p.get()) || changed;
    }
    if (changed)
      for (auto& g : groups) upload(g, false, 0);
    if (!overlap) kt.collect();
  };

  // one step of every group as a graph: the kernels read the step index from
  // dstep, which the graph's last node advances
  auto capture_step = [&](int j0) {
    int* jp = dstep.template as<int>();
    hipLaunchKernelGGL(k_step_set, dim3(1), dim3(64), 0, st, jp, j0);
    LYAP_LAUNCHED("k_step_set");
    LYAP_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipGraph_t gr = nullptr;
    try {
      for (auto& g : groups)
        if (g.nwg > 0)
          launch_batch_step<T>(g.desc.template as<BatchDesc<T>>(), g.map.template as<int2>(), g.nwg, g.S, g.nt, j0,
                               st, nullptr, jp);
      hipLaunchKernelGGL(k_step_next, dim3(1), dim3(64), 0, st, jp);
      LYAP_LAUNCHED("k_step_next");
    } catch (...) {
      (void)hipStreamEndCapture(st, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      throw;
    }
    LYAP_HIP(hipStreamEndCapture(st, &gr));
    sgs.g.push_back(gr);
    hipGraphExec_t ex = nullptr;
    LYAP_HIP(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
    sgs.x.push_back(ex);
    sg_valid = true;
  };

  const auto t_pass1 = Clock::now();
  // host time by activity (printed with opts->verbose)
  double h_poll = 0.0, h_check = 0.0, h_wait = 0.0, h_step = 0.0;
  int n_launched_checks = 0;
  int j = 0;
  while (n_active > 0) {
    auto th = Clock::now();
    if (n_pending > 0) poll_checks(!overlap);
    h_poll += ms_since(th);
    if (n_active == 0) break;
    // launch the checks that are due now
    th = Clock::now();
    for (auto& p : P) {
      if (!p->active || chk_pending[p->id]) continue;
      if (j >= p->next_check || j >= maxit) {
        launch_check(p.get(), j);
        ++n_launched_checks;
      }
    }
    h_check += ms_since(th);
    if (!overlap && n_pending > 0) continue;
    if (j >= maxit) {
      // every remaining active problem has a check in flight: wait for them
      if (n_pending > 0) poll_checks(true);
      continue;
    }
    // a problem whose check is still in flight keeps stepping (its next check
    // is decided when the result arrives)
    th = Clock::now();
    if (j >= kAhead) LYAP_HIP(hipEventSynchronize(er.ev[j % kAhead]));
    h_wait += ms_since(th);
    th = Clock::now();
    if (graphs) {
      if (!sg_valid) capture_step(j);
      LYAP_HIP(hipGraphLaunch(sgs.x.back(), st));
    } else {
      for (auto& g : groups)
        if (g.nwg > 0)
          launch_batch_step<T>(g.desc.template as<BatchDesc<T>>(), g.map.template as<int2>(), g.nwg, g.S, g.nt, j,
                               st, &kt);
    }
    LYAP_HIP(hipEventRecord(er.ev[j % kAhead], st));
    h_step += ms_since(th);
    ++j;
    for (auto& p : P)
      if (p->active) p->m = j;
  }
  if (o.verbose)
    std::fprintf(stderr,
                 "[batch] pass 1: %d steps, %d checks; host ms: polling %.1f, check launches %.1f, "
                 "step throttle waits %.1f, step launches %.1f\n",
                 j, n_launched_checks, h_poll, h_check, h_wait, h_step);
  if (n_pending > 0) poll_checks(true);
  if (overlap)
    for (int i = 0; i < count; ++i) LYAP_HIP(hipStreamWaitEvent(st, ev_chk[i], 0));
  for (auto& p : P)
    if (p->m_final == 0) p->m_final = p->m;
  const double pass1_ms = ms_since(t_pass1) - check_ms;

  // ---- finalisation per problem
  const auto t_fin = Clock::now();
  kt.mark(LYAP_K_FINAL);
  for (auto& p : P) {
    const int S = p->S;
    const size_t LS = log_stride(S);
    if (p->checked_m != p->m_final) {  // (only when max_iter ended without a due check)
      LYAP_HIP(hipStreamSynchronize(st));
      p->ck->run(p->band.template as<double>(), p->m_final * S, p->glog.template as<double>() + L_R * S * S,
                 p->log.template as<double>() + (size_t)(p->m_final - 1) * LS + L_R * S * S, chk.template as<CheckOut>() + p->id);
      LYAP_HIP(hipMemcpyAsync(hchk.template as<CheckOut>() + p->id, chk.template as<CheckOut>() + p->id, sizeof(CheckOut),
                              hipMemcpyDeviceToHost, cstream(p->id)));
      LYAP_HIP(hipStreamSynchronize(cstream(p->id)));
      const CheckOut& c = hchk.template as<CheckOut>()[p->id];
      p->last_res = c.res / (p->beta * p->beta);
      p->hm.push_back(p->m_final);
      p->hr.push_back(p->last_res);
      p->lam_absmax = std::max(std::fabs(c.lam_min), std::fabs(c.lam_max));
    }
  }
  // tau_{m+1,m} of every problem in one pass (for the truncation threshold)
  HostBuf htau((size_t)count * 64 * sizeof(double));
  for (auto& p : P) {
    const int S = p->S;
    LYAP_HIP(hipMemcpyAsync(htau.template as<double>() + 64 * p->id,
                            p->log.template as<double>() + (size_t)(p->m_final - 1) * log_stride(S) + L_R * S * S,
                            S * S * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  LYAP_HIP(hipStreamSynchronize(st));
  // the problems are finalised side by side, each on its check stream: the
  // pivoted Cholesky factorisations advance in turn (32 pivots per round, one
  // wait per round for all of them), then every shifted solve and assembly
  std::vector<std::unique_ptr<FinaliseJob>> jobs(count);
  for (auto& p : P) {
    const int S = p->S;
    const double* tau = htau.template as<double>() + 64 * p->id;
    double tf = 0.0;
    for (int i = 0; i < S * S; ++i) tf += tau[i] * tau[i];
    tf = std::sqrt(tf);
    const double b2 = p->beta * p->beta;
    double eps = o.trunc_eps;
    if (!(eps >= 0.0)) eps = std::min(1e-12, 0.05 * o.tol / (p->lam_absmax + tf)) * b2;
    out[p->id].trunc_eps = eps;
    jobs[p->id] = std::make_unique<FinaliseJob>(*p->ck, p->band.template as<double>(),
                                                p->glog.template as<double>() + L_R * S * S, eps, cstream(p->id));
  }
  auto sync_checks = [&]() {
    if (overlap)
      for (int i = 0; i < kCS; ++i) LYAP_HIP(hipStreamSynchronize(cs.s[i]));
    else
      LYAP_HIP(hipStreamSynchronize(st));
  };
  for (;;) {
    std::vector<int> launched;
    for (auto& p : P)
      if (jobs[p->id]->pchol_launch()) launched.push_back(p->id);
    if (launched.empty()) break;
    sync_checks();
    for (int id : launched) jobs[id]->pchol_read();
  }
  for (auto& p : P) p->t = jobs[p->id]->launch_tail(p->M);
  sync_checks();
  for (auto& p : P) jobs[p->id]->finish();
  jobs.clear();
  kt.collect();
  const double fin_ms = ms_since(t_fin);

  // ---- second pass, grouped
  const auto t_p2 = Clock::now();
  int mmax = 0;
  for (auto& p : P) {
    bool owned = false;
    out[p->id].Z = alloc_output(o, (size_t)p->n * std::max(p->t, 1) * sizeof(double), &owned);
    out[p->id].owns_Z = owned ? 1 : 0;
    const int R = ring_blocks(p->S);
    p->ring.alloc((size_t)R * p->n * p->S * sizeof(T));
    if (p->t > 0) {
      LYAP_HIP(hipMemsetAsync(out[p->id].Z, 0, (size_t)p->n * p->t * sizeof(double), st));
      launch_init_store<T>(p->C, p->ldc, p->n, p->S, p->glog.template as<double>(), p->ring.template as<T>(), stream_grid(p->n), st);
      mmax = std::max(mmax, p->m_final);
    }
  }
  // problems with t == 0 take no part in the replay
  for (auto& p : P)
    if (p->t <= 0) p->m_final = 0;
  for (auto& g : groups) upload(g, true, 0);
  std::vector<int> first(count, 0);
  std::vector<std::vector<const void*>> pend(count);
  // Z accumulation beside the replays: a flush of blocks [f, f + cnt) waits for
  // the replays launched so far (the last of its blocks was written by replay
  // f + cnt - 2), and replay f + R - 1, the first to overwrite one of its ring
  // slots (block f + R), waits for the flush.  At most two flushes of a problem
  // are outstanding, so four events per problem rotate.
  constexpr int kFlushEv = 4;
  struct FlushWait {
    int step;
    hipEvent_t ev;
  };
  std::vector<std::deque<FlushWait>> fwait(count);
  struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool() { for (auto e : ev) (void)hipEventDestroy(e); }
  } fpool;
  std::vector<int> fnext(count, 0);
  if (overlap) {
    fpool.ev.resize((size_t)count * kFlushEv + 1);
    for (auto& e : fpool.ev) LYAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  for (int i = 0; i < mmax; ++i) {
    bool map_changes = false;
    if (overlap)
      for (auto& p : P)
        while (!fwait[p->id].empty() && fwait[p->id].front().step <= i) {
          LYAP_HIP(hipStreamWaitEvent(st, fwait[p->id].front().ev, 0));
          fwait[p->id].pop_front();
        }
    for (auto& g : groups) {
      if (g.nwg > 0) {
        kt.mark(LYAP_K_REPLAY);
        launch_batch_replay<T>(g.desc.template as<BatchDesc<T>>(), g.map.template as<int2>(), g.nwg, g.S, g.nt, i, st);
      }
      for (Problem<T>* p : g.probs)
        if (i + 2 == p->m_final) map_changes = true;  // leaves the replay map after this step
    }
    bool replays_marked = false;
    for (auto& p : P) {
      if (i >= p->m_final) continue;
      const int S = p->S;
      const int R = ring_blocks(S);
      if (pend[p->id].empty()) first[p->id] = i;
      pend[p->id].push_back(p->ring.template as<T>() + (size_t)(i % R) * p->n * S);
      // (the first flush of each problem is shortened by a problem-dependent
      // amount so that the problems' flushes spread over the replay steps)
      const int flen = zflush_max_blocks(S) - (overlap && first[p->id] == 0 ? (p->id * 17) % 32 : 0);
      if ((int)pend[p->id].size() == flen || i == p->m_final - 1) {
        hipStream_t fq = st;
        if (overlap) {
          fq = cstream(p->id);
          hipEvent_t er_ = fpool.ev.back();
          if (!replays_marked) LYAP_HIP(hipEventRecord(er_, st));
          replays_marked = true;
          LYAP_HIP(hipStreamWaitEvent(fq, er_, 0));
        }
        kt.mark(LYAP_K_ZFLUSH);
        launch_zflush<T>(pend[p->id].data(), (int)pend[p->id].size(), p->n, S,
                         p->M.template as<double>() + (size_t)first[p->id] * S * p->t, p->t, out[p->id].Z, p->n, 0, fq);
        if (overlap) {
          hipEvent_t fe = fpool.ev[(size_t)p->id * kFlushEv + fnext[p->id]];
          fnext[p->id] = (fnext[p->id] + 1) % kFlushEv;
          LYAP_HIP(hipEventRecord(fe, fq));
          fwait[p->id].push_back(FlushWait{first[p->id] + R - 1, fe});
        }
        pend[p->id].clear();
      }
    }
    if (map_changes)
      for (auto& g : groups) upload(g, true, i + 1);
  }
  LYAP_HIP(hipStreamSynchronize(st));
  if (overlap) sync_checks();
  kt.collect();
  const double p2_ms = ms_since(t_p2);

  lyap_status worst = LYAP_OK;
  for (auto& p : P) {
    lyap_result& r = out[p->id];
    r.m = p->m_final;
    r.t = p->t;
    r.res = p->last_res;
    r.status = p->status;
    store_history(&r, p->hm, p->hr);
    r.times_ms[LYAP_T_PASS1] = pass1_ms;
    r.times_ms[LYAP_T_CHECKS] = check_ms;
    r.times_ms[LYAP_T_FINAL] = fin_ms;
    r.times_ms[LYAP_T_PASS2] = p2_ms;
    r.times_ms[LYAP_T_TOTAL] = ms_since(t_entry);
    r.times_ms[LYAP_T_TO_TOL] = p->t_to_tol;
    if (p->status != LYAP_OK && (worst == LYAP_OK || p->status < 0)) worst = p->status;
  }
  // batch-level kernel times in the first result
  for (int i = 0; i < LYAP_K_COUNT; ++i) {
    out[0].kern_ms[i] = kt.ms[i];
    out[0].kern_n[i] = kt.n[i];
  }
  return worst;
}

}  // namespace
}  // namespace lyap

extern "C" lyap_status lyap_solve_batched(int32_t count, const lyap_op* A, const double* const* C, const int32_t* s,
                                          const int64_t* ldc, const lyap_opts* opts, int32_t tune,
                                          lyap_result* out) {
  using namespace lyap;
  clear_error();
  if (!out || count <= 0 || !A || !C || !s || !ldc) {
    set_error("bad arguments (count <= 0 or NULL array)");
    return LYAP_E_ARG;
  }
  for (int i = 0; i < count; ++i) std::memset(&out[i], 0, sizeof(lyap_result));
  lyap_opts o;
  if (opts) o = *opts;
  else lyap_opts_default(&o);
  try {
    for (int i = 0; i < count; ++i) {
      validate_op(&A[i]);
      LYAP_REQUIRE(C[i] != nullptr, LYAP_E_ARG, "problem %d: C is NULL", i);
      LYAP_REQUIRE(s[i] >= 1 && s[i] <= 8, LYAP_E_ARG, "problem %d: s=%d out of range 1..8", i, s[i]);
      LYAP_REQUIRE(ldc[i] >= A[i].n && s[i] <= A[i].n, LYAP_E_ARG, "problem %d: bad ldc or s > n", i);
    }
    LYAP_REQUIRE(o.tol > 0.0 && o.tol < 1.0, LYAP_E_ARG, "tol=%g must be in (0,1)", o.tol);
    LYAP_REQUIRE(o.max_iter >= 1 && (int64_t)o.max_iter * 8 <= (int64_t)1 << 20, LYAP_E_ARG,
                 "max_iter=%d out of range", o.max_iter);
    LYAP_REQUIRE(o.check_every >= 0, LYAP_E_ARG, "check_every must be >= 0");
    LYAP_REQUIRE((tune & ~(3 | LYAP_BATCH_GRAPHS)) == 0 && (tune & 3) <= 2, LYAP_E_ARG,
                 "tune=%d must be 0, 1 or 2, optionally with LYAP_BATCH_GRAPHS", tune);
    LYAP_REQUIRE(!(tune & LYAP_BATCH_GRAPHS) || o.profile == 0, LYAP_E_ARG,
                 "LYAP_BATCH_GRAPHS cannot be combined with per-kernel profiling");
    LYAP_REQUIRE(o.method == LYAP_METHOD_STD, LYAP_E_UNSUPPORTED, "the batched solver builds standard Krylov spaces");
    LYAP_REQUIRE(o.two_pass != 0, LYAP_E_UNSUPPORTED, "the batched solver uses the two-pass strategy");
    LYAP_REQUIRE(o.storage == LYAP_STORE_F64 || o.storage == LYAP_STORE_F32, LYAP_E_ARG, "unknown storage %d",
                 o.storage);
    // the per-problem buffers (a few thousand, most of them small) come from
    // the device block cache and go back to it: every buffer is released
    // after the streams that use it have been synchronised
    BlockCacheScope cache;
    return o.storage == LYAP_STORE_F64 ? batched_impl<double>(count, A, C, s, ldc, o, tune, out)
                                       : batched_impl<float>(count, A, C, s, ldc, o, tune, out);
  } catch (const Error& e) {
    for (int i = 0; i < count; ++i)
      if (out[i].status == 0) out[i].status = e.st;
    return e.st;
  }
}
