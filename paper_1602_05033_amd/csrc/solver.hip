// lyap_solve for the standard block Krylov space: Algorithm 1 driving the
// block Lanczos kernels, the GPU residual check of Proposition 1 on the
// schedule chosen below, the truncated factor of Y~ and the second Lanczos
// pass of Section 3.3 (or the stored basis).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <limits>
#include <type_traits>
#include <memory>
#include <vector>

#include "check.hpp"
#include "lanczos.hpp"
#include "side.hpp"
#include "solver.hpp"

using namespace lyap;

extern "C" void lyap_opts_default(lyap_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->max_iter = 5000;
  o->method = LYAP_METHOD_STD;
  o->check_every = 0;
  o->storage = LYAP_STORE_F64;
  o->two_pass = 1;
  o->trunc_eps = -1.0;
  o->inner_pc = LYAP_PC_JACOBI;
  o->inner_tol = 1e-12;
  o->inner_max_iter = 5000;
  o->flush_blocks = 0;
}

extern "C" void lyap_result_free(lyap_result* r) {
  if (!r) return;
  std::free(r->hist_m);
  std::free(r->hist_res);
  std::free(r->T_band);
  std::free(r->gamma);
  std::free(r->tau);
  if (r->Z && r->owns_Z) (void)hipFree(r->Z);
  std::memset(r, 0, sizeof(*r));
}

namespace lyap {

double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// -------------------------------------------------------------- check schedule
int CheckSchedule::first() const {
  if (d > 0) return std::min(d, max_iter);
  return std::min(10, max_iter);
}

int CheckSchedule::next(int m, double res, double tol) {
  hist.emplace_back(m, std::log10(std::max(res, 1e-300)));
  if (d > 0) return std::min(m + d, max_iter);
  const int grow_by = std::max(5, (int)(this->grow * m));
  int nxt = m + grow_by;
  if (hist.size() >= 2) {
    const auto& a = hist[hist.size() - 2];
    const auto& b = hist[hist.size() - 1];
    const double slope = (b.second - a.second) / double(b.first - a.first);
    if (slope < 0) {
      const double gap = (std::log10(tol) - b.second) / slope;  // steps to the predicted crossing
      const int step = (int)std::ceil(aim * gap);
      nxt = m + std::max(1, std::min(step, grow_by));
    }
  }
  return std::min(nxt, max_iter);
}

// One residual check in flight: its stream (owned unless it is the solver's),
// completion event, workspace and result buffers, and the step it checks.
struct CheckSlot {
  hipStream_t st = nullptr;
  bool own = false;
  hipEvent_t ev = nullptr;
  std::unique_ptr<Checker> ck;
  DevBuf chk;
  HostBuf hchk, hflags;
  int mm = 0;
  ~CheckSlot() {
    // a check still running reads the Lanczos side's buffers: let it end
    if (own && st) (void)hipStreamSynchronize(st);
    if (ev) (void)hipEventDestroy(ev);
    if (own && st) (void)hipStreamDestroy(st);
  }
};

// -------------------------------------------------------------- result helpers
void store_history(lyap_result* out, const std::vector<int>& hm, const std::vector<double>& hr) {
  out->n_hist = (int)hm.size();
  out->hist_m = (int32_t*)std::malloc(std::max<size_t>(1, hm.size()) * sizeof(int32_t));
  out->hist_res = (double*)std::malloc(std::max<size_t>(1, hr.size()) * sizeof(double));
  for (size_t i = 0; i < hm.size(); ++i) {
    out->hist_m[i] = hm[i];
    out->hist_res[i] = hr[i];
  }
}

double* alloc_output(const lyap_opts& o, size_t bytes, bool* owned) {
  void* p = nullptr;
  if (o.alloc) {
    p = o.alloc(bytes ? bytes : 8, o.alloc_ctx);
    LYAP_REQUIRE(p != nullptr, LYAP_E_NOMEM, "allocator callback returned NULL for %zu bytes", bytes);
    *owned = false;
  } else {
    hipError_t e = hipMalloc(&p, bytes ? bytes : 8);
    LYAP_REQUIRE(e == hipSuccess, LYAP_E_NOMEM, "hipMalloc(%zu) for Z failed", bytes);
    *owned = true;
  }
  return (double*)p;
}

void rowmajor_to_colmajor(const double* rm, int rows, int cols, double* cm) {
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) cm[i + (size_t)j * rows] = rm[(size_t)i * cols + j];
}

// Algorithmic HBM bytes per launch of the streaming kernels (per-row model).
template <typename T>
void fill_kernel_bytes(int n, int S, double coef, const KernelTimer& kt, double zflush_bytes, double* kb) {
  const double nsb = (double)n * S * sizeof(T);
  kb[LYAP_K_SPMM_GRAM] = 3.0 * nsb + coef * n;
  // CGS2 (S <= 4): two update sweeps of 4 nsb; block MGS twice: four of 3.75 nsb on average
  kb[LYAP_K_UPD_GRAM] = (S <= 4 ? 4.0 : 3.75) * nsb;
  kb[LYAP_K_CHOL_GRAM] = 1.0 * nsb;
  kb[LYAP_K_CHOL_STORE] = 2.0 * nsb;
  kb[LYAP_K_REPLAY] = 3.0 * nsb + coef * n;
  kb[LYAP_K_ZFLUSH] = kt.n[LYAP_K_ZFLUSH] > 0 ? zflush_bytes / kt.n[LYAP_K_ZFLUSH] : 0.0;
}
template void fill_kernel_bytes<float>(int, int, double, const KernelTimer&, double, double*);
template void fill_kernel_bytes<double>(int, int, double, const KernelTimer&, double, double*);

// -------------------------------------------------------------- one Krylov space
template <typename T>
LanczosSide<T>::LanczosSide(const lyap_op* A, const double* C, int S, int64_t ldc, int max_iter, bool two_pass,
                            hipStream_t st, KernelTimer* kt)
    : C_(C), ldc_(ldc), n_((int)A->n), S_(S), maxit_(max_iter), two_pass_(two_pass), st_(st), kt_(kt) {
  if constexpr (std::is_same_v<T, double>) make_op_f64(A, op_, st);
  else make_op_f32(A, op_, st);
  blk_ = (size_t)n_ * S * sizeof(T);
  LS_ = log_stride(S);
  grid_ = stream_grid(n_);
  Vb0_.alloc(blk_);
  Vb1_.alloc(blk_);
  Wb_.alloc(blk_);
  zero_.alloc(blk_);
  logb_.alloc(((size_t)maxit_ + 1) * LS_ * sizeof(double));
  glog_.alloc(LS_ * sizeof(double));
  band_.alloc((size_t)(S + 1) * S * (maxit_ + 2) * sizeof(double));
  // partial Gram matrices of every workgroup: 2 S x S per workgroup in the CGS2 sweeps
  partA_.alloc((size_t)kSGrid * 2 * S * S * sizeof(double));
  partB_.alloc((size_t)kSGrid * 2 * S * S * sizeof(double));
  flags_.alloc(64);
  hflags_.alloc(64);
  LYAP_HIP(hipMemsetAsync(flags_.p, 0, 64, st_));
  LYAP_HIP(hipMemsetAsync(zero_.p, 0, blk_, st_));
  LYAP_HIP(hipMemsetAsync(Vb0_.p, 0, blk_, st_));
  LYAP_HIP(hipMemsetAsync(band_.p, 0, band_.bytes, st_));
}

template <typename T>
void LanczosSide<T>::init() {
  T* V1p = two_pass_ ? Vb1_.as<T>() : nullptr;
  if (!two_pass_) {
    stored_.emplace_back(blk_);
    V1p = stored_.back().as<T>();
  }
  if (kt_) kt_->mark(LYAP_K_INIT);
  launch_init<T>(C_, ldc_, n_, S_, glog_.as<double>(), partA_.as<double>(), partB_.as<double>(), flags_.as<int>(),
                 V1p, grid_, st_);
  hglog_.assign(LS_, 0.0);
  LYAP_HIP(hipMemcpyAsync(hglog_.data(), glog_.p, LS_ * sizeof(double), hipMemcpyDeviceToHost, st_));
  LYAP_HIP(hipMemcpyAsync(hflags_.p, flags_.p, 64, hipMemcpyDeviceToHost, st_));
  LYAP_HIP(hipStreamSynchronize(st_));
  const int* f = hflags_.as<int>();
  const double trC = hglog_[L_FLAG * S_ * S_ + 1];
  LYAP_REQUIRE(f[1] == 0 && std::isfinite(trC), LYAP_E_NUMERIC, "C contains NaN or Inf");
  LYAP_REQUIRE(trC > 0.0, LYAP_E_ARG, "C is zero");
  LYAP_REQUIRE(f[0] == 0, LYAP_E_BREAKDOWN, "C is numerically rank deficient (deflation not implemented)");
  beta_ = std::sqrt(trC);
  Vprev_ = two_pass_ ? Vb0_.as<T>() : zero_.as<T>();
  Vcur_ = V1p;
}

template <typename T>
void LanczosSide<T>::step() {
  T* Vnext;
  if (two_pass_) {
    Vnext = Vprev_;  // V_{j+1} overwrites V_{j-1}
  } else {
    stored_.emplace_back(blk_);
    Vnext = stored_.back().as<T>();
  }
  StepArgs<T> sa{};
  sa.op = op_.dev;
  sa.n = n_;
  sa.W = Wb_.as<T>();
  sa.band = band_.as<double>();
  sa.flags = flags_.as<int>();
  sa.Vprev = Vprev_;
  sa.Vcur = Vcur_;
  sa.Vnext = Vnext;
  sa.log = logb_.as<double>() + (size_t)m_ * LS_;
  sa.j = m_;
  launch_step<T>(sa, S_, grid_, partA_.as<double>(), partB_.as<double>(), st_, kt_);
  ++m_;
  Vprev_ = Vcur_;
  Vcur_ = Vnext;
}

template <typename T>
void LanczosSide<T>::read_flags(int* breakdown, int* nonfinite) {
  LYAP_HIP(hipMemcpyAsync(hflags_.p, flags_.p, 64, hipMemcpyDeviceToHost, st_));
  LYAP_HIP(hipStreamSynchronize(st_));
  *breakdown = hflags_.as<int>()[0];
  *nonfinite = hflags_.as<int>()[1];
}

template <typename T>
void LanczosSide<T>::accumulate_Z(int m, const double* Mrows, int t, double* Z, int64_t ldz, double* bytes_out) {
  const int S = S_;
  const int n = n_;
  double zbytes = 0.0;
  if (t > 0) {
    LYAP_HIP(hipMemsetAsync(Z, 0, (size_t)ldz * t * sizeof(double), st_));
    const int QB = zflush_max_blocks(S);
    if (two_pass_) {
      // Without per-kernel timing the Z accumulation runs on a stream of its
      // own beside the replays: a flush of blocks [f, f + cnt) waits for the
      // replays launched so far, and the replay that first overwrites one of
      // its ring slots (block f + R) waits for the flush; the ring holds two
      // flushes' blocks.  The flushes stay in order on their stream, so Z has
      // the same bits either way.
      const bool side_z = kt_ == nullptr || !kt_->on;
      const int R = (side_z ? 2 : 1) * QB + 2;
      DevBuf ringbuf((size_t)R * blk_);
      auto slot = [&](int i) { return (T*)((char*)ringbuf.p + (size_t)(i % R) * blk_); };
      struct ZStream {
        hipStream_t s = nullptr;
        std::vector<hipEvent_t> ev;
        ~ZStream() {
          if (s) (void)hipStreamSynchronize(s);
          for (auto e : ev) (void)hipEventDestroy(e);
          if (s) (void)hipStreamDestroy(s);
        }
      } zs;
      constexpr int kZEv = 4;  // at most two flushes outstanding
      if (side_z) {
        LYAP_HIP(hipStreamCreateWithFlags(&zs.s, hipStreamNonBlocking));
        zs.ev.resize(kZEv + 1);
        for (auto& e : zs.ev) LYAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      }
      std::vector<std::pair<int, hipEvent_t>> waits;  // (replay step, flush done)
      int nev = 0;
      launch_init_store<T>(C_, ldc_, n, S, glog_.as<double>(), slot(0), grid_, st_);
      std::vector<const void*> pend;
      int first = 0;
      for (int i = 0; i < m; ++i) {
        if (i + 1 < m) {
          while (!waits.empty() && waits.front().first <= i) {
            LYAP_HIP(hipStreamWaitEvent(st_, waits.front().second, 0));
            waits.erase(waits.begin());
          }
          const T* vp = i > 0 ? slot(i - 1) : zero_.as<T>();
          if (kt_) kt_->mark(LYAP_K_REPLAY);
          launch_replay<T>(op_.dev, S, vp, slot(i), slot(i + 1), logb_.as<double>() + (size_t)i * LS_, grid_, st_);
        }
        if (pend.empty()) first = i;
        pend.push_back(slot(i));
        if ((int)pend.size() == QB || i == m - 1) {
          if (kt_) kt_->mark(LYAP_K_ZFLUSH);
          zbytes += (double)pend.size() * blk_ + 2.0 * n * t * sizeof(double);
          hipStream_t fq = st_;
          if (side_z) {
            LYAP_HIP(hipEventRecord(zs.ev[kZEv], st_));
            LYAP_HIP(hipStreamWaitEvent(zs.s, zs.ev[kZEv], 0));
            fq = zs.s;
          }
          launch_zflush<T>(pend.data(), (int)pend.size(), n, S, Mrows + (size_t)first * S * t, t, Z, ldz, 0, fq);
          if (side_z) {
            hipEvent_t fe = zs.ev[nev];
            nev = (nev + 1) % kZEv;
            LYAP_HIP(hipEventRecord(fe, zs.s));
            waits.emplace_back(first + R - 1, fe);
          }
          pend.clear();
        }
      }
      if (side_z) LYAP_HIP(hipStreamSynchronize(zs.s));
      LYAP_HIP(hipStreamSynchronize(st_));  // the ring is released on return
    } else {
      std::vector<const void*> ptrs;
      for (int i = 0; i < m; ++i) ptrs.push_back(stored_[i].p);
      if (kt_) kt_->mark(LYAP_K_ZFLUSH);
      zbytes += (double)m * blk_ + 2.0 * n * t * sizeof(double) * ((m + QB - 1) / QB);
      launch_zflush<T>(ptrs.data(), m, n, S, Mrows, t, Z, ldz, 0, st_);
    }
  }
  if (bytes_out) *bytes_out += zbytes;
}

template class LanczosSide<float>;
template class LanczosSide<double>;

// -------------------------------------------------------------- standard Krylov
template <typename T>
lyap_status solve_std(const lyap_op* A, const double* C, int S, int64_t ldc, const lyap_opts& o, lyap_result* out) {
  const auto t_entry = Clock::now();
  hipStream_t st = (hipStream_t)o.stream;
  const int n = (int)A->n;
  out->n = n;
  out->s = S;
  out->ell = S;
  const int maxit = o.max_iter;
  KernelTimer kt;
  kt.st = st;
  kt.on = o.profile != 0;
  LanczosSide<T> side(A, C, S, ldc, maxit, o.two_pass != 0, st, &kt);

  side.init();
  out->beta = side.beta();
  const double beta2 = out->beta * out->beta;

  // Residual checks run on other streams while the Lanczos steps continue:
  // a check at mm reads only T_mm's band, gamma and tau_{mm+1,mm}, which later
  // steps never write.  The host keeps at most kAhead steps queued ahead of
  // the GPU, so after the converging check the extra steps are few; they are
  // simply not used (the accepted basis is the checked one).  With a fixed
  // schedule (opts->check_every > 0) the check points do not depend on the
  // results, so up to kSlots checks run at once, each on a stream and with a
  // workspace of its own, and are read in the order they were issued: the
  // first that meets the tolerance ends the iteration, exactly as with one
  // check at a time (later ones still running are not used), and the steps
  // stay at most kAhead past the next check point.  The adaptive schedule
  // places each check from the previous result: one at a time.  With
  // opts->profile the checks run on the solver's stream, one at a time.
  constexpr int kAhead = 24, kSlots = 3;
  const bool overlap = o.profile == 0;
  const bool fixed = o.check_every > 0;
  const int nslots = overlap && fixed ? kSlots : 1;
  std::vector<std::unique_ptr<CheckSlot>> slots;
  for (int i = 0; i < nslots; ++i) {
    slots.emplace_back(new CheckSlot);
    CheckSlot& sl = *slots.back();
    if (overlap) {
      LYAP_HIP(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking));
      sl.own = true;
    } else {
      sl.st = st;
    }
    LYAP_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    sl.ck.reset(new Checker(S, S, sl.st));
    sl.chk.alloc(sizeof(CheckOut));
    sl.hchk.alloc(sizeof(CheckOut));
    sl.hflags.alloc(64);
  }
  struct EventRing {
    std::vector<hipEvent_t> ev;
    ~EventRing() { for (auto e : ev) (void)hipEventDestroy(e); }
  } er;
  er.ev.resize(kAhead + 1);
  for (auto& e : er.ev) LYAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipEvent_t ev_step = er.ev[kAhead];

  CheckSchedule sched{o.check_every, maxit};
  std::vector<int> hm;
  std::vector<double> hr;
  double check_ms = 0.0;
  int next_check = sched.first();
  int m = 0;
  lyap_status status = LYAP_NOT_CONVERGED;
  double last_res = INFINITY;
  double lam_absmax = 0.0;
  int checked_m = 0;
  double t_to_tol = 0.0;
  int head = 0, npend = 0;  // checks in flight: slots head, head + 1, ... (mod nslots)
  int last_launched = 0;
  CheckSlot* done_slot = slots[0].get();  // the slot of the last check read

  auto launch_check = [&](CheckSlot& sl, int mm) {
    LYAP_HIP(hipEventRecord(ev_step, st));
    LYAP_HIP(hipStreamWaitEvent(sl.st, ev_step, 0));
    kt.mark(LYAP_K_CHECK);
    sl.ck->run(side.band(), mm * S, side.gamma_dev(), side.tau_dev(mm), sl.chk.as<CheckOut>());
    LYAP_HIP(hipMemcpyAsync(sl.hchk.p, sl.chk.p, sizeof(CheckOut), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipMemcpyAsync(sl.hflags.p, side.flags_dev(), 2 * sizeof(int), hipMemcpyDeviceToHost, sl.st));
    LYAP_HIP(hipEventRecord(sl.ev, sl.st));
    sl.mm = mm;
  };
  auto wait_check = [&](CheckSlot& sl) {
    const auto t0 = Clock::now();
    LYAP_HIP(hipEventSynchronize(sl.ev));
    check_ms += ms_since(t0);
    kt.collect();
  };
  // Reads the finished check; returns true when the iteration stops.
  auto finish_check = [&](CheckSlot& sl) -> bool {
    done_slot = &sl;
    out->n_checks++;
    const int mm = sl.mm;
    const CheckOut c = *sl.hchk.as<CheckOut>();
    const int fb = sl.hflags.as<int>()[0], fn = sl.hflags.as<int>()[1];
    // non-finite values that follow a breakdown belong to the breakdown
    LYAP_REQUIRE(!(fn > 0 && fn <= mm && (fb == 0 || fn <= fb)), LYAP_E_NUMERIC,
                 "non-finite values in the Lanczos recurrence at step %d", fn);
    if (fb > 0 && fb <= mm) {
      // a rank-deficient block at step fb-1: check the basis it ends instead
      LYAP_HIP(hipStreamSynchronize(st));
      launch_check(sl, fb);
      out->n_checks++;
      wait_check(sl);
      const CheckOut cb = *sl.hchk.as<CheckOut>();
      LYAP_REQUIRE(std::isfinite(cb.res), LYAP_E_NUMERIC, "residual is not finite at m=%d", fb);
      const double rel = cb.res / beta2;
      hm.push_back(fb);
      hr.push_back(rel);
      last_res = rel;
      checked_m = fb;
      lam_absmax = std::max(std::fabs(cb.lam_min), std::fabs(cb.lam_max));
      m = fb;
      if (rel <= o.tol) {
        status = LYAP_OK;
        t_to_tol = ms_since(t_entry);
      } else {
        status = LYAP_E_BREAKDOWN;
        set_error("block Lanczos breakdown at m=%d with residual %.3e above tol", fb, rel);
      }
      return true;
    }
    LYAP_REQUIRE(std::isfinite(c.res), LYAP_E_NUMERIC, "residual is not finite at m=%d", mm);
    const double rel = c.res / beta2;
    hm.push_back(mm);
    hr.push_back(rel);
    last_res = rel;
    checked_m = mm;
    lam_absmax = std::max(std::fabs(c.lam_min), std::fabs(c.lam_max));
    if (o.verbose) std::fprintf(stderr, "[lyap] m=%d k=%d res=%.3e\n", mm, mm * S, rel);
    LYAP_REQUIRE(c.lam_max < 0.0, LYAP_E_INDEFINITE,
                 "Ritz value %.3e >= 0 at m=%d: the operator is not negative definite", c.lam_max, mm);
    if (rel <= o.tol) {
      status = LYAP_OK;
      m = mm;
      t_to_tol = ms_since(t_entry);
      return true;
    }
    if (mm >= maxit) {
      m = mm;
      return true;
    }
    if (!fixed) next_check = sched.next(mm, rel, o.tol);
    return false;
  };

  const auto t_pass1 = Clock::now();
  int steps = 0;  // steps enqueued
  while (true) {
    if (npend > 0) {
      CheckSlot& sl = *slots[head];
      const hipError_t q = hipEventQuery(sl.ev);
      // wait when nothing else can proceed: the steps are done, or (fixed
      // schedule) every slot is busy and the steps are kAhead past the next
      // check point
      const bool stuck = steps >= maxit || (fixed && npend == nslots && steps >= next_check + kAhead);
      if (q == hipSuccess || stuck || !overlap) {
        if (q != hipSuccess) wait_check(sl);
        --npend;
        head = (head + 1) % nslots;
        if (finish_check(sl)) break;
        continue;
      } else if (q != hipErrorNotReady) {
        LYAP_HIP(q);
      }
    }
    if (npend < nslots && next_check > last_launched && (steps >= next_check || steps >= maxit)) {
      // always at the scheduled point (not at however far the steps have run
      // ahead), so that the result does not depend on timing
      const int mm = std::min(next_check, steps);
      launch_check(*slots[(head + npend) % nslots], mm);
      ++npend;
      last_launched = mm;
      if (fixed) next_check = std::min(mm + sched.d, maxit);
      continue;
    }
    if (steps >= maxit) continue;  // a check is pending
    if (fixed && steps >= next_check + kAhead) continue;  // waits for a slot
    if (steps >= kAhead) LYAP_HIP(hipEventSynchronize(er.ev[steps % kAhead]));
    side.step();
    LYAP_HIP(hipEventRecord(er.ev[steps % kAhead], st));
    ++steps;
  }
  // finalisation reads the results of the check that ended the iteration
  if (overlap) LYAP_HIP(hipStreamWaitEvent(st, done_slot->ev, 0));
  const double pass1_ms = ms_since(t_pass1) - check_ms;
  out->m = m;
  out->res = last_res;
  store_history(out, hm, hr);
  (void)checked_m;

  // ------------------------------------------------------------ finalisation
  const auto t_fin = Clock::now();
  std::vector<double> tau_h(S * S);
  LYAP_HIP(hipMemcpyAsync(tau_h.data(), side.tau_dev(m), S * S * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  double tau_f = 0.0;
  for (double v : tau_h) tau_f += v * v;
  tau_f = std::sqrt(tau_f);
  double eps = o.trunc_eps;
  if (!(eps >= 0.0)) eps = std::min(1e-12, 0.05 * o.tol / (lam_absmax + tau_f)) * beta2;
  out->trunc_eps = eps;
  DevBuf M;
  kt.mark(LYAP_K_FINAL);
  const int t = finalise_factor(*done_slot->ck, side.band(), side.gamma_dev(), eps, M, st);
  kt.collect();
  out->t = t;
  const double fin_ms = ms_since(t_fin);

  // ------------------------------------------------------------ Z (the side keeps
  // the steps it took; a breakdown check at mm < m uses the first mm blocks)
  const auto t_p2 = Clock::now();
  double zflush_bytes = 0.0;
  bool owned = false;
  out->Z = alloc_output(o, (size_t)n * std::max(t, 1) * sizeof(double), &owned);
  out->owns_Z = owned ? 1 : 0;
  side.accumulate_Z(m, M.as<double>(), t, out->Z, n, &zflush_bytes);
  LYAP_HIP(hipStreamSynchronize(st));
  kt.collect();
  const double p2_ms = ms_since(t_p2);

  if (o.want_T) {
    const int k = m * S;
    out->T_band = (double*)std::malloc((size_t)(S + 1) * k * sizeof(double));
    LYAP_HIP(hipMemcpy(out->T_band, side.band(), (size_t)(S + 1) * k * sizeof(double), hipMemcpyDeviceToHost));
    // entries below row k belong to tau_{m+1,m}; clear them
    for (int c = 0; c < k; ++c)
      for (int d = 0; d <= S; ++d)
        if (c + d >= k) out->T_band[(size_t)c * (S + 1) + d] = 0.0;
    out->gamma = (double*)std::malloc(S * S * sizeof(double));
    out->tau = (double*)std::malloc(S * S * sizeof(double));
    rowmajor_to_colmajor(side.gamma_host(), S, S, out->gamma);
    rowmajor_to_colmajor(tau_h.data(), S, S, out->tau);
  }
  out->times_ms[LYAP_T_PASS1] = pass1_ms;
  out->times_ms[LYAP_T_CHECKS] = check_ms;
  out->times_ms[LYAP_T_FINAL] = fin_ms;
  out->times_ms[LYAP_T_PASS2] = p2_ms;
  out->times_ms[LYAP_T_TOTAL] = ms_since(t_entry);
  out->times_ms[LYAP_T_TO_TOL] = t_to_tol;
  const double b = sizeof(T);
  const double coef = side.op().coef_bytes_per_row();
  // per step: 14 nsb with CGS2 (S <= 4), 21 nsb with block MGS twice
  out->bytes_pass1 = (int64_t)((double)m * n * ((S <= 4 ? 14.0 : 21.0) * S * b + coef));
  out->bytes_spmm = (int64_t)((double)m * n * (2.0 * S * b + coef));
  for (int i = 0; i < LYAP_K_COUNT; ++i) {
    out->kern_ms[i] = kt.ms[i];
    out->kern_n[i] = kt.n[i];
  }
  fill_kernel_bytes<T>(n, S, coef, kt, zflush_bytes, out->kern_bytes);
  out->status = status;
  return status;
}

template lyap_status solve_std<float>(const lyap_op*, const double*, int, int64_t, const lyap_opts&, lyap_result*);
template lyap_status solve_std<double>(const lyap_op*, const double*, int, int64_t, const lyap_opts&, lyap_result*);

// ------------------------------------------------------ rank-deficient start block
// Gram matrix C^T C of an n x S column-major block: FP64 partials per
// workgroup, summed in a fixed order by one workgroup.
template <int S>
__global__ __launch_bounds__(kBlock) void k_cols_gram(const double* __restrict__ C, int64_t ldc, int n,
                                                      double* __restrict__ part) {
  __shared__ double red[pow2_at_least(S * S) * (kBlock / 64)];
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    double c[S];
#pragma unroll
    for (int i = 0; i < S; ++i) c[i] = C[(size_t)i * ldc + r];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) acc[i * S + j] = fma(c[i], c[j], acc[i * S + j]);
  }
  write_partial<S * S, kBlock>(acc, red, part);
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_cols_gram_sum(const double* __restrict__ part, int nparts,
                                                          double* __restrict__ out) {
  __shared__ double red[pow2_at_least(S * S) * (kBlock / 64)];
  reduce_partials<S * S, kBlock>(part, nparts, red);
  if (threadIdx.x < S * S) out[threadIdx.x] = red[threadIdx.x];
}

// Ce = C W: n x s times s x r (W row-major), Ce column-major with leading dimension n.
__global__ __launch_bounds__(kBlock) void k_cols_mix(const double* __restrict__ C, int64_t ldc, int n, int s,
                                                     const double* __restrict__ W, int r, double* __restrict__ Ce) {
  for (int row = blockIdx.x * kBlock + threadIdx.x; row < n; row += gridDim.x * kBlock) {
    double c[8];
    for (int i = 0; i < s; ++i) c[i] = C[(size_t)i * ldc + row];
    for (int j = 0; j < r; ++j) {
      double acc = 0.0;
      for (int i = 0; i < s; ++i) acc = fma(c[i], W[i * r + j], acc);
      Ce[(size_t)j * n + row] = acc;
    }
  }
}

// Eigenvalues (descending) and eigenvectors (columns of V, row-major s x s) of
// a small symmetric matrix by cyclic Jacobi rotations (host, s <= 8).
static void sym_eig_jacobi(std::vector<double> G, int s, std::vector<double>& lam, std::vector<double>& V) {
  std::vector<double> U((size_t)s * s, 0.0);
  for (int i = 0; i < s; ++i) U[i * s + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        tot += G[i * s + j] * G[i * s + j];
        if (i != j) off += G[i * s + j] * G[i * s + j];
      }
    if (off <= 1e-36 * tot) break;
    for (int p = 0; p < s; ++p)
      for (int q = p + 1; q < s; ++q) {
        const double apq = G[p * s + q];
        if (apq == 0.0) continue;
        const double theta = (G[q * s + q] - G[p * s + p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < s; ++k) {  // G <- G J
          const double gp = G[k * s + p], gq = G[k * s + q];
          G[k * s + p] = c * gp - sn * gq;
          G[k * s + q] = sn * gp + c * gq;
        }
        for (int k = 0; k < s; ++k) {  // G <- J^T G
          const double gp = G[p * s + k], gq = G[q * s + k];
          G[p * s + k] = c * gp - sn * gq;
          G[q * s + k] = sn * gp + c * gq;
        }
        for (int k = 0; k < s; ++k) {  // U <- U J
          const double up = U[k * s + p], uq = U[k * s + q];
          U[k * s + p] = c * up - sn * uq;
          U[k * s + q] = sn * up + c * uq;
        }
      }
  }
  std::vector<int> ord(s);
  for (int i = 0; i < s; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return G[a * s + a] > G[b * s + b]; });
  lam.assign(s, 0.0);
  V.assign((size_t)s * s, 0.0);
  for (int j = 0; j < s; ++j) {
    lam[j] = G[ord[j] * s + ord[j]];
    for (int i = 0; i < s; ++i) V[i * s + j] = U[i * s + ord[j]];
  }
}

// Numerical rank of C: the eigenvalues of C^T C above 10 n eps lambda_max
// (eps = 2^-52).  The paper takes a full-rank start block and leaves
// deflation to the customary practice of block methods; for r < s the solve
// runs on Ce = C W_r (W_r the eigenvectors of the r largest eigenvalues), whose
// Ce Ce^T is C C^T without the dropped eigenvalues.  Returns r (Ce untouched
// when r = s); throws E_ARG for C = 0 and E_NUMERIC for NaN/Inf.
int deflate_start(const double* C, int n, int s, int64_t ldc, hipStream_t st, DevBuf& Ce) {
  const int grid = grid_for(n, 8, 1024);
  DevBuf part((size_t)grid * s * s * sizeof(double)), tot((size_t)s * s * sizeof(double));
  switch (s) {
#define LYAP_GRAM_CASE(SS)                                                                                      \
  case SS:                                                                                                      \
    hipLaunchKernelGGL((k_cols_gram<SS>), dim3(grid), dim3(kBlock), 0, st, C, ldc, n, part.as<double>());       \
    hipLaunchKernelGGL((k_cols_gram_sum<SS>), dim3(1), dim3(kBlock), 0, st, part.as<double>(), grid,            \
                       tot.as<double>());                                                                       \
    break;
    LYAP_GRAM_CASE(1)
    LYAP_GRAM_CASE(2)
    LYAP_GRAM_CASE(3)
    LYAP_GRAM_CASE(4)
    LYAP_GRAM_CASE(5)
    LYAP_GRAM_CASE(6)
    LYAP_GRAM_CASE(7)
    LYAP_GRAM_CASE(8)
#undef LYAP_GRAM_CASE
    default:
      LYAP_REQUIRE(false, LYAP_E_ARG, "s=%d out of range 1..8", s);
  }
  LYAP_LAUNCHED("k_cols_gram");
  std::vector<double> G((size_t)s * s);
  LYAP_HIP(hipMemcpyAsync(G.data(), tot.p, G.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  for (double g : G) LYAP_REQUIRE(std::isfinite(g), LYAP_E_NUMERIC, "C contains NaN or Inf");
  std::vector<double> lam, V;
  sym_eig_jacobi(G, s, lam, V);
  LYAP_REQUIRE(lam[0] > 0.0, LYAP_E_ARG, "C is zero");
  const double thr = 10.0 * n * std::numeric_limits<double>::epsilon() * lam[0];
  int r = 0;
  while (r < s && lam[r] > thr) ++r;
  if (r == s) return s;
  std::vector<double> Wr((size_t)s * r);
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < r; ++j) Wr[i * r + j] = V[i * s + j];
  DevBuf Wd(Wr.size() * sizeof(double));
  LYAP_HIP(hipMemcpyAsync(Wd.p, Wr.data(), Wr.size() * sizeof(double), hipMemcpyHostToDevice, st));
  Ce.alloc((size_t)n * r * sizeof(double));
  hipLaunchKernelGGL(k_cols_mix, dim3(grid_for(n, 1, 2048)), dim3(kBlock), 0, st, C, ldc, n, s, Wd.as<double>(), r,
                     Ce.as<double>());
  LYAP_LAUNCHED("k_cols_mix");
  LYAP_HIP(hipStreamSynchronize(st));  // Wd and the partials are released on return
  return r;
}

}  // namespace lyap

extern "C" lyap_status lyap_solve(const lyap_op* A, const double* C, int32_t s, int64_t ldc, const lyap_opts* opts,
                                  lyap_result* out) {
  clear_error();
  if (!out) {
    set_error("out is NULL");
    return LYAP_E_ARG;
  }
  std::memset(out, 0, sizeof(*out));
  lyap_opts o;
  if (opts) o = *opts;
  else lyap_opts_default(&o);
  try {
    validate_op(A);
    LYAP_REQUIRE(C != nullptr, LYAP_E_ARG, "C is NULL");
    LYAP_REQUIRE(s >= 1 && s <= 8, LYAP_E_ARG, "s=%d out of range 1..8", s);
    LYAP_REQUIRE(ldc >= A->n, LYAP_E_ARG, "ldc=%lld < n=%lld", (long long)ldc, (long long)A->n);
    LYAP_REQUIRE(s <= A->n, LYAP_E_ARG, "s > n");
    LYAP_REQUIRE(o.tol > 0.0 && o.tol < 1.0, LYAP_E_ARG, "tol=%g must be in (0,1)", o.tol);
    LYAP_REQUIRE(o.max_iter >= 1 && (int64_t)o.max_iter * s <= (int64_t)1 << 20, LYAP_E_ARG,
                 "max_iter=%d out of range", o.max_iter);
    LYAP_REQUIRE(o.check_every >= 0, LYAP_E_ARG, "check_every must be >= 0");
    LYAP_REQUIRE(o.storage == LYAP_STORE_F64 || o.storage == LYAP_STORE_F32, LYAP_E_ARG, "unknown storage %d",
                 o.storage);
    LYAP_REQUIRE(o.method == LYAP_METHOD_STD || o.method == LYAP_METHOD_EXT, LYAP_E_ARG, "unknown method %d",
                 o.method);
    // a rank-deficient C runs on its deflated columns (r of them)
    DevBuf Ce;
    const int r = deflate_start(C, (int)A->n, s, ldc, (hipStream_t)o.stream, Ce);
    if (r < s) {
      LYAP_REQUIRE(o.method == LYAP_METHOD_STD || r == 1 || r == 2 || r == 4, LYAP_E_UNSUPPORTED,
                   "C has numerical rank %d < s=%d; the extended Krylov kernels take blocks of 1, 2 or 4 columns",
                   r, s);
      C = Ce.as<double>();
      ldc = A->n;
      s = r;
    }
    if (o.method == LYAP_METHOD_STD) {
      lyap_status st = o.storage == LYAP_STORE_F64 ? solve_std<double>(A, C, s, ldc, o, out)
                                                   : solve_std<float>(A, C, s, ldc, o, out);
      out->status = st;
      return st;
    }
    if (o.method == LYAP_METHOD_EXT) {
      lyap_status st = o.storage == LYAP_STORE_F64 ? solve_ext<double>(A, C, s, ldc, o, out)
                                                   : solve_ext<float>(A, C, s, ldc, o, out);
      out->status = st;
      return st;
    }
    LYAP_REQUIRE(false, LYAP_E_ARG, "unknown method %d", o.method);
  } catch (const Error& e) {
    out->status = e.st;
    return e.st;
  }
  return LYAP_E_ARG;
}

extern "C" lyap_status lyap_ctri(const double* T_band, int32_t ell, int32_t k, const double* gamma,
                                 const double* tau, double* res, double* lam, void* stream) {
  clear_error();
  try {
    LYAP_REQUIRE(T_band && gamma && tau && res, LYAP_E_ARG, "NULL argument");
    LYAP_REQUIRE(ell >= 1 && ell <= 16 && k >= ell && k % ell == 0, LYAP_E_ARG, "bad ell=%d / k=%d", ell, k);
    hipStream_t st = (hipStream_t)stream;
    DevBuf band((size_t)(ell + 1) * k * sizeof(double));
    DevBuf g(ell * ell * sizeof(double)), t(ell * ell * sizeof(double));
    std::vector<double> grm(ell * ell), trm(ell * ell);
    for (int i = 0; i < ell; ++i)
      for (int j = 0; j < ell; ++j) {
        grm[i * ell + j] = gamma[i + j * ell];
        trm[i * ell + j] = tau[i + j * ell];
      }
    LYAP_HIP(hipMemcpyAsync(band.p, T_band, band.bytes, hipMemcpyHostToDevice, st));
    LYAP_HIP(hipMemcpyAsync(g.p, grm.data(), ell * ell * sizeof(double), hipMemcpyHostToDevice, st));
    LYAP_HIP(hipMemcpyAsync(t.p, trm.data(), ell * ell * sizeof(double), hipMemcpyHostToDevice, st));
    DevBuf chk(sizeof(CheckOut));
    Checker ck(ell, ell, st);
    ck.run(band.as<double>(), k, g.as<double>(), t.as<double>(), chk.as<CheckOut>());
    CheckOut h;
    LYAP_HIP(hipMemcpyAsync(&h, chk.p, sizeof(CheckOut), hipMemcpyDeviceToHost, st));
    if (lam) LYAP_HIP(hipMemcpyAsync(lam, ck.lam(), (size_t)k * sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipStreamSynchronize(st));
    *res = h.res;
    return LYAP_OK;
  } catch (const Error& e) {
    return e.st;
  }
}
