// Native host scheduler of the TSBTS integration: eras, passes and block steps
// (Algorithm 2), the time-symmetry criterion (Eq. blockcondition), the symmetrization
// rules (Algorithm 1) and the dynamic era size (Algorithm 3), driving the kernels of this
// library with one host/device synchronisation per block step (to read the criterion).
//
// Times are integers in ticks of 2^-20; every step is a power of two of ticks.  Block
// steps stay aligned (a step only doubles at a multiple of twice its size), so at any
// block time T all particles of one level dt sit at floor(T/dt)*dt: the next block time
// and the active set follow from per-level member lists in O(levels).
//
// Readings (shared with the reference scheduler used by the tests):
//   admissible(b, e): largest power of two <= (b + e)/2, within [dt_min, dt_max];
//   first pass: step <- min(step, admissible(b, b)), or twice the step at a multiple of
//     twice the step when that is admissible;
//   later passes: even time: double if admissible with the end value at t+2dt, else keep
//     if admissible with the end value at t+dt, else halve; odd time: keep or halve.  End
//     values come from the previous pass's criterion values of the particle, linear in
//     time between stored values, the start value past the last one;
//   dynamic era: size = (last - first next block time) clamped to [dt_max/8, dt_max],
//     rounded up to a power of two, dt_max when that is below the largest step in use
//     (an era shorter than a step leaves the particle unsymmetrized); the era ends at
//     the next multiple of the size;
//   era start: from the second pass on, the step of every particle at the era start is
//     chosen again by the later-pass rule (from the step that brought it there) with the
//     previous pass's end values, so the first step of an era is symmetrized too.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "predict.hpp"
#include "rule_pool.hpp"

namespace tsbts {

constexpr int kTickBits = 20;
constexpr double kTick = 1.0 / (1 << kTickBits);
constexpr int kMaxLevel = 40;

int64_t admissible_ticks(double begin, double end, int64_t dt_min, int64_t dt_max) {
  const double avg = 0.5 * (begin + end);
  const double x = avg / kTick;
  if (!std::isfinite(x) || x >= static_cast<double>(dt_max)) return dt_max;
  if (x < 1.0) return dt_min;
  int e = 0;
  std::frexp(x, &e);  // x = f * 2^e, f in [0.5, 1)
  const int64_t p2 = int64_t(1) << (e - 1);
  return std::min(dt_max, std::max(dt_min, p2));
}

int64_t era_end_rule(int64_t t0, int64_t first, int64_t last, int64_t largest,
                     int64_t dt_max, int64_t era) {
  if (era > 0) return t0 + era;
  // Algorithm 3: last minus first next block time, clamped to [dt_max/8, dt_max]
  const int64_t size = std::min(dt_max, std::max(dt_max / 8, last - first));
  int64_t p2 = 1;
  while (p2 < size) p2 *= 2;  // smallest power of two >= size
  if (p2 < largest) p2 = dt_max;  // shorter than a step in use: no past to symmetrize it
  return (t0 / p2 + 1) * p2;
}

// step_rule with the previous pass's values at the ends of the two candidate steps given
// on demand by end_dt() and end_2dt(): each is needed on some branches only.
// Whether tb is a multiple of 2 dt, and whether tb / dt (rounded down) is even, for
// tb >= 0: bit tests when dt is a power of two (every step of the scheduler), the
// divisions otherwise.
inline bool multiple_of_2dt(int64_t tb, int64_t dt) {
  if (dt > 0 && (dt & (dt - 1)) == 0 && tb >= 0) return (tb & (2 * dt - 1)) == 0;
  return tb % (2 * dt) == 0;
}
inline bool even_multiple(int64_t tb, int64_t dt) {
  if (dt > 0 && (dt & (dt - 1)) == 0 && tb >= 0) return (tb & dt) == 0;
  return (tb / dt) % 2 == 0;
}

template <class E1, class E2>
int64_t step_rule_lazy(int first_pass, int64_t dt, int64_t tb, double begin, E1 end_dt,
                       E2 end_2dt, int64_t dt_min, int64_t dt_max) {
  if (first_pass) {
    const int64_t lvl = admissible_ticks(begin, begin, dt_min, dt_max);
    if (lvl >= 2 * dt && multiple_of_2dt(tb, dt)) return 2 * dt;
    return std::min(dt, lvl);
  }
  const bool even = even_multiple(tb, dt);
  if (even && 2 * dt <= dt_max && 2 * dt <= admissible_ticks(begin, end_2dt(), dt_min, dt_max))
    return 2 * dt;
  if (dt <= admissible_ticks(begin, end_dt(), dt_min, dt_max)) return dt;
  return std::max(dt / 2, dt_min);
}

int64_t step_rule(int first_pass, int64_t dt, int64_t tb, double begin, double end_dt,
                  double end_2dt, int64_t dt_min, int64_t dt_max) {
  return step_rule_lazy(
      first_pass, dt, tb, begin, [&] { return end_dt; }, [&] { return end_2dt; }, dt_min,
      dt_max);
}

namespace {

// Smallest l with 2^l >= dt (0 for dt <= 1).
int level_of(int64_t dt) {
  if (dt <= 1) return 0;
  return 64 - __builtin_clzll(static_cast<uint64_t>(dt - 1));
}

// Criterion values of one pass grouped by particle (time order kept).
struct CritHistory {
  std::vector<int32_t> pid;
  std::vector<int64_t> t;
  std::vector<double> c;
  std::vector<int64_t> off;  // n + 1 after close()
  std::vector<int64_t> gt;
  std::vector<double> gc;
  std::vector<int64_t> cur;  // per particle: the record value_at found last

  void clear() {
    pid.clear();
    t.clear();
    c.clear();
  }
  void add(int32_t p, int64_t tt, double cc) {
    pid.push_back(p);
    t.push_back(tt);
    c.push_back(cc);
  }
  // make room for k more records (filled with set); returns the first one's index
  size_t extend(size_t k) {
    const size_t base = pid.size();
    pid.resize(base + k);
    t.resize(base + k);
    c.resize(base + k);
    return base;
  }
  void set(size_t r, int32_t p, int64_t tt, double cc) {
    pid[r] = p;
    t[r] = tt;
    c[r] = cc;
  }
  void close(int64_t n) {
    off.assign(n + 1, 0);
    for (int32_t p : pid) ++off[p + 1];
    for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    gt.resize(pid.size());
    gc.resize(pid.size());
    for (size_t r = 0; r < pid.size(); ++r) {
      const int64_t d = fill[pid[r]]++;
      gt[d] = t[r];
      gc[d] = c[r];
    }
    cur.assign(off.begin(), off.end() - 1);
  }
  // value of particle i at time tt, linear between stored values, fallback past the last
  double value_at(int32_t i, int64_t tt, double fallback) {
    const int64_t lo = off[i], hi = off[i + 1];
    // last record with time <= tt, else the first (at or before the era start): found
    // from the particle's cursor, which a pass's queries move by a few records at most
    int64_t k = cur[i];
    while (k > lo && gt[k] > tt) --k;
    while (k + 1 < hi && gt[k + 1] <= tt) ++k;
    cur[i] = k;
    if (gt[k] == tt) return gc[k];
    if (k + 1 >= hi) return fallback;
    const double w = static_cast<double>(tt - gt[k]) / static_cast<double>(gt[k + 1] - gt[k]);
    return (1.0 - w) * gc[k] + w * gc[k + 1];
  }
  // fetch the records value_at(i, ...) starts from into the cache
  void prefetch(int32_t i) const {
    if (static_cast<size_t>(i) >= cur.size()) return;
    const size_t k = static_cast<size_t>(cur[i]);
    if (k >= gt.size()) return;
    __builtin_prefetch(&gt[k]);
    __builtin_prefetch(&gc[k]);
  }
};

}  // namespace

struct Scheduler {
  int64_t n = 0;
  double eta = 0.1;
  int passes = 3;
  int64_t dt_min = 1, dt_max = 1 << 14, era = 0;
  std::vector<int64_t> t, dt;
  std::vector<int64_t> dtp;  // the step that brought each particle to t (0: none yet)
  std::vector<double> dtc;
  int64_t time = 0;
  // level member lists
  std::vector<int32_t> mem[kMaxLevel + 1];
  std::vector<int32_t> lvl, pos;
  std::vector<uint64_t> list_bits;  // one bit per particle, zero between block steps
  // the step rule of long lists on several host threads (rule_threads; 1: this one only)
  int rule_threads = 4;
  std::unique_ptr<RulePool> pool;
  // per part of the list: the positions whose particle changes level, in list order
  std::vector<int32_t> moved[16];
  // criterion histories
  CritHistory prev, cur;
  bool have_prev = false;
  // staging
  // pinned host buffers; the criterion and the step updates cross the link without a
  // copy: the kernels write dtc_h and read dtn_h through their device mappings
  int32_t *idx_h = nullptr;
  double *dtc_h = nullptr, *dtn_h = nullptr;
  double *dtc_hd = nullptr, *dtn_hd = nullptr;  // device views of dtc_h, dtn_h
  int32_t *idx_d = nullptr;
  double *acc_d = nullptr;
  double *s0 = nullptr;  // era-start device copy: r, v, a (3n each), t_last, dt
  std::vector<int64_t> s0_t, s0_dt, s0_dtp;
  std::vector<double> s0_dtc;
  int64_t stats[4] = {0, 0, 0, 0};  // block steps, force calls, interactions, eras
  // wall-clock breakdown of the block steps by active-set class (tsbts_sched_timing)
  double phase_s[4][4] = {};
  int64_t phase_n[4][2] = {};
  int crit_before = 0;  // criterion with the predicted velocities, fused with the force
  int pred_on_load = 1;  // small active sets: prediction (and on few particles the
                         // criterion) folded into the force kernel
  // The new steps chosen after a block step are not scattered by a launch of their own:
  // the corrector tags each target with (step id, list position), and the next block
  // step's first kernel takes the pending steps from dtn_h through those tags.  At the
  // end of a pass the last step's are stored by tsbts_set_dt.
  int64_t *tag_d = nullptr;  // [n] device
  int64_t step_id = 0;       // block steps issued so far (tags are unique per step)
  bool pending = false;      // dtn_h holds new steps of step `pending_step` not yet stored
  int64_t pending_step = 0;
  int32_t pending_k = 0;     // its active-set size (its list is still in idx_d)
  // the same steps as exponents, dt = 2^exp, passed by value when at most kInlinePend
  int8_t pend_exp[tsbts::kInlinePend];

  void rebuild_levels() {
    for (auto &m : mem) m.clear();
    for (int64_t i = 0; i < n; ++i) {
      const int l = level_of(dt[i]);
      lvl[i] = l;
      pos[i] = static_cast<int32_t>(mem[l].size());
      mem[l].push_back(static_cast<int32_t>(i));
    }
  }
  // Put the active list idx_h[0 .. k) in particle order (through a bitmap: k bit sets and
  // a scan of n/64 words), so that the step rule reads the particles' host state in
  // address order.
  void sort_list(int32_t k) {
    uint64_t *w = list_bits.data();
    for (int32_t q = 0; q < k; ++q)
      w[idx_h[q] >> 6] |= uint64_t(1) << (idx_h[q] & 63);
    int32_t q = 0;
    for (size_t b = 0; b < list_bits.size(); ++b) {
      uint64_t x = w[b];
      if (!x) continue;
      w[b] = 0;
      while (x) {
        idx_h[q++] = static_cast<int32_t>(b * 64 + __builtin_ctzll(x));
        x &= x - 1;
      }
    }
  }
  // fetch particle i's host state (scattered over n when the active list comes in
  // level-list order) into the cache, with the start of its criterion history
  void prefetch(int32_t i) const {
    __builtin_prefetch(&t[i]);
    __builtin_prefetch(&dt[i]);
    __builtin_prefetch(&dtp[i]);
    __builtin_prefetch(&dtc[i]);
    __builtin_prefetch(&lvl[i]);
    if (static_cast<size_t>(i) < prev.cur.size()) {
      __builtin_prefetch(&prev.off[i]);
      __builtin_prefetch(&prev.cur[i]);
    }
  }
  void move(int32_t i, int l) {
    const int o = lvl[i];
    if (o == l) return;
    auto &src = mem[o];
    const int32_t last = src.back();
    src[pos[i]] = last;
    pos[last] = pos[i];
    src.pop_back();
    lvl[i] = l;
    pos[i] = static_cast<int32_t>(mem[l].size());
    mem[l].push_back(i);
  }
  // next block time over occupied levels (members of a level share their time)
  int64_t next_time() const {
    int64_t best = INT64_MAX;
    for (int l = 0; l <= kMaxLevel; ++l)
      if (!mem[l].empty()) best = std::min(best, t[mem[l][0]] + (int64_t(1) << l));
    return best;
  }
  int64_t era_end(int64_t t0) const {
    if (era > 0) return t0 + era;
    int64_t lo = INT64_MAX, hi = INT64_MIN, largest = 0;
    for (int l = 0; l <= kMaxLevel; ++l) {
      if (mem[l].empty()) continue;
      const int64_t nx = t[mem[l][0]] + (int64_t(1) << l);
      lo = std::min(lo, nx);
      hi = std::max(hi, nx);
      largest = int64_t(1) << l;
    }
    return era_end_rule(t0, lo, hi, largest, dt_max, era);
  }
};

}  // namespace tsbts

using tsbts::Scheduler;

namespace {

int sfail(tsbts_ctx *c, int st, const char *msg) {
  snprintf(c->err, sizeof(c->err), "%s", msg);
  return st;
}

#define SCHED_HIP(expr)                                                        \
  do {                                                                         \
    hipError_t _e = (expr);                                                    \
    if (_e != hipSuccess) {                                                    \
      snprintf(c->err, sizeof(c->err), "%s: %s", #expr, hipGetErrorString(_e)); \
      return TSBTS_EHIP;                                                       \
    }                                                                          \
  } while (0)

#define SCHED_CALL(expr)        \
  do {                          \
    int _s = (expr);            \
    if (_s != TSBTS_OK) return _s; \
  } while (0)

// Wait for the criterion values of a block step, dtc_h[0 .. k), which the step's last
// kernel writes through the coherent mapping of dtc_h (set to kUnsetBits before the
// launches; no arithmetic gives that NaN payload): the host spins on the values rather
// than waiting for the stream's completion signal.  The step's other results are read
// only by later launches on the stream, which follow it anyway.  Every 20 us of spinning
// it asks for the stream's status, so a failed or lost launch ends the wait with an error.
constexpr uint64_t kUnsetBits = 0x7ff4deadbeef0001ull;

int wait_criterion(tsbts_ctx *c, Scheduler &S, int32_t k, hipStream_t st) {
  using clk = std::chrono::steady_clock;
  const auto *bits = reinterpret_cast<const uint64_t *>(S.dtc_h);
  auto t0 = clk::now();
  uint32_t spins = 0;
  for (int32_t q = 0; q < k;) {
    if (__atomic_load_n(bits + q, __ATOMIC_ACQUIRE) != kUnsetBits) {
      ++q;
      continue;
    }
    if ((++spins & 255) != 0 || clk::now() - t0 < std::chrono::microseconds(20)) continue;
    const hipError_t e = hipStreamQuery(st);
    if (e == hipErrorNotReady) {
      t0 = clk::now();
      continue;
    }
    SCHED_HIP(e);
    // the stream is idle: every value of the step is in place
    for (; q < k; ++q)
      if (__atomic_load_n(bits + q, __ATOMIC_ACQUIRE) == kUnsetBits) {
        snprintf(c->err, sizeof(c->err), "block step ended without criterion value %d", q);
        return TSBTS_EHIP;
      }
  }
  return TSBTS_OK;
}

// Store the new steps of the last block step, if the next block step has not (its list
// is still in idx_d).
int flush_steps(tsbts_ctx *c, Scheduler &S, hipStream_t st) {
  if (!S.pending) return TSBTS_OK;
  S.pending = false;
  return tsbts_set_dt(c, S.idx_d, S.pending_k, S.dtn_hd, st);
}

// One pass of an era: block steps until the next block time passes T1.
// Active lists longer than this are put in particle order (Scheduler::sort_list).
constexpr int32_t kSortList = 1024;
// Active lists of at least this many particles share the step rule among host threads.
constexpr int32_t kParallelRule = 8192;

int run_pass(tsbts_ctx *c, Scheduler &S, int p, int64_t T1, hipStream_t st) {
  const int64_t n = S.n;
  S.cur.clear();
  for (int64_t i = 0; i < n; ++i) S.cur.add(static_cast<int32_t>(i), S.t[i], S.dtc[i]);
  SCHED_CALL(tsbts_history_begin(c, st));
  using clk = std::chrono::steady_clock;
  auto t_prev = clk::now();
  for (;;) {
    const auto t_top = clk::now();
    const int64_t tb = S.next_time();
    if (tb > T1) break;
    // active set: all members of the levels whose next time is tb
    int32_t k = 0;
    for (int l = 0; l <= tsbts::kMaxLevel; ++l) {
      if (S.mem[l].empty() || S.t[S.mem[l][0]] + (int64_t(1) << l) != tb) continue;
      std::copy(S.mem[l].begin(), S.mem[l].end(), S.idx_h + k);
      k += static_cast<int32_t>(S.mem[l].size());
    }
    if (k > kSortList) S.sort_list(k);
    const double tbs = static_cast<double>(tb) * tsbts::kTick;
    const int64_t step = ++S.step_id;
    std::fill(reinterpret_cast<uint64_t *>(S.dtc_h), reinterpret_cast<uint64_t *>(S.dtc_h) + k,
              kUnsetBits);
    // small lists travel by value in the first kernel's arguments (it writes idx_d)
    tsbts::InlineIdx in;
    in.out = S.idx_d;
    in.k = 0;
    if (k <= tsbts::kInlineIdx && !c->check_idx) {
      in.k = k;
      std::copy(S.idx_h, S.idx_h + k, in.v);
    } else {
      SCHED_HIP(hipMemcpyAsync(S.idx_d, S.idx_h, sizeof(int32_t) * k, hipMemcpyHostToDevice,
                               st));
    }
    const tsbts::PendingSteps pend{S.tag_d, S.dtn_hd, S.pending_step,
                                   S.pending_k <= tsbts::kInlinePend ? S.pend_exp : nullptr,
                                   S.pending_k};
    const tsbts::PendingSteps *pp = S.pending ? &pend : nullptr;
    const tsbts::InlineIdx *ip = in.k ? &in : nullptr;
    const tsbts::StepTags tags{S.tag_d, step};
    if (S.pred_on_load && !S.crit_before && k <= tsbts::small_act_limit(c)) {
      int crit_done = 0;
      SCHED_CALL(tsbts::force_correct_predicted(c, S.idx_d, k, tbs, p > 0 ? 1 : 0, S.acc_d,
                                                st, &tags, pp, ip, S.eta, S.dtc_hd,
                                                &crit_done));
      if (!crit_done) SCHED_CALL(tsbts_timestep(c, S.idx_d, k, S.eta, S.dtc_hd, st));
    } else if (S.crit_before) {
      SCHED_CALL(tsbts::predict_pending(c, tbs, p > 0 ? 1 : 0, pp, ip, st));
      SCHED_CALL(tsbts::force_criterion_correct(c, S.idx_d, k, tbs, S.eta, S.acc_d, S.dtc_hd,
                                                st, &tags));
    } else {
      SCHED_CALL(tsbts::predict_pending(c, tbs, p > 0 ? 1 : 0, pp, ip, st));
      SCHED_CALL(tsbts::force_correct(c, S.idx_d, k, tbs, S.acc_d, st, &tags));
      SCHED_CALL(tsbts_timestep(c, S.idx_d, k, S.eta, S.dtc_hd, st));
    }
    const auto t_issued = clk::now();
    SCHED_CALL(wait_criterion(c, S, k, st));
    const auto t_done = clk::now();
    // Step rule of every listed particle: its own state only (its cursor into the previous
    // pass's criterion history included), so that parts of a long list can go to other
    // host threads; the level lists change afterwards, in list order.  The state of the
    // particles a few places ahead is fetched while one is handled (random accesses over
    // n otherwise take most of the loop's time at large n).
    const size_t rec0 = S.cur.extend(static_cast<size_t>(k));
    auto rule = [&](int32_t q0, int32_t q1, std::vector<int32_t> &moved) {
      constexpr int32_t kAhead = 16;
      moved.clear();
      for (int32_t q = q0; q < q1; ++q) {
        if (q + kAhead < q1) S.prefetch(S.idx_h[q + kAhead]);
        if (q + kAhead / 2 < q1) S.prev.prefetch(S.idx_h[q + kAhead / 2]);
        const int32_t i = S.idx_h[q];
        const double b = S.dtc_h[q];
        S.dtc[i] = b;
        S.dtp[i] = tb - S.t[i];
        S.t[i] = tb;
        S.cur.set(rec0 + q, i, tb, b);
        const int64_t d = S.dt[i];
        const int64_t nd = tsbts::step_rule_lazy(
            p == 0, d, tb, b, [&] { return S.prev.value_at(i, tb + d, b); },
            [&] { return S.prev.value_at(i, tb + 2 * d, b); }, S.dt_min, S.dt_max);
        S.dtn_h[q] = static_cast<double>(nd) * tsbts::kTick;
        if (q < tsbts::kInlinePend)
          S.pend_exp[q] = static_cast<int8_t>(tsbts::level_of(nd) - tsbts::kTickBits);
        if (nd != d) {
          S.dt[i] = nd;
          moved.push_back(q);
        }
      }
    };
    if (k >= kParallelRule && S.rule_threads > 1) {
      if (!S.pool || S.pool->parts() != S.rule_threads) {
        S.pool.reset();
        try {
          S.pool.reset(new tsbts::RulePool(S.rule_threads));
        } catch (...) {  // no threads: this one does it all
          S.pool.reset();
          S.rule_threads = 1;
        }
      }
    }
    int parts = 1;
    if (k >= kParallelRule && S.pool) {
      parts = S.pool->parts();
      const std::function<void(int, int)> part = [&](int w, int np) {
        rule(static_cast<int32_t>(int64_t(k) * w / np),
             static_cast<int32_t>(int64_t(k) * (w + 1) / np), S.moved[w]);
      };
      S.pool->run(part);
    } else {
      rule(0, k, S.moved[0]);
    }
    // level changes in list order (the parts are consecutive ranges of the list)
    for (int w = 0; w < parts; ++w)
      for (const int32_t q : S.moved[w]) {
        const int32_t i = S.idx_h[q];
        S.move(i, tsbts::level_of(S.dt[i]));  // steps are 2^l ticks throughout
      }
    // the next block step's first kernel stores these steps; dtn_h is rewritten only
    // after the next synchronisation, when that kernel has run
    S.pending = true;
    S.pending_step = step;
    S.pending_k = k;
    S.stats[0] += 1;
    S.stats[1] += 1;
    S.stats[2] += static_cast<int64_t>(k) * n;
    const auto t_end = clk::now();
    const int cls = k <= 32 ? 0 : k <= 256 ? 1 : k <= 1024 ? 2 : 3;
    auto sec = [](clk::duration d) { return std::chrono::duration<double>(d).count(); };
    S.phase_s[cls][0] += sec(t_issued - t_top);
    S.phase_s[cls][1] += sec(t_done - t_issued);
    S.phase_s[cls][2] += sec(t_end - t_done);
    S.phase_s[cls][3] += sec(t_end - t_prev);
    S.phase_n[cls][0] += 1;
    S.phase_n[cls][1] += k;
    t_prev = t_end;
  }
  SCHED_CALL(flush_steps(c, S, st));
  SCHED_CALL(tsbts_history_end(c, st));
  S.cur.close(n);
  std::swap(S.prev, S.cur);
  S.have_prev = true;
  return TSBTS_OK;
}

// Later passes: the steps of the particles at the era start T0 chosen again from the
// steps that brought them there, with the previous pass's end values; the device copy
// of the steps follows.
int first_steps(tsbts_ctx *c, Scheduler &S, int64_t T0, hipStream_t st) {
  const int64_t n = S.n;
  // the last step update of the previous pass may still be reading dtn_h
  SCHED_HIP(hipStreamSynchronize(st));
  for (int64_t i = 0; i < n; ++i) {
    if (S.t[i] == T0 && S.dtp[i] > 0) {
      const int64_t d = S.dtp[i];
      const double b = S.dtc[i];
      const int32_t ii = static_cast<int32_t>(i);
      S.dt[i] = tsbts::step_rule_lazy(
          0, d, T0, b, [&] { return S.prev.value_at(ii, T0 + d, b); },
          [&] { return S.prev.value_at(ii, T0 + 2 * d, b); }, S.dt_min, S.dt_max);
    }
    S.dtn_h[i] = static_cast<double>(S.dt[i]) * tsbts::kTick;
  }
  SCHED_HIP(hipMemcpyAsync(c->dt, S.dtn_h, sizeof(double) * n, hipMemcpyHostToDevice, st));
  // dtn_h is rewritten by the next block step on the host: wait for the copy
  SCHED_HIP(hipStreamSynchronize(st));
  return TSBTS_OK;
}

void free_sched(Scheduler *S) {
  if (!S) return;
  if (S->idx_h) (void)hipHostFree(S->idx_h);
  if (S->dtc_h) (void)hipHostFree(S->dtc_h);
  if (S->dtn_h) (void)hipHostFree(S->dtn_h);
  if (S->idx_d) (void)hipFree(S->idx_d);
  if (S->acc_d) (void)hipFree(S->acc_d);
  if (S->s0) (void)hipFree(S->s0);
  if (S->tag_d) (void)hipFree(S->tag_d);
  delete S;
}

}  // namespace

namespace tsbts {
void destroy_scheduler(tsbts_ctx *c) {
  free_sched(static_cast<Scheduler *>(c->sched));
  c->sched = nullptr;
}

namespace {

// No C++ exception crosses the C interface: a host allocation that fails (the scheduler's
// vectors) or a host thread that cannot be started becomes a status and a message.
template <class F>
int guarded(tsbts_ctx *c, const char *what, F &&f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    snprintf(c->err, sizeof(c->err), "%s: host memory allocation failed", what);
    return TSBTS_ENOMEM;
  } catch (const std::exception &e) {
    snprintf(c->err, sizeof(c->err), "%s: %s", what, e.what());
    return TSBTS_ESTATE;
  } catch (...) {
    snprintf(c->err, sizeof(c->err), "%s: unexpected host failure", what);
    return TSBTS_ESTATE;
  }
}

}  // namespace
}  // namespace tsbts

extern "C" {

int tsbts_sched_admissible(double begin, double end, int64_t dt_min, int64_t dt_max,
                           int64_t *out) {
  if (!out || dt_min < 1 || dt_max < dt_min) return TSBTS_EINVAL;
  *out = tsbts::admissible_ticks(begin, end, dt_min, dt_max);
  return TSBTS_OK;
}

int tsbts_sched_rule(int first_pass, int64_t dt, int64_t t_block, double begin, double end_dt,
                     double end_2dt, int64_t dt_min, int64_t dt_max, int64_t *out) {
  if (!out || dt < 1 || dt_min < 1 || dt_max < dt_min || t_block % dt != 0) return TSBTS_EINVAL;
  *out = tsbts::step_rule(first_pass, dt, t_block, begin, end_dt, end_2dt, dt_min, dt_max);
  return TSBTS_OK;
}

int tsbts_sched_era_end(int64_t t0, const int64_t *t_ticks, const int64_t *dt_ticks, int64_t n,
                        int64_t dt_max, int64_t era, int64_t *out) {
  if (!t_ticks || !dt_ticks || !out || n < 1 || t0 < 0 || era < 0 || dt_max < 1 ||
      (dt_max & (dt_max - 1)) || dt_max > (int64_t(1) << tsbts::kMaxLevel))
    return TSBTS_EINVAL;
  if (era > 0 && era % dt_max != 0) return TSBTS_EINVAL;
  int64_t lo = INT64_MAX, hi = INT64_MIN, largest = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t d = dt_ticks[i], ti = t_ticks[i];
    if (d < 1 || (d & (d - 1)) || d > dt_max || ti < 0 || ti > t0 || ti % d != 0 ||
        ti + d <= t0)
      return TSBTS_EINVAL;  // not an era-start state
    lo = std::min(lo, ti + d);
    hi = std::max(hi, ti + d);
    largest = std::max(largest, d);
  }
  *out = tsbts::era_end_rule(t0, lo, hi, largest, dt_max, era);
  return TSBTS_OK;
}

static int sched_init(tsbts_ctx *c, double eta, int passes, double dt_min, double dt_max,
                      double era, hipStream_t st) {
  if (!c) return TSBTS_EINVAL;
  if (!c->r || !c->v || !c->a || !c->m || !c->t_last || !c->dt)
    return sfail(c, TSBTS_ESTATE, "tsbts_sched_init: no particle state bound");
  const double k_min = dt_min / tsbts::kTick, k_max = dt_max / tsbts::kTick;
  if (!(eta > 0.0) || passes < 1 || k_min < 1.0 || k_max < k_min || k_min != std::floor(k_min) ||
      k_max != std::floor(k_max) || k_max > double(int64_t(1) << tsbts::kMaxLevel))
    return sfail(c, TSBTS_EINVAL, "tsbts_sched_init: invalid eta, passes or step bounds");
  const int64_t imin = static_cast<int64_t>(k_min), imax = static_cast<int64_t>(k_max);
  if ((imin & (imin - 1)) || (imax & (imax - 1)))
    return sfail(c, TSBTS_EINVAL, "tsbts_sched_init: step bounds must be powers of two");
  const double k_era = era / tsbts::kTick;
  if (era > 0.0 && (k_era != std::floor(k_era) || static_cast<int64_t>(k_era) % imax != 0))
    return sfail(c, TSBTS_EINVAL, "tsbts_sched_init: a fixed era must be a multiple of dt_max");
  tsbts::destroy_scheduler(c);
  Scheduler *S = new (std::nothrow) Scheduler();
  if (!S) return TSBTS_ENOMEM;
  c->sched = S;
  const int64_t n = c->n;
  S->n = n;
  S->eta = eta;
  S->passes = passes;
  S->dt_min = imin;
  S->dt_max = imax;
  S->era = era > 0.0 ? static_cast<int64_t>(k_era) : 0;
  S->t.assign(n, 0);
  S->dt.assign(n, 0);
  S->dtp.assign(n, 0);
  S->dtc.assign(n, 0.0);
  S->lvl.assign(n, 0);
  S->pos.assign(n, 0);
  S->list_bits.assign((n + 63) / 64, 0);
  SCHED_HIP(hipHostMalloc(reinterpret_cast<void **>(&S->idx_h), sizeof(int32_t) * n));
  // coherent: the kernels' criterion values reach host memory as they are written
  SCHED_HIP(hipHostMalloc(reinterpret_cast<void **>(&S->dtc_h), sizeof(double) * n,
                          hipHostMallocMapped | hipHostMallocCoherent));
  SCHED_HIP(hipHostMalloc(reinterpret_cast<void **>(&S->dtn_h), sizeof(double) * n));
  SCHED_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&S->dtc_hd), S->dtc_h, 0));
  SCHED_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&S->dtn_hd), S->dtn_h, 0));
  SCHED_HIP(hipMalloc(reinterpret_cast<void **>(&S->idx_d), sizeof(int32_t) * n));
  SCHED_HIP(hipMalloc(reinterpret_cast<void **>(&S->acc_d), sizeof(double) * 3 * n));
  SCHED_HIP(hipMalloc(reinterpret_cast<void **>(&S->s0), sizeof(double) * 11 * n));
  SCHED_HIP(hipMalloc(reinterpret_cast<void **>(&S->tag_d), sizeof(int64_t) * n));
  SCHED_HIP(hipMemsetAsync(S->tag_d, 0xff, sizeof(int64_t) * n, st));  // -1: no step
  // Algorithm 2, step 1: forces, criterion and block steps of all particles at t = 0
  for (int64_t i = 0; i < n; ++i) S->idx_h[i] = static_cast<int32_t>(i);
  SCHED_HIP(hipMemcpyAsync(S->idx_d, S->idx_h, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  SCHED_HIP(tsbts::launch_fill(c->t_last, n, 0.0, st));
  SCHED_HIP(tsbts::launch_fill(c->a, 3 * n, 0.0, st));
  SCHED_HIP(tsbts::launch_fill(c->dt, n, 0.0, st));
  SCHED_CALL(tsbts_predict(c, 0.0, 0, st));
  SCHED_CALL(tsbts_force(c, S->idx_d, static_cast<int32_t>(n), 0.0, c->a, nullptr, st));
  // the force output has the same [3][n] layout as the bound accelerations
  SCHED_CALL(tsbts_timestep(c, S->idx_d, static_cast<int32_t>(n), eta, S->dtc_hd, st));
  SCHED_HIP(hipStreamSynchronize(st));
  for (int64_t i = 0; i < n; ++i) {
    S->dtc[i] = S->dtc_h[i];
    S->dt[i] = tsbts::admissible_ticks(S->dtc[i], S->dtc[i], imin, imax);
    S->dtn_h[i] = static_cast<double>(S->dt[i]) * tsbts::kTick;
  }
  SCHED_HIP(hipMemcpyAsync(c->dt, S->dtn_h, sizeof(double) * n, hipMemcpyHostToDevice, st));
  SCHED_HIP(hipStreamSynchronize(st));
  S->rebuild_levels();
  return TSBTS_OK;
}

static int sched_era(tsbts_ctx *c, double *era_end, hipStream_t st) {
  if (!c) return TSBTS_EINVAL;
  Scheduler *S = static_cast<Scheduler *>(c->sched);
  if (!S) return sfail(c, TSBTS_ESTATE, "tsbts_sched_era: call tsbts_sched_init first");
  const int64_t n = S->n;
  const int64_t T0 = S->time;
  const int64_t T1 = S->era_end(T0);
  // era-start state: device copy and host mirrors
  double *s0 = S->s0;
  SCHED_HIP(hipMemcpyAsync(s0, c->r, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
  SCHED_HIP(hipMemcpyAsync(s0 + 3 * n, c->v, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
  SCHED_HIP(hipMemcpyAsync(s0 + 6 * n, c->a, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
  SCHED_HIP(hipMemcpyAsync(s0 + 9 * n, c->t_last, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  SCHED_HIP(hipMemcpyAsync(s0 + 10 * n, c->dt, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  S->s0_t = S->t;
  S->s0_dt = S->dt;
  S->s0_dtp = S->dtp;
  S->s0_dtc = S->dtc;
  S->have_prev = false;
  for (int p = 0; p < S->passes; ++p) {
    if (p > 0) {
      SCHED_HIP(hipMemcpyAsync(c->r, s0, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
      SCHED_HIP(hipMemcpyAsync(c->v, s0 + 3 * n, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
      SCHED_HIP(hipMemcpyAsync(c->a, s0 + 6 * n, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
      SCHED_HIP(hipMemcpyAsync(c->t_last, s0 + 9 * n, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      SCHED_HIP(hipMemcpyAsync(c->dt, s0 + 10 * n, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      S->t = S->s0_t;
      S->dt = S->s0_dt;
      S->dtp = S->s0_dtp;
      S->dtc = S->s0_dtc;
      SCHED_CALL(first_steps(c, *S, T0, st));
    }
    S->rebuild_levels();
    SCHED_CALL(run_pass(c, *S, p, T1, st));
  }
  S->time = T1;
  S->stats[3] += 1;
  if (era_end) *era_end = static_cast<double>(T1) * tsbts::kTick;
  return TSBTS_OK;
}

int tsbts_sched_option(tsbts_ctx *c, int option, int value) {
  if (!c) return TSBTS_EINVAL;
  Scheduler *S = static_cast<Scheduler *>(c->sched);
  if (!S) return sfail(c, TSBTS_ESTATE, "tsbts_sched_option: call tsbts_sched_init first");
  if (option == TSBTS_SCHED_RULE_THREADS) {
    if (value < 1 || value > 16) return sfail(c, TSBTS_EINVAL, "rule threads must be 1 .. 16");
    S->rule_threads = value;
    return TSBTS_OK;
  }
  if (option != TSBTS_SCHED_CRITERION_BEFORE_CORRECTOR &&
      option != TSBTS_SCHED_PREDICT_ON_LOAD)
    return sfail(c, TSBTS_EINVAL, "tsbts_sched_option: unknown option");
  if (value != 0 && value != 1) return sfail(c, TSBTS_EINVAL, "option value must be 0 or 1");
  if (option == TSBTS_SCHED_CRITERION_BEFORE_CORRECTOR)
    S->crit_before = value;
  else
    S->pred_on_load = value;
  return TSBTS_OK;
}

int tsbts_sched_timing(const tsbts_ctx *c, double *seconds, int64_t *counts) {
  if (!c || !c->sched) return TSBTS_EINVAL;
  const Scheduler *S = static_cast<const Scheduler *>(c->sched);
  if (seconds) std::copy(&S->phase_s[0][0], &S->phase_s[0][0] + 16, seconds);
  if (counts) std::copy(&S->phase_n[0][0], &S->phase_n[0][0] + 8, counts);
  return TSBTS_OK;
}

int tsbts_sched_prev_steps(const tsbts_ctx *c, int64_t *dtp_ticks) {
  if (!c || !c->sched || !dtp_ticks) return TSBTS_EINVAL;
  const Scheduler *S = static_cast<const Scheduler *>(c->sched);
  std::copy(S->dtp.begin(), S->dtp.end(), dtp_ticks);
  return TSBTS_OK;
}

static int sched_restore(tsbts_ctx *c, const int64_t *t_ticks, const int64_t *dt_ticks,
                         const int64_t *dtp_ticks, const double *dtc, const int64_t *stats,
                         double time, hipStream_t st) {
  if (!c) return TSBTS_EINVAL;
  Scheduler *S = static_cast<Scheduler *>(c->sched);
  if (!S) return sfail(c, TSBTS_ESTATE, "tsbts_sched_restore: call tsbts_sched_init first");
  if (!t_ticks || !dt_ticks || !dtp_ticks || !dtc)
    return sfail(c, TSBTS_EINVAL, "tsbts_sched_restore: null state array");
  const double k_time = time / tsbts::kTick;
  if (!(k_time >= 0.0) || k_time != std::floor(k_time) || k_time > 9.0e15)
    return sfail(c, TSBTS_EINVAL, "tsbts_sched_restore: time is not a multiple of 2^-20");
  const int64_t T = static_cast<int64_t>(k_time);
  const int64_t n = S->n;
  auto pow2 = [](int64_t x) { return x > 0 && (x & (x - 1)) == 0; };
  for (int64_t i = 0; i < n; ++i) {
    const int64_t ti = t_ticks[i], di = dt_ticks[i], pi = dtp_ticks[i];
    // an era end: every particle aligned to its step, at or before T, next time after T
    const bool ok = pow2(di) && di >= S->dt_min && di <= S->dt_max && ti >= 0 && ti <= T &&
                    ti % di == 0 && ti + di > T && (pi == 0 || (pow2(pi) && pi <= ti && ti % pi == 0)) &&
                    std::isfinite(dtc[i]) && dtc[i] > 0.0;
    if (!ok) {
      snprintf(c->err, sizeof(c->err),
               "tsbts_sched_restore: particle %lld is not in an era-end state",
               static_cast<long long>(i));
      return TSBTS_EINVAL;
    }
  }
  S->t.assign(t_ticks, t_ticks + n);
  S->dt.assign(dt_ticks, dt_ticks + n);
  S->dtp.assign(dtp_ticks, dtp_ticks + n);
  S->dtc.assign(dtc, dtc + n);
  S->time = T;
  if (stats) std::copy(stats, stats + 4, S->stats);
  S->have_prev = false;
  S->pending = false;  // every pass ends with its steps stored
  // device copies of the times and steps (the bound t_last and dt), staged through the
  // pinned buffers; no step update of an earlier block step can still be reading them
  SCHED_HIP(hipStreamSynchronize(st));
  for (int64_t i = 0; i < n; ++i) {
    S->dtn_h[i] = static_cast<double>(S->dt[i]) * tsbts::kTick;
    S->dtc_h[i] = static_cast<double>(S->t[i]) * tsbts::kTick;
  }
  SCHED_HIP(hipMemcpyAsync(c->dt, S->dtn_h, sizeof(double) * n, hipMemcpyHostToDevice, st));
  SCHED_HIP(hipMemcpyAsync(c->t_last, S->dtc_h, sizeof(double) * n, hipMemcpyHostToDevice, st));
  SCHED_HIP(hipStreamSynchronize(st));
  S->rebuild_levels();
  return TSBTS_OK;
}

int tsbts_sched_state(const tsbts_ctx *c, int64_t *t_ticks, int64_t *dt_ticks, double *dtc,
                      int64_t *stats, double *time) {
  if (!c || !c->sched) return TSBTS_EINVAL;
  const Scheduler *S = static_cast<const Scheduler *>(c->sched);
  if (t_ticks) std::copy(S->t.begin(), S->t.end(), t_ticks);
  if (dt_ticks) std::copy(S->dt.begin(), S->dt.end(), dt_ticks);
  if (dtc) std::copy(S->dtc.begin(), S->dtc.end(), dtc);
  if (stats) std::copy(S->stats, S->stats + 4, stats);
  if (time) *time = static_cast<double>(S->time) * tsbts::kTick;
  return TSBTS_OK;
}

int tsbts_sched_init(tsbts_ctx *c, double eta, int passes, double dt_min, double dt_max,
                     double era, hipStream_t st) {
  if (!c) return TSBTS_EINVAL;
  return tsbts::guarded(c, "tsbts_sched_init",
                        [&] { return sched_init(c, eta, passes, dt_min, dt_max, era, st); });
}

int tsbts_sched_era(tsbts_ctx *c, double *era_end, hipStream_t st) {
  if (!c) return TSBTS_EINVAL;
  return tsbts::guarded(c, "tsbts_sched_era", [&] { return sched_era(c, era_end, st); });
}

int tsbts_sched_restore(tsbts_ctx *c, const int64_t *t_ticks, const int64_t *dt_ticks,
                        const int64_t *dtp_ticks, const double *dtc, const int64_t *stats,
                        double time, hipStream_t st) {
  if (!c) return TSBTS_EINVAL;
  return tsbts::guarded(c, "tsbts_sched_restore", [&] {
    return sched_restore(c, t_ticks, dt_ticks, dtp_ticks, dtc, stats, time, st);
  });
}

}  // extern "C"
