// Internal declarations of the TSBTS HIP library: the context, device helpers shared by
// the kernels, and the host-side launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tsbts.h"

namespace tsbts {

constexpr int kWG = 256;    // threads per workgroup (4 wave64)
constexpr int kTJ = 256;    // j-particles per LDS tile
constexpr int kPad = 512;   // particle arrays are padded to a multiple of this
constexpr float kFarF = 1.0e18f;  // position of padding particles (zero mass)
constexpr double kFar = 1.0e18;

// Plane indices of the context's particle arrays.
//   p64: [5][npad] float64: x, y, z, m, w = m^(-2/3)
//   v64: [3][npad] float64: velocities at the predicted time
//   p32: [8][npad] float32: x_hi, y_hi, z_hi, m, x_lo, y_lo, z_lo, w = m^(-2/3)
enum { P64_X = 0, P64_M = 3, P64_W = 4, P64_PLANES = 5 };
enum { P32_XH = 0, P32_M = 3, P32_XL = 4, P32_W = 7, P32_VX = 8, P32_E = 11, P32_PLANES = 12 };
// History record state planes: r(3), v(3), a(3)
constexpr int kHistPlanes = 9;

struct History {
  // records being appended during a pass
  int32_t *pid = nullptr, *rank = nullptr;
  double *t = nullptr, *s = nullptr;  // s: [9][cap]
  int64_t cap = 0, count = 0;
  bool recording = false;
  // finished pass, grouped by particle
  double *ht = nullptr, *hs = nullptr;  // hs: [9][hcap]
  int32_t *off = nullptr;               // [n + 1]
  int32_t *cur = nullptr;               // [n] interpolation cursor
  int64_t hcap = 0, hcount = 0;
  bool valid = false;
  int32_t *cnt = nullptr;               // [n] records per particle in the current pass
  int32_t *tsum = nullptr;              // per-tile sums of the offset scan
};

}  // namespace tsbts

struct tsbts_ctx {
  int64_t n = 0, npad = 0;
  double eps = 0.0;
  int precision = TSBTS_MIXED;
  int flags = 0;
  int device = 0;
  // bound caller state
  double *r = nullptr, *v = nullptr, *a = nullptr, *t_last = nullptr, *dt = nullptr;
  const double *m = nullptr;
  // predicted particle arrays
  double *p64 = nullptr, *v64 = nullptr;
  float *p32 = nullptr;
  double pred_t = 0.0;
  bool have_pred = false;
  // partial sums of split-j reductions
  double *part = nullptr;
  int64_t part_cap = 0;  // elements
  // adjoint seeds in particle order (all-active adjoint), [4][npad]
  double *gord = nullptr;
  // energy partials
  double *epart = nullptr;
  int64_t epart_cap = 0;
  tsbts::History h;
  // native host scheduler (tsbts_sched_*), owned
  void *sched = nullptr;
  // launch-shape tuning (tsbts_tune)
  int tune_blocks = 8192;
  int tune_ipl = 0;
  int tune_chunk = 0;  // j-particles per split unit of the scalar-load kernels (0: automatic)
  int tune_sym = 2;    // symmetric all-targets kernels: 0 off, 1 on, 2 automatic
  int check_idx = 0;   // device range check of every active set (TSBTS_TUNE_CHECK_INDICES)
  int *idx_flag_h = nullptr, *idx_flag_d = nullptr;  // its results: [0] an index out of
                                                      // range, [1] a repeated index
                                                      // (mapped pinned memory)
  int32_t *idx_seen = nullptr;  // [n] occurrence counters of the check
  // finished-workgroup counts of the small-set force [0] and criterion [1] launches whose
  // last workgroup reduces the partials (last_workgroup); zero between launches
  uint32_t *done = nullptr;
  // symmetric all-targets kernels: work items (int4) and partials
  void *sym_items = nullptr;
  int sym_items_n = 0;
  int64_t sym_items_npad = 0;
  int sym_chunk = 0;
  void *sym_part = nullptr;
  int64_t sym_part_bytes = 0;
  // split calls of large partial active sets (split.hip): one allocation for the compact
  // copies of the targets and of the other particles (split_cap particles each), the
  // marks and scan of the other particles, the symmetric part's results and work items
  void *split_buf = nullptr;
  int64_t split_cap = 0;
  int tune_split = 2;  // 0 off, 1 from kSplitMinAct targets, 2 automatic
  char err[512] = {0};
};

namespace tsbts {

// ------------------------------------------------------------------ device helpers

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Renumber
// so that each XCD receives a contiguous range of logical block ids; nblk is a multiple
// of 8.
__device__ __forceinline__ int xcd_linear(int bid, int nblk) {
  return (bid & 7) * (nblk >> 3) + (bid >> 3);
}

__device__ __forceinline__ float rsq_f32(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_f64_approx(double x) { return __builtin_amdgcn_rsq(x); }

// 1/sqrt(s) in float64: hardware estimate refined by Newton-Raphson iterations
// y <- y (3 - s y^2) / 2, each of which roughly doubles the number of correct bits.
template <int STEPS>
__device__ __forceinline__ double rsqrt_f64(double s) {
  double y = rsq_f64_approx(s);
  const double hs = 0.5 * s;
#pragma unroll
  for (int k = 0; k < STEPS; ++k) y = y * fma(-hs * y, y, 1.5);
  return y;
}

// Split a float64 into a float32 pair whose sum carries ~48 significant bits.
__device__ __forceinline__ void split_hilo(double x, float &hi, float &lo) {
  hi = static_cast<float>(x);
  lo = static_cast<float>(x - static_cast<double>(hi));
}

// m^(-2/3): the per-source weight of the free-fall criterion term (infinite for m = 0).
__device__ __forceinline__ double ff_weight(double m) {
  return m > 0.0 ? 1.0 / cbrt(m * m) : __builtin_inf();
}

// Fixed-order butterfly reductions over one wave64 (every lane receives the result).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = fmin(x, __shfl_xor(x, off, 64));
  return x;
}

// Reduction over one wave64 of NV values per lane (NV a power of two, at most 64) by
// recursive halving: at each of the log2(NV) stages a lane keeps half of its values and
// combines them with its partner's copies of the same values (one shuffle per kept value,
// 63 shuffles for 64 values where separate butterflies take 384); the remaining stages
// combine the one value left across lanes.  Lane l returns value l >> (6 - log2 NV),
// combined over all 64 lanes (the same in every lane of its group); x is consumed.
template <int NV, class T, class Op>
__device__ __forceinline__ T wave_reduce_many(T (&x)[NV], int lane, Op op) {
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "power of two up to 64");
  constexpr int M = NV == 1 ? 0 : NV == 2 ? 1 : NV == 4 ? 2 : NV == 8 ? 3 : NV == 16 ? 4
                  : NV == 32 ? 5 : 6;
#pragma unroll
  for (int s = 0; s < M; ++s) {
    const int o = 32 >> s;
    const int half = NV >> (s + 1);
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      // both elements read first: a select between array elements would become a select
      // of addresses, which keeps a float64 array out of registers
      const T a = x[i], b = x[half + i];
      const T keep = up ? b : a;
      const T send = up ? a : b;
      x[i] = op(keep, __shfl_xor(send, o, 64));
    }
  }
  T r = x[0];
#pragma unroll
  for (int o = 32 >> M; o >= 1; o >>= 1) r = op(r, __shfl_xor(r, o, 64));
  return r;
}

// Whether this workgroup is the last of its launch (a one-dimensional grid) to get here,
// for a launch whose last workgroup finishes a reduction over every workgroup's stores.
// Every thread makes its stores visible device-wide (agent-scope fence: across the XCDs'
// separate L2 caches) before one thread counts the workgroup in `done`; the last one
// resets the count to zero for the next launch and, after an acquire fence of every
// thread, sees all stores made before the other workgroups counted.  No workgroup waits
// for another.  Every thread of the workgroup must call it.
__device__ __forceinline__ bool last_workgroup(uint32_t *done) {
  __shared__ uint32_t last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t before = atomicAdd(done, 1u);
    last = before + 1 == gridDim.x ? 1u : 0u;
    if (last) atomicExch(done, 0u);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  return true;
}

// Split-j partials are combined by one thread per target when there are few slices and
// by one wave per target (lanes striding over the slices) when there are many.
constexpr int kWaveReduceSlices = 16;
// ... but only for few targets: with many targets one thread per target reads the
// partials coalesced, while one wave per target would touch a cache line per slice.
constexpr int64_t kWaveReduceMaxTargets = 4096;
__host__ __device__ inline bool use_wave_reduce(int n_slices, int64_t n_targets) {
  return n_slices >= kWaveReduceSlices && n_targets <= kWaveReduceMaxTargets;
}
// From kRowsReduceMinTargets targets on (force and criterion), many slices are combined
// by a workgroup per 64 consecutive targets instead, its kRowsWaves waves each adding a
// contiguous range of slices: rows of 64 consecutive partials are read coalesced (the
// wave-per-target form touches a cache line per 8-byte partial).  Below that there are
// too few such workgroups (at 256 targets 4, each wave walking 128 slices: 43 against
// 34 us per call at N = 131072).
constexpr int64_t kRowsReduceMinTargets = 2048;
constexpr int kRowsWaves = 16;
__host__ __device__ inline bool use_rows_reduce(int n_slices, int64_t n_targets) {
  return n_slices >= kWaveReduceSlices && n_targets >= kRowsReduceMinTargets;
}

// The small-set kernels' last workgroup reduces the partials (W values per slice) itself
// when the launch has at most kFuseSlices workgroups and each of its threads then reads
// at most kFuseLoads partials; otherwise a reduction kernel follows.  Every workgroup of a
// fused launch pays an agent-scope fence (an L2 write-back on this multi-XCD part): at 16
// workgroups that costs less than a second launch, at 512 (N = 131072) it costs 20 us
// more.
constexpr int kFuseLoads = 32;
constexpr int kFuseSlices = 64;
__host__ __device__ inline bool fuse_small_reduce(int n_slices, int W) {
  const int parts = W <= kWG ? kWG / W : 1;
  return W <= kWG && n_slices <= kFuseSlices && (n_slices + parts - 1) / parts <= kFuseLoads;
}

// Active sets up to this size use the j-parallel pair kernels (one source per lane).
constexpr int kSmallAct = 32;
// ... and for the float64 force kernel up to this size.
constexpr int kSmallActFp64 = 16;

__host__ __device__ constexpr int64_t round_up(int64_t x, int64_t q) {
  return (x + q - 1) / q * q;
}

// ------------------------------------------------------------------ launch plans

struct SplitPlan {
  int n_itiles;        // i-tiles of ipl*kWG targets
  int n_slices;        // j-slices
  int tiles_per_slice; // j-tiles of kTJ per slice
  int nblk;            // launched blocks (multiple of 8)
};

SplitPlan plan_split(int64_t n_targets, int ipl, int64_t n_jtiles, int target_blocks);

// Block -> (target tile, j-slice) of a split launch.  Each XCD takes a contiguous range of
// logical ids (xcd_linear).  When the slice count is a multiple of 8, each XCD's range is
// one group of n_slices/8 consecutive slices in which the slice varies fastest: the
// workgroups an XCD runs back to back share a target tile, whose gathered records then
// come from that XCD's L2, and sweep the group's slices, whose sources stay in the same
// L2.  Otherwise the target tile varies fastest over all slices.  Either way every
// (tile, slice) pair is computed by exactly one workgroup, as before the remapping.
__device__ __forceinline__ void split_tile(int bid, const SplitPlan &p, int &itile,
                                           int &slice) {
  const int L = xcd_linear(bid, p.nblk);
  const int g = (p.n_slices & 7) == 0 ? (p.n_slices >> 3) : 1;
  const int per = g * p.n_itiles;
  const int r = L % per;
  itile = r / g;
  slice = (L / per) * g + r % g;
}

// Targets per lane of the force and criterion kernels for an active set of n_act.
inline int targets_per_lane(const tsbts_ctx *c, int n_act) {
  if (c->tune_ipl) return c->tune_ipl;
  return n_act < 8192 ? 1 : 2;
}

// The force kernel reads its j-particles through wave-uniform (scalar) loads unless a
// targets-per-lane count was set, which selects the LDS-staged kernel.
inline bool force_scalar_j(const tsbts_ctx *c) { return c->tune_ipl == 0; }
inline int force_targets_per_lane(const tsbts_ctx *c, int n_act) {
  return force_scalar_j(c) ? 1 : targets_per_lane(c, n_act);
}
// j-particles per split unit of the scalar-load kernels: whole tiles of kTJ, or quarter
// tiles when whole tiles would give too few workgroups to fill the chip (small N or small
// active sets), so that the j-range splits over 4x more workgroups.
constexpr int kChunkSmall = 64;
inline int scalar_chunk(const tsbts_ctx *c, int n_act, int ipl) {
  if (c->tune_chunk) return c->tune_chunk;
  const int64_t itiles = (n_act + ipl * kWG - 1) / (ipl * kWG);
  return itiles * (c->npad / kTJ) < 512 ? kChunkSmall : kTJ;
}
// The criterion kernel likewise for large active sets (from 8192 targets, two targets per
// lane, twice the workgroups) and for small launches (one target per lane, quarter-tile
// units); in between the LDS-staged kernel with one target per lane measured faster.
inline bool criterion_scalar_j(const tsbts_ctx *c, int n_act) {
  return force_scalar_j(c) && (n_act >= 8192 || scalar_chunk(c, n_act, 1) == kChunkSmall);
}
inline int criterion_targets_per_lane(const tsbts_ctx *c, int n_act) {
  if (!criterion_scalar_j(c, n_act)) return targets_per_lane(c, n_act);
  return n_act >= 8192 ? 2 : 1;
}
inline int criterion_blocks(const tsbts_ctx *c, int n_act) {
  return criterion_scalar_j(c, n_act) && n_act >= 8192 ? 2 * c->tune_blocks : c->tune_blocks;
}

// ------------------------------------------------------------------ launchers
// Each returns a hipError_t from the launch (hipSuccess on success).

// New steps of the previous block step not yet stored (native scheduler; predict.hpp).
struct PendingSteps {
  const int64_t *tag;  // [n] (step << 32) | list position, written by the corrector
  const double *dt;    // [k] new steps, by position in that step's active list
  int64_t step;
  // the same steps as powers of two, dt[q] = 2^exp[q], when k <= kInlinePend (host
  // memory, copied into the launch arguments); null: the kernels read dt
  const int8_t *exp;
  int k;
};
struct InlineIdx;
hipError_t launch_predict(tsbts_ctx *c, double t_block, int use_history, hipStream_t st,
                          const PendingSteps *pend = nullptr, const InlineIdx *in = nullptr);
hipError_t launch_load_positions(tsbts_ctx *c, const double *r, const double *m,
                                 hipStream_t st);
hipError_t launch_snapshot(tsbts_ctx *c, double T, double *r_out, double *v_out,
                           hipStream_t st);

struct CorrectArgs;
// Force, potential and criterion (with the predicted velocities) in one pass; with corr,
// the corrector runs in its reduction.
int64_t fused_partials_needed(const tsbts_ctx *c, int n_act);
hipError_t launch_fused(tsbts_ctx *c, const int32_t *idx, int n_act, double eta, double *acc,
                        double *pot, double *dtc, hipStream_t st,
                        const CorrectArgs *corr = nullptr);
// Tags of the native scheduler's corrector: each target g gets tag[g] = (step << 32) | q.
struct StepTags {
  int64_t *tag;
  int64_t step;
};
int force_criterion_correct(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                            double eta, double *acc, double *dtc, hipStream_t stream,
                            const StepTags *tags = nullptr);
// Force on the active set and its corrector in the same launches (checked like the two
// entry points; returns a status code).  With `in`, the active list arrives by value
// and the first kernel writes it to idx (which must then not be checked beforehand).
// With dtc, also the criterion (eta) of the corrected targets when small_criterion_fused
// holds; *crit_done tells whether it did (else the caller runs tsbts_timestep).
int force_correct_predicted(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                            int use_history, double *acc, hipStream_t stream,
                            const StepTags *tags = nullptr,
                            const PendingSteps *pend = nullptr,
                            const InlineIdx *in = nullptr, double eta = 0.0,
                            double *dtc = nullptr, int *crit_done = nullptr);
int force_correct(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                  double *acc, hipStream_t stream, const StepTags *tags = nullptr);
// tsbts_predict with pending new steps and an inline active list (either may be null).
int predict_pending(tsbts_ctx *c, double t_block, int use_history, const PendingSteps *pend,
                    const InlineIdx *in, hipStream_t stream);
// With corr, every target's corrector (correct_one) runs where its force is final.
hipError_t launch_force(tsbts_ctx *c, const int32_t *idx, int n_act, double *acc,
                        double *pot, hipStream_t st, const CorrectArgs *corr = nullptr);
// Sources of a gather launch other than the context's predicted arrays (the second part
// of a split call): n particles that exclude every target (no self pair), padded to npad,
// planes laid out as the predicted arrays with stride npad; and the first part's results
// for each target, combined with the gather's where the target is finished: for the force
// [4][n_act] acceleration (x, y, z) and potential to add, for the criterion [2][n_act] the
// maximum of q and the minimum of s*w.
struct GatherSrc {
  const float *p32;   // [12][npad] or null (float64 mode)
  const double *p64;  // [5][npad]
  const double *v64;  // [3][npad]
  int64_t n, npad;
  const double *add;
};
// The gather force kernels (never the symmetric ones) with split-j partials in `part`
// and a split aiming for `blocks` workgroups; with `src`, its sources (always the
// scalar-load kernel).
hipError_t launch_force_gather(tsbts_ctx *c, const int32_t *idx, int n_act, double *acc,
                               double *pot, double *part, int blocks, hipStream_t st,
                               const CorrectArgs *corr = nullptr,
                               const GatherSrc *src = nullptr);
// float64 partials of that launch (0 when the j-range is not split).
int64_t force_partial_elems(const tsbts_ctx *c, int n_act, int blocks);
// Fixed partial-sum array of tsbts_force_noalloc: find its address on `device` (once per
// device); returns the HIP status of the lookup.
hipError_t noalloc_setup(int device);
// Its looked-up address on `device` (NULL before noalloc_setup succeeded there).
double *noalloc_partials(int device);
hipError_t launch_timestep(tsbts_ctx *c, const int32_t *idx, int n_act, double eta,
                           double *dtc, hipStream_t st);
// The gather criterion kernels with the sources `src` (the scalar-load kernel).
hipError_t launch_timestep_gather(tsbts_ctx *c, const int32_t *idx, int n_act, double eta,
                                  double *dtc, hipStream_t st, const GatherSrc *src);
// Split calls (split.hip): a large partial active set whose pairs among the targets are
// evaluated once for both (symmetric kernels on a compact copy of the targets) and whose
// pairs with the other particles by the gather kernels (a compact copy of those as
// sources).  split_applies: whether it serves a call of n_act targets; split_prepare
// allocates its buffers (host set-up; returns a status); the launches return
// hipErrorNotReady, with nothing launched, when the buffers are not there.
bool split_applies(const tsbts_ctx *c, int64_t n_act);
int split_prepare(tsbts_ctx *c, int64_t n_act);
hipError_t launch_force_split(tsbts_ctx *c, const int32_t *idx, int n_act, double *acc,
                              double *pot, hipStream_t st, const CorrectArgs *corr);
hipError_t launch_timestep_split(tsbts_ctx *c, const int32_t *idx, int n_act, double eta,
                                 double *dtc, hipStream_t st);
// Exclusive scan of cnt[0 .. n) into off[0 .. n] (off[n]: the total) with tile sums in
// tsum (one per 8192 counts); cur receives a copy of off[0 .. n) (may equal off).
hipError_t launch_exclusive_scan(const int32_t *cnt, int64_t n, int32_t *tsum, int32_t *off,
                                 int32_t *cur, hipStream_t st);
constexpr int64_t kScanCounts = 8192;  // counts per tile sum of launch_exclusive_scan
hipError_t launch_backward(tsbts_ctx *c, const int32_t *idx, int n_act, const double *ga,
                           const double *gp, double *gr, double *gm, hipStream_t st);
hipError_t launch_energy(tsbts_ctx *c, const double *r, const double *v, const double *m,
                         double *out, hipStream_t st);

hipError_t launch_correct(tsbts_ctx *c, const int32_t *idx, int n_act, double t_block,
                          const double *acc_new, hipStream_t st);
hipError_t launch_set_dt(tsbts_ctx *c, const int32_t *idx, int n_act, const double *dt_new,
                         hipStream_t st);
hipError_t launch_history_begin(tsbts_ctx *c, hipStream_t st);
hipError_t launch_history_end(tsbts_ctx *c, hipStream_t st);
hipError_t launch_leapfrog_adjoint(tsbts_ctx *c, int phase, double h, const double *rbar,
                                   double *vbar, double *abar, double *g_out,
                                   hipStream_t st);
// x[0 .. len) = v with a fill kernel (no memset node if a caller captures the stream).
hipError_t launch_fill(double *x, int64_t len, double v, hipStream_t st);
hipError_t launch_block_adjoint(tsbts_ctx *c, int phase, const int32_t *idx, int n_act,
                                double t_block, double *rbar, double *vbar, double *abar,
                                double *pbar, double *seeds, hipStream_t st);
// Largest active set of the j-parallel small-set kernels.
int small_act_limit(const tsbts_ctx *c);
// Predictor and force (with the corrector, if corr) in the small-set kernels, the sources
// predicted as they are loaded (n_act <= small_act_limit).
// With dtc (and corr), when small_criterion_fused holds, the launch's last workgroup also
// takes the criterion of the corrected targets into dtc (as launch_timestep would).
hipError_t launch_force_predicted(tsbts_ctx *c, const int32_t *idx, int n_act, double t_block,
                                  int use_history, double *acc, double *pot, hipStream_t st,
                                  const CorrectArgs *corr, const PendingSteps *pend = nullptr,
                                  const InlineIdx *in = nullptr, double eta = 0.0,
                                  double *dtc = nullptr);
// Whether launch_force_predicted takes the criterion of n_act targets itself: the one
// workgroup's passes over the particles are short (j-tiles times groups of 8 targets at
// most kCritFuseTiles).
constexpr int kCritFuseTiles = 8;
bool small_criterion_fused(const tsbts_ctx *c, int n_act);
// Symmetric all-targets criterion (timestep_sym.hip); plan from sym_plan.  With `set`, the
// kernels run on that particle set instead of the context's predicted arrays; with `raw`,
// each target's maximum and minimum go there unfinished ([2][n_act]) instead of to dtc.
struct SymPlan;
struct SymSet;
hipError_t launch_timestep_sym(tsbts_ctx *c, const SymPlan &plan, const int32_t *idx,
                               int n_act, double eta, double *dtc, hipStream_t st,
                               const SymSet *set = nullptr, double *raw = nullptr);
// Symmetric all-targets force (force_sym.hip): whether it serves the call, and its launch
// (on `set` instead of the context's predicted arrays when given).
bool force_sym_applies(const tsbts_ctx *c, int64_t n_act);
hipError_t launch_force_sym(tsbts_ctx *c, const SymPlan &plan, const int32_t *idx, int n_act,
                            double *acc, double *pot, hipStream_t st,
                            const CorrectArgs *corr, const SymSet *set = nullptr);
// Symmetric all-targets force adjoint (backward_sym.hip), after the seeds are ordered.
bool bwd_sym_applies(const tsbts_ctx *c, int64_t n_act);
hipError_t launch_bwd_sym(tsbts_ctx *c, const SymPlan &plan, double *gr, double *gm,
                          hipStream_t st);
// Adjoints of the passes of an era (hist_adjoint.hip).
hipError_t launch_interp_adjoint(tsbts_ctx *c, double t_block, double *pbar, double *hbar,
                                 hipStream_t st);
hipError_t launch_record_adjoint(tsbts_ctx *c, const int32_t *idx, int n_act, double t_block,
                                 const int32_t *off, const double *ht, int64_t n_records,
                                 const double *hbar, double *rbar, double *vbar,
                                 hipStream_t st);
hipError_t launch_accumulate3(int64_t len, const double *x0, const double *x1,
                              const double *x2, double *y0, double *y1, double *y2,
                              hipStream_t st);

// Free the native scheduler attached to a context (if any).
void destroy_scheduler(tsbts_ctx *c);

// Scratch needed by the split-j kernels for a given active-set size (float64 elements).
int64_t partial_elems_needed(const tsbts_ctx *c, int n_act);
int64_t energy_partials_needed(const tsbts_ctx *c);

}  // namespace tsbts
