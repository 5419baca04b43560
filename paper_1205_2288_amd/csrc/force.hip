// Softened direct-summation acceleration and potential of the active set against all
// particles (Algorithm 2, step 5; Plummer softening of Section 3).
//
// Layout and schedule (gfx950):
//   - a workgroup of 256 threads holds IPL*256 target particles, IPL per lane, in
//     registers (gathered through active_idx from the predicted arrays);
//   - the j-particles are streamed through LDS in tiles of 256 records, staged with
//     coalesced structure-of-arrays loads (one record per thread) and read back as
//     wave-uniform broadcasts;
//   - mixed precision accumulates each tile in float32 and folds the tile sums into
//     float64 accumulators; float64 mode accumulates in float64;
//   - when the active set is small the j-sum is split over workgroups (the paper's work
//     partitioning, Section 5), each writing float64 partials that a second kernel adds
//     in slice order (no atomics, bit-reproducible);
//   - logical block ids are renumbered so that the workgroups on one XCD share j-slices
//     and hit in that XCD's L2.
// The self pair (j == i) is masked by index, but only in the tiles that contain some
// lane's own particle: a wave-uniform vote picks a masked copy of the inner loop for
// those tiles and the unmasked one elsewhere, so the mask costs nothing on almost every
// tile and no large self term ever enters a float32 accumulator.
#include "correct.hpp"
#include "criterion.hpp"
#include "force_pair.hpp"
#include "predict.hpp"
#include "sym.hpp"
#include <algorithm>
#include <type_traits>

namespace tsbts {
namespace {

// The time-step criterion of the targets after their correction, taken by the last
// workgroup of a small predicted launch (small_criterion_last).
struct CritArgs {
  int on;
  int64_t n;  // particles; j >= n are padding
  const float *p32;
  const double *p64;
  const double *v64;
  int64_t npad;
  double eps2;
  double eta;
  double *dtc;
};

struct ForceArgs {
  const float *p32;
  const double *p64;
  int64_t npad;
  const int32_t *idx;
  int n_act;
  SplitPlan plan;
  int n_jtiles;
  float eps2f;
  double eps2;
  double *part;  // [S][4][n_act] raw sums when S > 1
  double *acc;   // [3][n_act]
  double *pot;   // [n_act] or null
  int blocks;    // workgroups a split launch aims for
  int ipl;       // targets per lane
  int scalar_j;  // j-particles through scalar loads (k_force_scalar)
  int chunk;     // j-particles per split unit of k_force_scalar
  int correct;   // apply the corrector to each target as its force is finished
  CorrectArgs corr;
  uint32_t *done;   // finished-workgroup count of the small-set kernels
  int fuse_reduce;  // the small-set kernel's last workgroup reduces the partials
  CritArgs crit;    // ... and then takes the criterion (k_force_small_pred)
  // Sources of k_force_scalar (null: the predicted arrays above): planes of stride snpad.
  // self = 0 when they exclude the targets (no self pair to skip).
  const float *s32 = nullptr;
  const double *s64 = nullptr;
  int64_t snpad = 0;
  int self = 1;
  // null, or [4][n_act]: acceleration (x, y, z) and potential from the other part of a
  // split call, added to each target's sums where it is finished
  const double *add = nullptr;
};

// Scale and store target q's sums; with the corrector, correct it (its inputs `ts` when
// the caller holds them, else read from the context).
template <class V, int NEWTON>
__device__ __forceinline__ void finish(const ForceArgs &A, int q, int64_t g, double sx,
                                       double sy, double sz, double sp,
                                       const TargetState *ts = nullptr) {
  const double k = Scale<V, NEWTON>::kAcc;
  double an[3] = {k * sx, k * sy, k * sz};
  double pn = -sp;
  if (A.add) {
#pragma unroll
    for (int c = 0; c < 3; ++c) an[c] += A.add[c * A.n_act + q];
    pn += A.add[3 * A.n_act + q];
  }
  A.acc[q] = an[0];
  A.acc[A.n_act + q] = an[1];
  A.acc[2 * A.n_act + q] = an[2];
  if (A.pot) A.pot[q] = pn;
  if (A.correct) correct_target(A.corr, q, g, an, ts ? *ts : load_target(A.corr, g));
}

template <class V, int NEWTON, int MASK, int POT, int IPL, class F>
__device__ __forceinline__ void tile_loop(const typename V::J *sj, const typename V::I *I,
                                          const int *g, int64_t jbase, F eps2, F *fx, F *fy,
                                          F *fz, F *fp) {
#pragma unroll 4
  for (int jj = 0; jj < kTJ; ++jj) {
    const typename V::J J = sj[jj];
#pragma unroll
    for (int k = 0; k < IPL; ++k)
      pair_acc<V, NEWTON, MASK, POT>(I[k], J, eps2, MASK && (jbase + jj == g[k]), fx[k], fy[k],
                                fz[k], fp[k]);
  }
}

template <class V, int NEWTON, int POT, int IPL>
__global__ __launch_bounds__(kWG) void k_force(ForceArgs A) {
  static_assert(kTJ == kWG, "one staged record per thread");
  using F = typename V::F;
  __shared__ typename V::J sj[kTJ];
  const int tid = threadIdx.x;
  int itile, slice;
  split_tile(blockIdx.x, A.plan, itile, slice);
  if (slice >= A.plan.n_slices) return;
  const int jt0 = slice * A.plan.tiles_per_slice;
  const int jt1 = min(jt0 + A.plan.tiles_per_slice, A.n_jtiles);
  const int64_t P = A.npad;
  const F eps2 = sizeof(F) == 4 ? static_cast<F>(A.eps2f) : static_cast<F>(A.eps2);

  typename V::I I[IPL];
  int q[IPL];
  int g[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    q[k] = (itile * IPL + k) * kWG + tid;
    g[k] = A.idx[min(q[k], A.n_act - 1)];
    I[k] = V::load_i(A.p32, A.p64, P, g[k]);
  }
  double sx[IPL], sy[IPL], sz[IPL], sp[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) sx[k] = sy[k] = sz[k] = sp[k] = 0.0;

  for (int jt = jt0; jt < jt1; ++jt) {
    const int64_t jbase = static_cast<int64_t>(jt) * kTJ;
    const typename V::J rec = V::load_j(A.p32, A.p64, P, jbase + tid, Scale<V, NEWTON>::kMass);
    __syncthreads();
    sj[tid] = rec;
    __syncthreads();
    F fx[IPL], fy[IPL], fz[IPL], fp[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) fx[k] = fy[k] = fz[k] = fp[k] = F(0);
    bool mine = false;
#pragma unroll
    for (int k = 0; k < IPL; ++k) mine |= (g[k] >= jbase && g[k] < jbase + kTJ);
    if (__ballot(mine) != 0)
      tile_loop<V, NEWTON, 1, POT, IPL>(sj, I, g, jbase, eps2, fx, fy, fz, fp);
    else
      tile_loop<V, NEWTON, 0, POT, IPL>(sj, I, g, jbase, eps2, fx, fy, fz, fp);
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      sx[k] += static_cast<double>(fx[k]);
      sy[k] += static_cast<double>(fy[k]);
      sz[k] += static_cast<double>(fz[k]);
      sp[k] += static_cast<double>(fp[k]);
    }
  }

#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    if (q[k] >= A.n_act) continue;
    if (A.plan.n_slices == 1) {
      finish<V, NEWTON>(A, q[k], g[k], sx[k], sy[k], sz[k], sp[k]);
    } else {
      double *out = A.part + static_cast<int64_t>(slice) * 4 * A.n_act;
      out[q[k]] = sx[k];
      out[A.n_act + q[k]] = sy[k];
      out[2 * A.n_act + q[k]] = sz[k];
      out[3 * A.n_act + q[k]] = sp[k];
    }
  }
}

// j-particles through scalar loads: the j index is the same on every lane, so the loads
// of the j record from the predicted arrays are wave-uniform and become scalar loads; the
// record then sits in SGPRs and the pair arithmetic takes it as scalar operands.  No LDS
// staging and no barriers; one target per lane.  Same tiles of kTJ j-particles, same
// self-pair vote and the same float32-in-tile / float64-across-tiles sums as k_force.
template <class V, int NEWTON, int MASK, int POT, int CH, class F>
__device__ __forceinline__ void scalar_tile(const ForceArgs &A, const typename V::I &I, int g,
                                            int64_t jbase, F eps2, F &fx, F &fy, F &fz,
                                            F &fp) {
#pragma unroll 8
  for (int jj = 0; jj < CH; ++jj) {
    const typename V::J J =
        V::load_j(A.s32, A.s64, A.snpad, jbase + jj, Scale<V, NEWTON>::kMass);
    pair_acc<V, NEWTON, MASK, POT>(I, J, eps2, MASK && (jbase + jj == g), fx, fy, fz, fp);
  }
}

// Split units of CH j-particles (A.n_jtiles counts them here).
template <class V, int NEWTON, int POT, int CH>
__global__ __launch_bounds__(kWG) void k_force_scalar(ForceArgs A) {
  using F = typename V::F;
  int itile, slice;
  split_tile(blockIdx.x, A.plan, itile, slice);
  if (slice >= A.plan.n_slices) return;
  const int jt0 = slice * A.plan.tiles_per_slice;
  const int jt1 = min(jt0 + A.plan.tiles_per_slice, A.n_jtiles);
  const F eps2 = sizeof(F) == 4 ? static_cast<F>(A.eps2f) : static_cast<F>(A.eps2);
  const int q = itile * kWG + static_cast<int>(threadIdx.x);
  const int g = A.idx[min(q, A.n_act - 1)];
  const typename V::I I = V::load_i(A.p32, A.p64, A.npad, g);
  const int gs = A.self ? g : -1;  // the target's index among the sources
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
  for (int jt = jt0; jt < jt1; ++jt) {
    const int64_t jbase = static_cast<int64_t>(jt) * CH;
    F fx = F(0), fy = F(0), fz = F(0), fp = F(0);
    if (__ballot(gs >= jbase && gs < jbase + CH) != 0)
      scalar_tile<V, NEWTON, 1, POT, CH>(A, I, gs, jbase, eps2, fx, fy, fz, fp);
    else
      scalar_tile<V, NEWTON, 0, POT, CH>(A, I, gs, jbase, eps2, fx, fy, fz, fp);
    sx += static_cast<double>(fx);
    sy += static_cast<double>(fy);
    sz += static_cast<double>(fz);
    sp += static_cast<double>(fp);
  }
  if (q >= A.n_act) return;
  if (A.plan.n_slices == 1) {
    finish<V, NEWTON>(A, q, g, sx, sy, sz, sp);
  } else {
    double *out = A.part + static_cast<int64_t>(slice) * 4 * A.n_act;
    out[q] = sx;
    out[A.n_act + q] = sy;
    out[2 * A.n_act + q] = sz;
    out[3 * A.n_act + q] = sp;
  }
}

// Small active sets (n_act <= kSmallAct): one 256-particle j-tile per workgroup, one
// source per lane, the targets broadcast from LDS.  The pairs of kSmallGroup targets are
// summed over the wave together (wave_reduce_many: one shuffle per kept value instead of a
// butterfly per value), then over the 4 waves in a fixed order into one float64 partial
// per tile and target.  Keeps every lane busy where an i-tile would leave all but n_act
// lanes idle.  When the partials are few (fuse_reduce) the launch's last workgroup adds
// them and finishes the targets (small_reduce_last) instead of a second kernel.
constexpr int kSmallGroup = 8;

template <class V, int NEWTON>
__device__ __forceinline__ void small_tile_sums(const ForceArgs &A, const typename V::I *si,
                                                const int *sg, const typename V::J &J,
                                                int64_t j, int tile) {
  using F = typename V::F;
  __shared__ F red[kSmallAct][4][kWG / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const F eps2 = sizeof(F) == 4 ? static_cast<F>(A.eps2f) : static_cast<F>(A.eps2);
  for (int q0 = 0; q0 < A.n_act; q0 += kSmallGroup) {
    F x[4 * kSmallGroup];
#pragma unroll
    for (int u = 0; u < kSmallGroup; ++u) {
      const int q = q0 + u;
      F ax = F(0), ay = F(0), az = F(0), pp = F(0);
      if (q < A.n_act) pair_acc<V, NEWTON, 1, 1>(si[q], J, eps2, j == sg[q], ax, ay, az, pp);
      x[4 * u] = ax;
      x[4 * u + 1] = ay;
      x[4 * u + 2] = az;
      x[4 * u + 3] = pp;
    }
    const F r = wave_reduce_many<4 * kSmallGroup>(x, lane, [](F a, F b) { return a + b; });
    // lane l holds value l >> 1: target q0 + (l >> 3), component (l >> 1) & 3
    const int q = q0 + (lane >> 3);
    if ((lane & 1) == 0 && q < A.n_act) red[q][(lane >> 1) & 3][w] = r;
  }
  __syncthreads();
  for (int t = tid; t < 4 * A.n_act; t += kWG) {
    const int q = t >> 2, c = t & 3;
    double s = 0.0;
#pragma unroll
    for (int ww = 0; ww < kWG / 64; ++ww) s += static_cast<double>(red[q][c][ww]);
    A.part[(static_cast<int64_t>(tile) * 4 + c) * A.n_act + q] = s;
  }
}

// The split-j reduction by the launch's last workgroup.  A slice's partials form a row of
// W = 4 n_act values; thread t adds value t % W over part t / W of the slices (P = kWG / W
// consecutive parts, coalesced rows), in slice order; the parts are then added in order
// and each target finishes (sg: the active list in LDS; ts: the corrector's inputs of
// target tid, held by thread tid, or null).
template <class V, int NEWTON>
__device__ __forceinline__ void small_reduce_last(const ForceArgs &A, const int *sg,
                                                  const TargetState *ts = nullptr) {
  __shared__ double sums[kWG];
  const int tid = threadIdx.x;
  const int W = 4 * A.n_act, P = kWG / W, S = A.plan.n_slices;
  const int L = (S + P - 1) / P;
  const int p = tid / W, v = tid - p * W;
  double s = 0.0;
  if (p < P) {
    const int s1 = min(S, (p + 1) * L);
#pragma unroll 8
    for (int sl = p * L; sl < s1; ++sl) s += A.part[static_cast<int64_t>(sl) * W + v];
  }
  sums[tid] = s;
  __syncthreads();
  if (tid < A.n_act) {
    double f[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double t = 0.0;
      for (int pp = 0; pp < P; ++pp) t += sums[pp * W + c * A.n_act + tid];
      f[c] = t;
    }
    finish<V, NEWTON>(A, tid, sg[tid], f[0], f[1], f[2], f[3], ts);
  }
}

// The criterion of the targets after their correction, by the launch's last workgroup
// alone (a small active set on few particles): lane l takes the particles l, l + 256, ...
// against kCritGroup targets at a time, the records of kCritBatch tiles loaded before
// their pairs so that one memory latency serves several tiles; the maxima and negated
// minima are then combined over the wave (wave_reduce_many) and over the 4 waves.  Max
// and min are exact, so dtc is what the criterion kernels give bit for bit.  The targets'
// corrected velocities were stored by this workgroup; every other particle's predicted
// record was stored before its workgroup counted itself in, so last_workgroup made it
// visible.
constexpr int kCritGroup = 8;
constexpr int kCritBatch = 4;

template <class V>
__device__ __forceinline__ void small_criterion_last(const ForceArgs &A, const int *sg) {
  using F = typename V::F;
  using SR = StepRec<V>;
  constexpr int G = kCritGroup;
  __shared__ typename SR::I ti[kSmallAct];
  __shared__ F red[kSmallAct][2][kWG / 64];
  const CritArgs &C = A.crit;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  __syncthreads();
  if (tid < A.n_act) ti[tid] = load_iv<V>(C, sg[tid]);
  __syncthreads();
  const F eps2 = static_cast<F>(C.eps2);
  const int n_tiles = static_cast<int>(C.npad / kTJ);
  const F inf = sizeof(F) == 4 ? static_cast<F>(__builtin_inff()) : static_cast<F>(__builtin_inf());
  for (int q0 = 0; q0 < A.n_act; q0 += G) {
    F qm[G], sm[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      qm[u] = F(0);
      sm[u] = inf;
    }
    for (int jt = 0; jt < n_tiles; jt += kCritBatch) {
      typename SR::J J[kCritBatch];
#pragma unroll
      for (int b = 0; b < kCritBatch; ++b)
        if (jt + b < n_tiles) J[b] = load_jv<V>(C, static_cast<int64_t>(jt + b) * kTJ + tid);
#pragma unroll
      for (int b = 0; b < kCritBatch; ++b) {
        if (jt + b >= n_tiles) break;
        const int64_t j = static_cast<int64_t>(jt + b) * kTJ + tid;
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int q = q0 + u;
          if (q < A.n_act) pair_step(ti[q], J[b], eps2, j == sg[q] || j >= C.n, qm[u], sm[u]);
        }
      }
    }
    F x[2 * G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      x[u] = qm[u];
      x[G + u] = -sm[u];
    }
    const F r = wave_reduce_many<2 * G>(x, lane, [](F a, F b) { return fmax(a, b); });
    // lane l holds value v = l >> 2: the maximum of target q0 + v (v < G), else the
    // negated minimum of target q0 + v - G
    const int v = lane >> 2;
    const int q = q0 + (v & (G - 1));
    if ((lane & 3) == 0 && q < A.n_act) {
      if (v < G)
        red[q][0][w] = r;
      else
        red[q][1][w] = -r;
    }
  }
  __syncthreads();
  if (tid < A.n_act) {
    double qmax = 0.0, swmin = __builtin_inf();
#pragma unroll
    for (int ww = 0; ww < kWG / 64; ++ww) {
      qmax = fmax(qmax, static_cast<double>(red[tid][0][ww]));
      swmin = fmin(swmin, static_cast<double>(red[tid][1][ww]));
    }
    C.dtc[tid] = finish_dt(C.eta, qmax, swmin);
  }
}

template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_force_small(ForceArgs A) {
  __shared__ typename V::I si[kSmallAct];
  __shared__ int sg[kSmallAct];
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int64_t P = A.npad;
  const int64_t j = static_cast<int64_t>(tile) * kTJ + tid;
  const typename V::J J = V::load_j(A.p32, A.p64, P, j, Scale<V, NEWTON>::kMass);
  if (tid < A.n_act) {
    sg[tid] = A.idx[tid];
    si[tid] = V::load_i(A.p32, A.p64, P, sg[tid]);
  }
  __syncthreads();
  small_tile_sums<V, NEWTON>(A, si, sg, J, j, tile);
  if (A.fuse_reduce && last_workgroup(A.done)) small_reduce_last<V, NEWTON>(A, sg);
}

// Source record of a policy built from a particle's predicted position and mass: the
// values V::load_j reads back from the planes the predictor stores for it.
template <class V>
__device__ __forceinline__ typename V::J j_from_state(double x, double y, double z, double m,
                                                      float ms) {
  typename V::J r;
  if constexpr (std::is_same<V, Fp64>::value) {
    r.x = x;
    r.y = y;
    r.z = z;
    r.m = m;
  } else if constexpr (std::is_same<V, MixSep64>::value) {
    r.x = x;
    r.y = y;
    r.z = z;
    r.m = static_cast<float>(m) * ms;
    r.w = static_cast<float>(ff_weight(m));
  } else {
    float hx, lx, hy, ly, hz, lz;
    split_hilo(x, hx, lx);
    split_hilo(y, hy, ly);
    split_hilo(z, hz, lz);
    r.a = make_float4(hx, hy, hz, static_cast<float>(m) * ms);
    r.b = make_float4(lx, ly, lz, static_cast<float>(ff_weight(m)));
  }
  return r;
}

template <class V>
__device__ __forceinline__ typename V::I i_from_state(double x, double y, double z) {
  typename V::I r;
  if constexpr (std::is_same<V, MixHiLo>::value) {
    split_hilo(x, r.xh, r.xl);
    split_hilo(y, r.yh, r.yl);
    split_hilo(z, r.zh, r.zl);
  } else {
    r.x = x;
    r.y = y;
    r.z = z;
  }
  return r;
}

// k_force_small with the prediction of its sources on load (the predictor's work folded
// into the force pass for small active sets): the thread that owns source j predicts it
// to the block time, stores its predicted planes (for the corrector and the criterion)
// and sums with the values in registers; each workgroup predicts the targets itself
// (active particles: their Taylor polynomial).  Same arithmetic as the predictor followed
// by k_force_small, so the results are the same bit for bit.
template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_force_small_pred(ForceArgs A, PredictArgs Pr,
                                                          InlineIdx in) {
  __shared__ typename V::I si[kSmallAct];
  __shared__ int sg[kSmallAct];
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int64_t j = static_cast<int64_t>(tile) * kTJ + tid;
  const float ms = Scale<V, NEWTON>::kMass;
  // Targets are active at the block time: their Taylor polynomial.  Thread q keeps target
  // q's corrector inputs (the values the prediction used, the position it gives, the
  // record count), so the last workgroup corrects without reading them back; the thread
  // that owns the target as a source stores the same predicted position.
  TargetState ts;
  if (tid < A.n_act) {
    const int g = in.k ? in.v[tid] : A.idx[tid];
    sg[tid] = g;
    const int64_t n = Pr.n;
    ts.tl = Pr.t_last[g];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ts.v[c] = Pr.v[c * n + g];
      ts.a[c] = Pr.a[c * n + g];
    }
    ts.cnt = A.correct && A.corr.record ? A.corr.cnt[g] : 0;
    double st[6];
    predict_taylor(Pr, g, ts.tl, st);
#pragma unroll
    for (int c = 0; c < 3; ++c) ts.rn[c] = st[c];
    si[tid] = i_from_state<V>(st[0], st[1], st[2]);
  }
  typename V::J J;
  if (j < Pr.n) {
    double st[6];
    predict_state(Pr, j, true, st);
    const double m = Pr.m[j];
    store_particle(Pr.o, j, st[0], st[1], st[2], st[3], st[4], st[5], m);
    J = j_from_state<V>(st[0], st[1], st[2], m, ms);
  } else {
    store_pad(Pr.o, j);
    J = j_from_state<V>(kFar, kFar, kFar, 0.0, ms);
  }
  if (blockIdx.x == 0) store_inline_idx(in, tid);
  __syncthreads();
  small_tile_sums<V, NEWTON>(A, si, sg, J, j, tile);
  if (!A.fuse_reduce || !last_workgroup(A.done)) return;
  small_reduce_last<V, NEWTON>(A, sg, &ts);
  if (A.crit.on) small_criterion_last<V>(A, sg);
}

// Add the slices' partials in slice order and finish (scale, sign).
template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_force_reduce(ForceArgs A) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q >= A.n_act) return;
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
  const int64_t stride = 4 * static_cast<int64_t>(A.n_act);
  for (int s = 0; s < A.plan.n_slices; ++s) {
    const double *in = A.part + s * stride;
    sx += in[q];
    sy += in[A.n_act + q];
    sz += in[2 * A.n_act + q];
    sp += in[3 * A.n_act + q];
  }
  finish<V, NEWTON>(A, q, A.idx[q], sx, sy, sz, sp);
}

// Same, one wave per target, lanes striding over the slices (many slices).
template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_force_reduce_wave(ForceArgs A) {
  const int q = blockIdx.x * (kWG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= A.n_act) return;
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
  const int64_t stride = 4 * static_cast<int64_t>(A.n_act);
  for (int s = lane; s < A.plan.n_slices; s += 64) {
    const double *in = A.part + s * stride;
    sx += in[q];
    sy += in[A.n_act + q];
    sz += in[2 * A.n_act + q];
    sp += in[3 * A.n_act + q];
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  sp = wave_sum(sp);
  if (lane == 0) finish<V, NEWTON>(A, q, A.idx[q], sx, sy, sz, sp);
}

// Same, a workgroup per 64 consecutive targets (one per lane) whose kRowsWaves waves each
// add a contiguous range of the slices in order; the waves' sums are then added in wave
// order (many targets and slices).
template <class V, int NEWTON>
__global__ __launch_bounds__(64 * kRowsWaves) void k_force_reduce_rows(ForceArgs A) {
  __shared__ double sums[kRowsWaves][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = blockIdx.x * 64 + lane;
  const int S = A.plan.n_slices;
  const int L = (S + kRowsWaves - 1) / kRowsWaves;
  const int s1 = min(S, (w + 1) * L);
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  if (q < A.n_act) {
    const int64_t stride = 4 * static_cast<int64_t>(A.n_act);
#pragma unroll 4
    for (int s = w * L; s < s1; ++s) {
      const double *in = A.part + s * stride;
#pragma unroll
      for (int c = 0; c < 4; ++c) t[c] += in[c * A.n_act + q];
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) sums[w][c][lane] = t[c];
  __syncthreads();
  if (w == 0 && q < A.n_act) {
    double f[4] = {0.0, 0.0, 0.0, 0.0};
    for (int ww = 0; ww < kRowsWaves; ++ww)
#pragma unroll
      for (int c = 0; c < 4; ++c) f[c] += sums[ww][c][lane];
    finish<V, NEWTON>(A, q, A.idx[q], f[0], f[1], f[2], f[3]);
  }
}

// The split-j reduction launch that suits the call (none when the j-range is not split).
template <class V, int NEWTON>
hipError_t launch_reduce(ForceArgs &A, hipStream_t st) {
  if (use_rows_reduce(A.plan.n_slices, A.n_act)) {
    const int nb = (A.n_act + 63) / 64;
    hipLaunchKernelGGL((k_force_reduce_rows<V, NEWTON>), dim3(nb), dim3(64 * kRowsWaves), 0, st,
                       A);
  } else if (use_wave_reduce(A.plan.n_slices, A.n_act)) {
    const int nb = (A.n_act + kWG / 64 - 1) / (kWG / 64);
    hipLaunchKernelGGL((k_force_reduce_wave<V, NEWTON>), dim3(nb), dim3(kWG), 0, st, A);
  } else if (A.plan.n_slices > 1) {
    const int nb = (A.n_act + kWG - 1) / kWG;
    hipLaunchKernelGGL((k_force_reduce<V, NEWTON>), dim3(nb), dim3(kWG), 0, st, A);
  }
  return hipGetLastError();
}

template <class V, int NEWTON>
hipError_t run_scalar(ForceArgs &A, hipStream_t st) {
  if (!A.s64) {
    A.s32 = A.p32;
    A.s64 = A.p64;
    A.snpad = A.npad;
    A.self = 1;
  }
  A.n_jtiles = static_cast<int>(A.snpad / A.chunk);
  A.plan = plan_split(A.n_act, 1, A.n_jtiles, A.blocks);
  const dim3 grid(A.plan.nblk), block(kWG);
  if (A.chunk == kChunkSmall) {
    if (A.pot)
      hipLaunchKernelGGL((k_force_scalar<V, NEWTON, 1, kChunkSmall>), grid, block, 0, st, A);
    else
      hipLaunchKernelGGL((k_force_scalar<V, NEWTON, 0, kChunkSmall>), grid, block, 0, st, A);
  } else {
    if (A.pot)
      hipLaunchKernelGGL((k_force_scalar<V, NEWTON, 1, kTJ>), grid, block, 0, st, A);
    else
      hipLaunchKernelGGL((k_force_scalar<V, NEWTON, 0, kTJ>), grid, block, 0, st, A);
  }
  return launch_reduce<V, NEWTON>(A, st);
}

template <class V, int NEWTON, int IPL>
hipError_t run(ForceArgs &A, hipStream_t st) {
  A.plan = plan_split(A.n_act, IPL, A.n_jtiles, A.blocks);
  if (A.pot)
    hipLaunchKernelGGL((k_force<V, NEWTON, 1, IPL>), dim3(A.plan.nblk), dim3(kWG), 0, st, A);
  else
    hipLaunchKernelGGL((k_force<V, NEWTON, 0, IPL>), dim3(A.plan.nblk), dim3(kWG), 0, st, A);
  return launch_reduce<V, NEWTON>(A, st);
}

template <class V, int NEWTON>
hipError_t run_small(ForceArgs &A, hipStream_t st, const PredictArgs *pred = nullptr,
                     const InlineIdx *in = nullptr) {
  A.plan.n_itiles = 1;
  A.plan.n_slices = A.n_jtiles;
  A.plan.tiles_per_slice = 1;
  A.plan.nblk = A.n_jtiles;
  A.fuse_reduce = fuse_small_reduce(A.plan.n_slices, 4 * A.n_act) ? 1 : 0;
  if (pred) {
    InlineIdx none;
    none.out = nullptr;
    none.k = 0;
    hipLaunchKernelGGL((k_force_small_pred<V, NEWTON>), dim3(A.n_jtiles), dim3(kWG), 0, st, A,
                       *pred, in ? *in : none);
  }
  else
    hipLaunchKernelGGL((k_force_small<V, NEWTON>), dim3(A.n_jtiles), dim3(kWG), 0, st, A);
  if (!A.fuse_reduce) return launch_reduce<V, NEWTON>(A, st);
  return hipGetLastError();
}

template <class V, int NEWTON>
hipError_t pick_ipl(ForceArgs &A, hipStream_t st) {
  // the float64 j-parallel kernel pays four float64 wave reductions per target, which
  // beyond 16 targets cost more than the target-parallel kernel saves
  const int small = std::is_same<V, Fp64>::value ? kSmallActFp64 : kSmallAct;
  if (A.n_act <= small) return run_small<V, NEWTON>(A, st);
  if (A.scalar_j) return run_scalar<V, NEWTON>(A, st);
  if (A.ipl == 4) return run<V, NEWTON, 4>(A, st);
  if (A.ipl == 2) return run<V, NEWTON, 2>(A, st);
  return run<V, NEWTON, 1>(A, st);
}

}  // namespace

SplitPlan plan_split(int64_t n_targets, int ipl, int64_t n_jtiles, int target_blocks) {
  SplitPlan p;
  p.n_itiles = static_cast<int>((n_targets + ipl * kWG - 1) / (ipl * kWG));
  int64_t s = (target_blocks + p.n_itiles - 1) / p.n_itiles;
  if (s < 1) s = 1;
  if (s > n_jtiles) s = n_jtiles;
  p.tiles_per_slice = static_cast<int>((n_jtiles + s - 1) / s);
  p.n_slices = static_cast<int>((n_jtiles + p.tiles_per_slice - 1) / p.tiles_per_slice);
  p.nblk = static_cast<int>(round_up(static_cast<int64_t>(p.n_itiles) * p.n_slices, 8));
  return p;
}

int64_t force_partial_elems(const tsbts_ctx *c, int n_act, int blocks) {
  // small sets: one partial per j-tile and target
  if (n_act <= small_act_limit(c)) return c->npad / kTJ * 4 * n_act;
  const SplitPlan pf =
      force_scalar_j(c)
          ? plan_split(n_act, 1, c->npad / scalar_chunk(c, n_act, 1), blocks)
          : plan_split(n_act, force_targets_per_lane(c, n_act), c->npad / kTJ, blocks);
  return pf.n_slices > 1 ? static_cast<int64_t>(pf.n_slices) * 4 * n_act : 0;
}

int64_t partial_elems_needed(const tsbts_ctx *c, int n_act) {
  const int64_t n_jtiles = c->npad / kTJ;
  const int64_t need_f = force_partial_elems(c, n_act, c->tune_blocks);
  // the criterion: small sets one partial per j-tile with 2 values per target
  if (n_act <= kSmallAct) return std::max(need_f, n_jtiles * 2 * n_act);
  const int ipl_c = criterion_targets_per_lane(c, n_act);
  const int64_t units_c =
      criterion_scalar_j(c, n_act) ? c->npad / scalar_chunk(c, n_act, ipl_c) : n_jtiles;
  const SplitPlan pc = plan_split(n_act, ipl_c, units_c, criterion_blocks(c, n_act));
  const int64_t need_c = pc.n_slices > 1 ? static_cast<int64_t>(pc.n_slices) * 2 * n_act : 0;
  return std::max(need_f, need_c);
}

hipError_t launch_force_gather(tsbts_ctx *c, const int32_t *idx, int n_act, double *acc,
                               double *pot, double *part, int blocks, hipStream_t st,
                               const CorrectArgs *corr, const GatherSrc *src) {
  ForceArgs A;
  A.crit.on = 0;
  A.correct = corr ? 1 : 0;
  if (corr) A.corr = *corr;
  A.p32 = c->p32;
  A.p64 = c->p64;
  A.npad = c->npad;
  A.idx = idx;
  A.n_act = n_act;
  A.n_jtiles = static_cast<int>(c->npad / kTJ);
  A.eps2f = static_cast<float>(c->eps * c->eps);
  A.eps2 = c->eps * c->eps;
  A.part = part;
  A.acc = acc;
  A.pot = pot;
  A.blocks = blocks;
  A.ipl = force_targets_per_lane(c, n_act);
  A.scalar_j = force_scalar_j(c) ? 1 : 0;
  A.chunk = scalar_chunk(c, n_act, 1);
  A.done = c->done;
  A.fuse_reduce = 0;
  if (src) {
    // the scalar-load kernel over the given sources (more targets than the small-set
    // kernels take: split calls only)
    if (n_act <= small_act_limit(c)) return hipErrorInvalidValue;
    A.s32 = src->p32;
    A.s64 = src->p64;
    A.snpad = src->npad;
    A.self = 0;
    A.add = src->add;
    A.scalar_j = 1;
    A.chunk = scalar_chunk(c, n_act, 1);
  }
  if (c->precision == TSBTS_FP64) return pick_ipl<Fp64, 0>(A, st);
  const bool sep64 = (c->flags & TSBTS_FLAG_HILO_SEPARATION) == 0;
  const bool newton = (c->flags & TSBTS_FLAG_NEWTON) != 0;
  if (sep64) return newton ? pick_ipl<MixSep64, 1>(A, st) : pick_ipl<MixSep64, 0>(A, st);
  return newton ? pick_ipl<MixHiLo, 1>(A, st) : pick_ipl<MixHiLo, 0>(A, st);
}

hipError_t launch_force(tsbts_ctx *c, const int32_t *idx, int n_act, double *acc,
                        double *pot, hipStream_t st, const CorrectArgs *corr) {
  // automatic split calls only without the potential: the symmetric kernel's potential
  // form (half the columns per transposition) costs what the split saves
  if (split_applies(c, n_act) && (!pot || c->tune_split == 1)) {
    const hipError_t e = launch_force_split(c, idx, n_act, acc, pot, st, corr);
    if (e != hipErrorNotReady) return e;
  }
  if (force_sym_applies(c, n_act)) {
    SymPlan plan;
    if (sym_plan(c, 4, 8, c->precision == TSBTS_FP64 ? 8 : 4, &plan))
      return launch_force_sym(c, plan, idx, n_act, acc, pot, st, corr);
  }
  return launch_force_gather(c, idx, n_act, acc, pot, c->part, c->tune_blocks, st, corr);
}

int small_act_limit(const tsbts_ctx *c) {
  return c->precision == TSBTS_FP64 ? kSmallActFp64 : kSmallAct;
}

bool small_criterion_fused(const tsbts_ctx *c, int n_act) {
  const int64_t tiles = c->npad / kTJ;
  const int groups = (n_act + kCritGroup - 1) / kCritGroup;
  return n_act <= small_act_limit(c) && fuse_small_reduce(static_cast<int>(tiles), 4 * n_act) &&
         tiles * groups <= kCritFuseTiles;
}

hipError_t launch_force_predicted(tsbts_ctx *c, const int32_t *idx, int n_act, double t_block,
                                  int use_history, double *acc, double *pot, hipStream_t st,
                                  const CorrectArgs *corr, const PendingSteps *pend,
                                  const InlineIdx *in, double eta, double *dtc) {
  ForceArgs A;
  A.crit.on = 0;
  if (dtc && corr && small_criterion_fused(c, n_act)) {
    A.crit.on = 1;
    A.crit.n = c->n;
    A.crit.p32 = c->p32;
    A.crit.p64 = c->p64;
    A.crit.v64 = c->v64;
    A.crit.npad = c->npad;
    A.crit.eps2 = c->eps * c->eps;
    A.crit.eta = eta;
    A.crit.dtc = dtc;
  }
  A.correct = corr ? 1 : 0;
  if (corr) A.corr = *corr;
  A.p32 = c->p32;
  A.p64 = c->p64;
  A.npad = c->npad;
  A.idx = idx;
  A.n_act = n_act;
  A.n_jtiles = static_cast<int>(c->npad / kTJ);
  A.eps2f = static_cast<float>(c->eps * c->eps);
  A.eps2 = c->eps * c->eps;
  A.part = c->part;
  A.acc = acc;
  A.pot = pot;
  A.blocks = c->tune_blocks;
  A.ipl = 1;
  A.scalar_j = 0;
  A.chunk = kTJ;
  A.done = c->done;
  A.fuse_reduce = 0;
  PredictArgs P = predict_args(c, t_block, use_history);
  set_pending(P, pend);
  if (c->precision == TSBTS_FP64) return run_small<Fp64, 0>(A, st, &P, in);
  const bool sep64 = (c->flags & TSBTS_FLAG_HILO_SEPARATION) == 0;
  const bool newton = (c->flags & TSBTS_FLAG_NEWTON) != 0;
  if (sep64)
    return newton ? run_small<MixSep64, 1>(A, st, &P, in) : run_small<MixSep64, 0>(A, st, &P, in);
  return newton ? run_small<MixHiLo, 1>(A, st, &P, in) : run_small<MixHiLo, 0>(A, st, &P, in);
}

}  // namespace tsbts
