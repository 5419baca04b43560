// Time-step criterion, Eq. (nbdt) of Section 2, for the active particles:
//   dtc_i = eta * min_{j != i} min(|r_ij| / |v_ij|, sqrt(|r_ij| / |a_ij|)),
//   |a_ij| = m_j |r_ij| / s^(3/2),  s = |r_ij|^2 + eps^2,
// so the free-fall term is s^(3/4) m_j^(-1/2) = (s m_j^(-2/3))^(3/4).
// Per pair the kernel keeps max(|v_ij|^2 / |r_ij|^2) and min(s * m_j^(-2/3)); the square
// root and the 3/4 power are taken once per target.  No transcendental per pair in
// float64 mode apart from the division; mixed mode uses the float32 reciprocal.
// Same tiling and split-j scheme as the force kernel; the self pair is masked by index
// in the tiles that hold some lane's own particle (wave-uniform vote), as in the force,
// and so are the padding particles of the last tile (at rest far away they would add a
// tiny nonzero v^2/r^2, which matters when every real relative velocity is zero).
#include "criterion.hpp"
#include "sym.hpp"

namespace tsbts {
namespace {

struct StepArgs {
  int64_t n;  // particles; j >= n are padding, excluded like the self pair
  const float *p32;
  const double *p64;
  const double *v64;
  int64_t npad;
  const int32_t *idx;
  int n_act;
  SplitPlan plan;
  int n_jtiles;
  double eps2;
  double eta;
  double *part;  // [S][2][n_act]: max q, min s*w
  double *dtc;
  int blocks;
  int ipl;
  int scalar_j;  // j-particles through scalar loads (k_timestep_scalar)
  int chunk;     // j-particles per split unit of k_timestep_scalar
  uint32_t *done;   // finished-workgroup count of k_timestep_small
  int fuse_reduce;  // its last workgroup reduces the partials
  // Sources of k_timestep_scalar (null s64: the predicted arrays above): sn particles,
  // planes of stride snpad; self = 0 when they exclude the targets.
  const float *s32 = nullptr;
  const double *s64 = nullptr, *sv64 = nullptr;
  int64_t snpad = 0, sn = 0;
  int self = 1;
  // null, or [2][n_act]: the other part of a split call's maximum of q and minimum of s*w
  // for each target, combined where it is finished
  const double *add = nullptr;
};

// The source planes of k_timestep_scalar (load_jv reads these fields).
struct SrcPlanes {
  const float *p32;
  const double *p64, *v64;
  int64_t npad;
};

// Finish target q from its maximum of q and minimum of s*w.
__device__ __forceinline__ void finish_target(const StepArgs &A, int q, double qm, double sm) {
  if (A.add) {
    qm = fmax(qm, A.add[q]);
    sm = fmin(sm, A.add[A.n_act + q]);
  }
  A.dtc[q] = finish_dt(A.eta, qm, sm);
}

template <class V, int MASK, int IPL, class J, class I, class F>
__device__ __forceinline__ void step_tile(const J *sj, const I *Ir, const int *g, int64_t jbase,
                                          int64_t n, F eps2, F *qmax, F *swmin) {
#pragma unroll 2
  for (int jj = 0; jj < kTJ; ++jj) {
    const J Jr = sj[jj];
#pragma unroll
    for (int k = 0; k < IPL; ++k)
      pair_step(Ir[k], Jr, eps2, MASK && (jbase + jj == g[k] || jbase + jj >= n), qmax[k],
                swmin[k]);
  }
}

template <class V, int IPL>
__global__ __launch_bounds__(kWG) void k_timestep(StepArgs A) {
  using F = typename V::F;
  using J = typename StepRec<V>::J;
  __shared__ J sj[kTJ];
  const int tid = threadIdx.x;
  int itile, slice;
  split_tile(blockIdx.x, A.plan, itile, slice);
  if (slice >= A.plan.n_slices) return;
  const int jt0 = slice * A.plan.tiles_per_slice;
  const int jt1 = min(jt0 + A.plan.tiles_per_slice, A.n_jtiles);
  const F eps2 = static_cast<F>(A.eps2);

  typename StepRec<V>::I I[IPL];
  int q[IPL], g[IPL];
  F qmax[IPL], swmin[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    q[k] = (itile * IPL + k) * kWG + tid;
    g[k] = A.idx[min(q[k], A.n_act - 1)];
    I[k] = load_iv<V>(A, g[k]);
    qmax[k] = F(0);
    swmin[k] = sizeof(F) == 4 ? static_cast<F>(__builtin_inff()) : static_cast<F>(__builtin_inf());
  }
  for (int jt = jt0; jt < jt1; ++jt) {
    const int64_t jbase = static_cast<int64_t>(jt) * kTJ;
    const J rec = load_jv<V>(A, jbase + tid);
    __syncthreads();
    sj[tid] = rec;
    __syncthreads();
    bool mine = false;
#pragma unroll
    for (int k = 0; k < IPL; ++k) mine |= (g[k] >= jbase && g[k] < jbase + kTJ);
    if (__ballot(mine) != 0 || jbase + kTJ > A.n)
      step_tile<V, 1, IPL>(sj, I, g, jbase, A.n, eps2, qmax, swmin);
    else
      step_tile<V, 0, IPL>(sj, I, g, jbase, A.n, eps2, qmax, swmin);
  }
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    if (q[k] >= A.n_act) continue;
    if (A.plan.n_slices == 1) {
      A.dtc[q[k]] = finish_dt(A.eta, qmax[k], swmin[k]);
    } else {
      double *out = A.part + static_cast<int64_t>(slice) * 2 * A.n_act;
      out[q[k]] = qmax[k];
      out[A.n_act + q[k]] = swmin[k];
    }
  }
}

// j-particles through scalar loads (wave-uniform j index): the j record comes straight
// from the predicted planes into SGPRs, no LDS staging and no barriers.  Same tiles, vote
// and partials as k_timestep.
template <class V, int MASK, int IPL, int CH, class I, class F>
__device__ __forceinline__ void scalar_step_tile(const SrcPlanes &S, int64_t sn, const I *Ir,
                                                 const int *g, int64_t jbase, F eps2, F *qmax,
                                                 F *swmin) {
#pragma unroll 4
  for (int jj = 0; jj < CH; ++jj) {
    const typename StepRec<V>::J Jr = load_jv<V>(S, jbase + jj);
#pragma unroll
    for (int k = 0; k < IPL; ++k)
      pair_step(Ir[k], Jr, eps2, MASK && (jbase + jj == g[k] || jbase + jj >= sn), qmax[k],
                swmin[k]);
  }
}

// Split units of CH j-particles (A.n_jtiles counts them here).
template <class V, int IPL, int CH>
__global__ __launch_bounds__(kWG) void k_timestep_scalar(StepArgs A) {
  using F = typename V::F;
  const int tid = threadIdx.x;
  int itile, slice;
  split_tile(blockIdx.x, A.plan, itile, slice);
  if (slice >= A.plan.n_slices) return;
  const int jt0 = slice * A.plan.tiles_per_slice;
  const int jt1 = min(jt0 + A.plan.tiles_per_slice, A.n_jtiles);
  const F eps2 = static_cast<F>(A.eps2);
  typename StepRec<V>::I I[IPL];
  int q[IPL], g[IPL];
  F qmax[IPL], swmin[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    q[k] = (itile * IPL + k) * kWG + tid;
    const int t = A.idx[min(q[k], A.n_act - 1)];
    I[k] = load_iv<V>(A, t);
    g[k] = A.self ? t : -1;  // the target's index among the sources
    qmax[k] = F(0);
    swmin[k] = sizeof(F) == 4 ? static_cast<F>(__builtin_inff()) : static_cast<F>(__builtin_inf());
  }
  const SrcPlanes S{A.s32, A.s64, A.sv64, A.snpad};
  for (int jt = jt0; jt < jt1; ++jt) {
    const int64_t jbase = static_cast<int64_t>(jt) * CH;
    bool mine = false;
#pragma unroll
    for (int k = 0; k < IPL; ++k) mine |= (g[k] >= jbase && g[k] < jbase + CH);
    if (__ballot(mine) != 0 || jbase + CH > A.sn)
      scalar_step_tile<V, 1, IPL, CH>(S, A.sn, I, g, jbase, eps2, qmax, swmin);
    else
      scalar_step_tile<V, 0, IPL, CH>(S, A.sn, I, g, jbase, eps2, qmax, swmin);
  }
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    if (q[k] >= A.n_act) continue;
    if (A.plan.n_slices == 1) {
      finish_target(A, q[k], qmax[k], swmin[k]);
    } else {
      double *out = A.part + static_cast<int64_t>(slice) * 2 * A.n_act;
      out[q[k]] = qmax[k];
      out[A.n_act + q[k]] = swmin[k];
    }
  }
}

// Small active sets: one j-tile per workgroup, one source per lane, targets from LDS.  The
// maxima of kStepGroup targets and their negated minima are combined over the wave
// together (wave_reduce_many with max), then over the 4 waves, into one partial per tile
// and target.  When the partials are few (fuse_reduce) the launch's last workgroup
// combines them and finishes the targets; max and min are exact, so the order of either
// combination leaves the results unchanged.
constexpr int kStepGroup = 16;

template <class V>
__global__ __launch_bounds__(kWG) void k_timestep_small(StepArgs A) {
  using F = typename V::F;
  __shared__ typename StepRec<V>::I si[kSmallAct];
  __shared__ int sg[kSmallAct];
  __shared__ F red[kSmallAct][2][kWG / 64];
  __shared__ double sums[kWG];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int tile = blockIdx.x;
  const int64_t j = static_cast<int64_t>(tile) * kTJ + tid;
  const F eps2 = static_cast<F>(A.eps2);
  const typename StepRec<V>::J J = load_jv<V>(A, j);
  if (tid < A.n_act) {
    sg[tid] = A.idx[tid];
    si[tid] = load_iv<V>(A, sg[tid]);
  }
  __syncthreads();
  for (int q0 = 0; q0 < A.n_act; q0 += kStepGroup) {
    F x[2 * kStepGroup];
#pragma unroll
    for (int u = 0; u < kStepGroup; ++u) {
      const int q = q0 + u;
      F qm = F(0);
      F sm = sizeof(F) == 4 ? static_cast<F>(__builtin_inff()) : static_cast<F>(__builtin_inf());
      if (q < A.n_act) pair_step(si[q], J, eps2, j == sg[q] || j >= A.n, qm, sm);
      x[u] = qm;
      x[kStepGroup + u] = -sm;
    }
    const F r = wave_reduce_many<2 * kStepGroup>(x, lane, [](F a, F b) { return fmax(a, b); });
    // lane l holds value v = l >> 1: the maximum of target q0 + v (v < kStepGroup), else
    // the negated minimum of target q0 + v - kStepGroup
    const int v = lane >> 1;
    const int q = q0 + (v & (kStepGroup - 1));
    if ((lane & 1) == 0 && q < A.n_act) {
      if (v < kStepGroup)
        red[q][0][w] = r;
      else
        red[q][1][w] = -r;
    }
  }
  __syncthreads();
  for (int t = tid; t < 2 * A.n_act; t += kWG) {
    const int q = t >> 1, c = t & 1;
    double s = static_cast<double>(red[q][c][0]);
#pragma unroll
    for (int ww = 1; ww < kWG / 64; ++ww)
      s = c == 0 ? fmax(s, static_cast<double>(red[q][c][ww]))
                 : fmin(s, static_cast<double>(red[q][c][ww]));
    A.part[(static_cast<int64_t>(tile) * 2 + c) * A.n_act + q] = s;
  }
  if (!A.fuse_reduce || !last_workgroup(A.done)) return;
  // the launch's last workgroup: a slice's partials form a row of W = 2 n_act values (the
  // maxima, then the minima); thread t combines value t % W over part t / W of the slices
  const int W = 2 * A.n_act, P = kWG / W, S = A.plan.n_slices;
  const int L = (S + P - 1) / P;
  const int p = tid / W, vv = tid - p * W;
  const bool is_max = vv < A.n_act;
  double acc = is_max ? 0.0 : __builtin_inf();
  if (p < P) {
    const int s1 = min(S, (p + 1) * L);
#pragma unroll 8
    for (int sl = p * L; sl < s1; ++sl) {
      const double x = A.part[static_cast<int64_t>(sl) * W + vv];
      acc = is_max ? fmax(acc, x) : fmin(acc, x);
    }
  }
  sums[tid] = acc;
  __syncthreads();
  if (tid < A.n_act) {
    double qm = 0.0, sm = __builtin_inf();
    for (int pp = 0; pp < P; ++pp) {
      qm = fmax(qm, sums[pp * W + tid]);
      sm = fmin(sm, sums[pp * W + A.n_act + tid]);
    }
    A.dtc[tid] = finish_dt(A.eta, qm, sm);
  }
}

__global__ __launch_bounds__(kWG) void k_timestep_reduce(StepArgs A) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q >= A.n_act) return;
  double qm = 0.0, sm = __builtin_inf();
  for (int s = 0; s < A.plan.n_slices; ++s) {
    const double *in = A.part + static_cast<int64_t>(s) * 2 * A.n_act;
    qm = fmax(qm, in[q]);
    sm = fmin(sm, in[A.n_act + q]);
  }
  finish_target(A, q, qm, sm);
}

__global__ __launch_bounds__(kWG) void k_timestep_reduce_wave(StepArgs A) {
  const int q = blockIdx.x * (kWG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= A.n_act) return;
  double qm = 0.0, sm = __builtin_inf();
  for (int s = lane; s < A.plan.n_slices; s += 64) {
    const double *in = A.part + static_cast<int64_t>(s) * 2 * A.n_act;
    qm = fmax(qm, in[q]);
    sm = fmin(sm, in[A.n_act + q]);
  }
  qm = wave_max(qm);
  sm = wave_min(sm);
  if (lane == 0) finish_target(A, q, qm, sm);
}

// Same, a workgroup per 64 consecutive targets whose kRowsWaves waves each combine a
// contiguous range of the slices (many targets and slices; max and min are exact).
__global__ __launch_bounds__(64 * kRowsWaves) void k_timestep_reduce_rows(StepArgs A) {
  __shared__ double sums[kRowsWaves][2][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = blockIdx.x * 64 + lane;
  const int S = A.plan.n_slices;
  const int L = (S + kRowsWaves - 1) / kRowsWaves;
  const int s1 = min(S, (w + 1) * L);
  double qm = 0.0, sm = __builtin_inf();
  if (q < A.n_act) {
#pragma unroll 4
    for (int s = w * L; s < s1; ++s) {
      const double *in = A.part + static_cast<int64_t>(s) * 2 * A.n_act;
      qm = fmax(qm, in[q]);
      sm = fmin(sm, in[A.n_act + q]);
    }
  }
  sums[w][0][lane] = qm;
  sums[w][1][lane] = sm;
  __syncthreads();
  if (w == 0 && q < A.n_act) {
    for (int ww = 1; ww < kRowsWaves; ++ww) {
      qm = fmax(qm, sums[ww][0][lane]);
      sm = fmin(sm, sums[ww][1][lane]);
    }
    finish_target(A, q, qm, sm);
  }
}

template <class V>
hipError_t run(StepArgs &A, hipStream_t st) {
  if (A.n_act <= kSmallAct) {
    A.plan.n_itiles = 1;
    A.plan.n_slices = A.n_jtiles;
    A.plan.tiles_per_slice = 1;
    A.plan.nblk = A.n_jtiles;
    A.fuse_reduce = fuse_small_reduce(A.plan.n_slices, 2 * A.n_act) ? 1 : 0;
    hipLaunchKernelGGL((k_timestep_small<V>), dim3(A.n_jtiles), dim3(kWG), 0, st, A);
    if (A.fuse_reduce) return hipGetLastError();
  } else if (A.scalar_j) {
    if (!A.s64) {
      A.s32 = A.p32;
      A.s64 = A.p64;
      A.sv64 = A.v64;
      A.snpad = A.npad;
      A.sn = A.n;
      A.self = 1;
    }
    A.n_jtiles = static_cast<int>(A.snpad / A.chunk);
    A.plan = plan_split(A.n_act, A.ipl, A.n_jtiles, A.blocks);
    const dim3 grid(A.plan.nblk), block(kWG);
    if (A.ipl == 2 && A.chunk == kTJ)
      hipLaunchKernelGGL((k_timestep_scalar<V, 2, kTJ>), grid, block, 0, st, A);
    else if (A.ipl == 2)
      hipLaunchKernelGGL((k_timestep_scalar<V, 2, kChunkSmall>), grid, block, 0, st, A);
    else if (A.chunk == kTJ)
      hipLaunchKernelGGL((k_timestep_scalar<V, 1, kTJ>), grid, block, 0, st, A);
    else
      hipLaunchKernelGGL((k_timestep_scalar<V, 1, kChunkSmall>), grid, block, 0, st, A);
  } else {
    A.plan = plan_split(A.n_act, A.ipl, A.n_jtiles, A.blocks);
    if (A.ipl == 4)
      hipLaunchKernelGGL((k_timestep<V, 4>), dim3(A.plan.nblk), dim3(kWG), 0, st, A);
    else if (A.ipl == 2)
      hipLaunchKernelGGL((k_timestep<V, 2>), dim3(A.plan.nblk), dim3(kWG), 0, st, A);
    else
      hipLaunchKernelGGL((k_timestep<V, 1>), dim3(A.plan.nblk), dim3(kWG), 0, st, A);
  }
  if (use_rows_reduce(A.plan.n_slices, A.n_act)) {
    const int nb = (A.n_act + 63) / 64;
    hipLaunchKernelGGL(k_timestep_reduce_rows, dim3(nb), dim3(64 * kRowsWaves), 0, st, A);
  } else if (use_wave_reduce(A.plan.n_slices, A.n_act)) {
    const int nb = (A.n_act + kWG / 64 - 1) / (kWG / 64);
    hipLaunchKernelGGL(k_timestep_reduce_wave, dim3(nb), dim3(kWG), 0, st, A);
  } else if (A.plan.n_slices > 1) {
    const int nb = (A.n_act + kWG - 1) / kWG;
    hipLaunchKernelGGL(k_timestep_reduce, dim3(nb), dim3(kWG), 0, st, A);
  }
  return hipGetLastError();
}

}  // namespace

namespace {

// The gather kernels' arguments for the context's predicted arrays.
StepArgs gather_args(tsbts_ctx *c, const int32_t *idx, int n_act, double eta, double *dtc) {
  StepArgs A;
  A.n = c->n;
  A.p32 = c->p32;
  A.p64 = c->p64;
  A.v64 = c->v64;
  A.npad = c->npad;
  A.idx = idx;
  A.n_act = n_act;
  A.n_jtiles = static_cast<int>(c->npad / kTJ);
  A.eps2 = c->eps * c->eps;
  A.eta = eta;
  A.part = c->part;
  A.dtc = dtc;
  A.blocks = criterion_blocks(c, n_act);
  A.ipl = criterion_targets_per_lane(c, n_act);
  A.scalar_j = criterion_scalar_j(c, n_act) ? 1 : 0;
  A.chunk = scalar_chunk(c, n_act, A.ipl);
  A.done = c->done + 1;
  A.fuse_reduce = 0;
  return A;
}

hipError_t run_precision(const tsbts_ctx *c, StepArgs &A, hipStream_t st) {
  if (c->precision == TSBTS_FP64) return run<Fp64>(A, st);
  if (c->flags & TSBTS_FLAG_HILO_SEPARATION) return run<MixHiLo>(A, st);
  return run<MixSep64>(A, st);
}

}  // namespace

hipError_t launch_timestep(tsbts_ctx *c, const int32_t *idx, int n_act, double eta,
                           double *dtc, hipStream_t st) {
  if (split_applies(c, n_act)) {
    const hipError_t e = launch_timestep_split(c, idx, n_act, eta, dtc, st);
    if (e != hipErrorNotReady) return e;
  }
  if (criterion_sym_applies(c, n_act)) {
    SymPlan plan;
    const int vb = c->precision == TSBTS_FP64 ? 8 : 4;
    if (sym_plan(c, 2, vb, vb, &plan))
      return launch_timestep_sym(c, plan, idx, n_act, eta, dtc, st);
  }
  StepArgs A = gather_args(c, idx, n_act, eta, dtc);
  return run_precision(c, A, st);
}

hipError_t launch_timestep_gather(tsbts_ctx *c, const int32_t *idx, int n_act, double eta,
                                  double *dtc, hipStream_t st, const GatherSrc *src) {
  // the scalar-load kernel in the shape gather_args gives it from 8192 targets (two
  // targets per lane), whose partials partial_elems_needed provides for
  if (n_act < 8192 || !criterion_scalar_j(c, n_act)) return hipErrorInvalidValue;
  StepArgs A = gather_args(c, idx, n_act, eta, dtc);
  A.s32 = src->p32;
  A.s64 = src->p64;
  A.sv64 = src->v64;
  A.snpad = src->npad;
  A.sn = src->n;
  A.self = 0;
  A.add = src->add;
  A.scalar_j = 1;
  return run_precision(c, A, st);
}

}  // namespace tsbts
