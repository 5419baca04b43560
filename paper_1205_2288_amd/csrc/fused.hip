// Force, potential and time-step criterion of the active set in one pass over the pairs.
//
// A variant of Algorithm 2's order: the paper evaluates the criterion (Eq. nbdt) after the
// corrector (step 7 after step 6), with the corrected velocities of the active particles;
// here it is evaluated with the state the force sees, i.e. the predicted velocities
// v + a h of the active particles.  Positions are the same either way (the corrector sets
// r to the prediction), so the free-fall term is unchanged and the collision term differs
// only through (a_new - a) h / 2 in the active velocities, O(h^2) relative.  In exchange
// the pair's separation, loads and loop are shared by the two sums.
//
// Same scalar-load structure as k_force_scalar (one target per lane, j-particles through
// wave-uniform loads in units of CH, self / padding masked by a wave vote), with the force
// and criterion pair arithmetic of the two separate kernels, so that the force is bitwise
// the one k_force_scalar returns for the same split.  Partials [S][6][n_act]: the force and
// potential sums, max v^2/r^2 and min s m^(-2/3).
#include "correct.hpp"
#include "criterion.hpp"
#include "force_pair.hpp"

namespace tsbts {
namespace {

struct FusedArgs {
  int64_t n, npad;
  const float *p32;
  const double *p64;
  const double *v64;
  const int32_t *idx;
  int n_act;
  SplitPlan plan;
  int n_units;  // j-units of CH particles
  float eps2f;
  double eps2;
  double eta;
  double *part;  // [S][6][n_act]
  double *acc;   // [3][n_act]
  double *pot;   // [n_act] or null
  double *dtc;   // [n_act]
  int correct;   // apply the corrector in the reduction
  CorrectArgs corr;
};

template <class V, int NEWTON>
__device__ __forceinline__ void finish_all(const FusedArgs &A, int q, int64_t g, double sx,
                                           double sy, double sz, double sp, double qm,
                                           double sm) {
  const double k = Scale<V, NEWTON>::kAcc;
  const double an[3] = {k * sx, k * sy, k * sz};
  A.acc[q] = an[0];
  A.acc[A.n_act + q] = an[1];
  A.acc[2 * A.n_act + q] = an[2];
  if (A.pot) A.pot[q] = -sp;
  A.dtc[q] = finish_dt(A.eta, qm, sm);
  if (A.correct) correct_one(A.corr, q, g, an);
}

template <class V, int NEWTON, int MASK, int POT, int CH, class F>
__device__ __forceinline__ void fused_unit(const FusedArgs &A, const typename V::I &If,
                                           const typename StepRec<V>::I &Ic, int g,
                                           int64_t jbase, F eps2, F &fx, F &fy, F &fz, F &fp,
                                           F &qm, F &sm) {
#pragma unroll 4
  for (int jj = 0; jj < CH; ++jj) {
    const int64_t j = jbase + jj;
    const typename V::J Jf = V::load_j(A.p32, A.p64, A.npad, j, Scale<V, NEWTON>::kMass);
    const typename StepRec<V>::J Jc = load_jv<V>(A, j);
    const bool skip = MASK && (j == g || j >= A.n);
    pair_acc<V, NEWTON, MASK, POT>(If, Jf, eps2, skip, fx, fy, fz, fp);
    pair_step(Ic, Jc, eps2, skip, qm, sm);
  }
}

template <class V, int NEWTON, int POT, int CH>
__global__ __launch_bounds__(kWG) void k_fused(FusedArgs A) {
  using F = typename V::F;
  int itile, slice;
  split_tile(blockIdx.x, A.plan, itile, slice);
  if (slice >= A.plan.n_slices) return;
  const int jt0 = slice * A.plan.tiles_per_slice;
  const int jt1 = min(jt0 + A.plan.tiles_per_slice, A.n_units);
  const F eps2 = sizeof(F) == 4 ? static_cast<F>(A.eps2f) : static_cast<F>(A.eps2);
  const int q = itile * kWG + static_cast<int>(threadIdx.x);
  const int g = A.idx[min(q, A.n_act - 1)];
  const typename V::I If = V::load_i(A.p32, A.p64, A.npad, g);
  const typename StepRec<V>::I Ic = load_iv<V>(A, g);
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
  F qm = F(0);
  F sm = sizeof(F) == 4 ? static_cast<F>(__builtin_inff()) : static_cast<F>(__builtin_inf());
  for (int jt = jt0; jt < jt1; ++jt) {
    const int64_t jbase = static_cast<int64_t>(jt) * CH;
    F fx = F(0), fy = F(0), fz = F(0), fp = F(0);
    if (__ballot(g >= jbase && g < jbase + CH) != 0 || jbase + CH > A.n)
      fused_unit<V, NEWTON, 1, POT, CH>(A, If, Ic, g, jbase, eps2, fx, fy, fz, fp, qm, sm);
    else
      fused_unit<V, NEWTON, 0, POT, CH>(A, If, Ic, g, jbase, eps2, fx, fy, fz, fp, qm, sm);
    sx += static_cast<double>(fx);
    sy += static_cast<double>(fy);
    sz += static_cast<double>(fz);
    sp += static_cast<double>(fp);
  }
  if (q >= A.n_act) return;
  double *out = A.part + static_cast<int64_t>(slice) * 6 * A.n_act;
  out[q] = sx;
  out[A.n_act + q] = sy;
  out[2 * A.n_act + q] = sz;
  out[3 * A.n_act + q] = sp;
  out[4 * A.n_act + q] = static_cast<double>(qm);
  out[5 * A.n_act + q] = static_cast<double>(sm);
}

// Combine the slices in slice order (sums; max and min are exact) and finish: one thread
// per target, one wave per target with the lanes striding over many slices, or (below)
// rows of 64 targets, in the force reduction's order for the same call.  Always a
// separate launch: the corrector it may apply rewrites velocity planes the pair loop reads.
template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_fused_reduce(FusedArgs A) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q >= A.n_act) return;
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0, qm = 0.0, sm = __builtin_inf();
  const int64_t stride = 6 * static_cast<int64_t>(A.n_act);
  for (int s = 0; s < A.plan.n_slices; ++s) {
    const double *in = A.part + s * stride;
    sx += in[q];
    sy += in[A.n_act + q];
    sz += in[2 * A.n_act + q];
    sp += in[3 * A.n_act + q];
    qm = fmax(qm, in[4 * A.n_act + q]);
    sm = fmin(sm, in[5 * A.n_act + q]);
  }
  finish_all<V, NEWTON>(A, q, A.idx[q], sx, sy, sz, sp, qm, sm);
}

template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_fused_reduce_wave(FusedArgs A) {
  const int q = blockIdx.x * (kWG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= A.n_act) return;
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0, qm = 0.0, sm = __builtin_inf();
  const int64_t stride = 6 * static_cast<int64_t>(A.n_act);
  for (int s = lane; s < A.plan.n_slices; s += 64) {
    const double *in = A.part + s * stride;
    sx += in[q];
    sy += in[A.n_act + q];
    sz += in[2 * A.n_act + q];
    sp += in[3 * A.n_act + q];
    qm = fmax(qm, in[4 * A.n_act + q]);
    sm = fmin(sm, in[5 * A.n_act + q]);
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  sp = wave_sum(sp);
  qm = wave_max(qm);
  sm = wave_min(sm);
  if (lane == 0) finish_all<V, NEWTON>(A, q, A.idx[q], sx, sy, sz, sp, qm, sm);
}

// Same, a workgroup per 64 consecutive targets whose kRowsWaves waves each combine a
// contiguous range of the slices in order, then the waves in order: the association of
// the force's k_force_reduce_rows, so the results stay those of the separate kernels.
template <class V, int NEWTON>
__global__ __launch_bounds__(64 * kRowsWaves) void k_fused_reduce_rows(FusedArgs A) {
  __shared__ double sums[kRowsWaves][6][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = blockIdx.x * 64 + lane;
  const int S = A.plan.n_slices;
  const int L = (S + kRowsWaves - 1) / kRowsWaves;
  const int s1 = min(S, (w + 1) * L);
  double t[6] = {0.0, 0.0, 0.0, 0.0, 0.0, __builtin_inf()};
  if (q < A.n_act) {
    const int64_t stride = 6 * static_cast<int64_t>(A.n_act);
#pragma unroll 4
    for (int s = w * L; s < s1; ++s) {
      const double *in = A.part + s * stride;
#pragma unroll
      for (int c = 0; c < 4; ++c) t[c] += in[c * A.n_act + q];
      t[4] = fmax(t[4], in[4 * A.n_act + q]);
      t[5] = fmin(t[5], in[5 * A.n_act + q]);
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) sums[w][c][lane] = t[c];
  __syncthreads();
  if (w == 0 && q < A.n_act) {
    double f[6] = {0.0, 0.0, 0.0, 0.0, 0.0, __builtin_inf()};
    for (int ww = 0; ww < kRowsWaves; ++ww) {
#pragma unroll
      for (int c = 0; c < 4; ++c) f[c] += sums[ww][c][lane];
      f[4] = fmax(f[4], sums[ww][4][lane]);
      f[5] = fmin(f[5], sums[ww][5][lane]);
    }
    finish_all<V, NEWTON>(A, q, A.idx[q], f[0], f[1], f[2], f[3], f[4], f[5]);
  }
}

template <class V, int NEWTON, int CH>
void launch_main(FusedArgs &A, hipStream_t st) {
  const dim3 grid(A.plan.nblk), block(kWG);
  if (A.pot)
    hipLaunchKernelGGL((k_fused<V, NEWTON, 1, CH>), grid, block, 0, st, A);
  else
    hipLaunchKernelGGL((k_fused<V, NEWTON, 0, CH>), grid, block, 0, st, A);
}

template <class V, int NEWTON>
hipError_t run(FusedArgs &A, int chunk, hipStream_t st) {
  if (chunk == kChunkSmall)
    launch_main<V, NEWTON, kChunkSmall>(A, st);
  else
    launch_main<V, NEWTON, kTJ>(A, st);
  if (use_rows_reduce(A.plan.n_slices, A.n_act)) {
    const int nb = (A.n_act + 63) / 64;
    hipLaunchKernelGGL((k_fused_reduce_rows<V, NEWTON>), dim3(nb), dim3(64 * kRowsWaves), 0, st,
                       A);
  } else if (use_wave_reduce(A.plan.n_slices, A.n_act)) {
    const int nb = (A.n_act + kWG / 64 - 1) / (kWG / 64);
    hipLaunchKernelGGL((k_fused_reduce_wave<V, NEWTON>), dim3(nb), dim3(kWG), 0, st, A);
  } else {
    const int nb = (A.n_act + kWG - 1) / kWG;
    hipLaunchKernelGGL((k_fused_reduce<V, NEWTON>), dim3(nb), dim3(kWG), 0, st, A);
  }
  return hipGetLastError();
}

}  // namespace

int64_t fused_partials_needed(const tsbts_ctx *c, int n_act) {
  const SplitPlan p =
      plan_split(n_act, 1, c->npad / scalar_chunk(c, n_act, 1), c->tune_blocks);
  return static_cast<int64_t>(p.n_slices) * 6 * n_act;
}

hipError_t launch_fused(tsbts_ctx *c, const int32_t *idx, int n_act, double eta, double *acc,
                        double *pot, double *dtc, hipStream_t st, const CorrectArgs *corr) {
  FusedArgs A;
  A.n = c->n;
  A.npad = c->npad;
  A.p32 = c->p32;
  A.p64 = c->p64;
  A.v64 = c->v64;
  A.idx = idx;
  A.n_act = n_act;
  const int chunk = scalar_chunk(c, n_act, 1);
  A.n_units = static_cast<int>(c->npad / chunk);
  A.plan = plan_split(n_act, 1, A.n_units, c->tune_blocks);
  A.eps2f = static_cast<float>(c->eps * c->eps);
  A.eps2 = c->eps * c->eps;
  A.eta = eta;
  A.part = c->part;
  A.acc = acc;
  A.pot = pot;
  A.dtc = dtc;
  A.correct = corr ? 1 : 0;
  if (corr) A.corr = *corr;
  if (c->precision == TSBTS_FP64) return run<Fp64, 0>(A, chunk, st);
  const bool sep64 = (c->flags & TSBTS_FLAG_HILO_SEPARATION) == 0;
  const bool newton = (c->flags & TSBTS_FLAG_NEWTON) != 0;
  if (sep64) return newton ? run<MixSep64, 1>(A, chunk, st) : run<MixSep64, 0>(A, chunk, st);
  return newton ? run<MixHiLo, 1>(A, chunk, st) : run<MixHiLo, 0>(A, chunk, st);
}

}  // namespace tsbts
