// Time-step criterion (Eq. nbdt of Section 2) when every particle is a target: each
// unordered pair is evaluated once for both of its particles (symmetric all-targets
// scheme of sym.hpp).  The per-pair terms are the gather kernels' (pair_step_sym), and
// maxima and minima do not depend on the order in which they are taken, so the result
// equals the gather kernels' bit for bit.  Partials: [slot][2][rows] and [row group][2][n]
// of max v^2/r^2 and min s m^(-2/3) (the column minima stored negated), in the kernel's
// float type.
#include "criterion.hpp"
#include "sym.hpp"

namespace tsbts {
namespace {

struct StepSymArgs {
  int64_t n, npad;
  const float *p32;
  const double *p64;
  const double *v64;
  double eps2;
  SymPlan plan;
  const int32_t *idx;
  int n_act;
  double eta;
  double *dtc;
  double *raw;  // null, or [2][n_act]: max q and min s*w unfinished instead of dtc
};

// A row particle's weights in the column role (see pair_step_sym).
template <class V>
__device__ __forceinline__ void col_weights(const StepSymArgs &A, int64_t k,
                                            typename V::F &w, typename V::F &e) {
  if constexpr (sizeof(typename V::F) == 4) {
    w = A.p32[P32_W * A.npad + k];
    e = A.p32[P32_E * A.npad + k];
  } else {
    w = A.p64[P64_W * A.npad + k];
    e = 0.0;
  }
}

template <class F>
__device__ __forceinline__ F inf_of() {
  if constexpr (sizeof(F) == 4) return __builtin_inff();
  else return __builtin_inf();
}

// kSymBlock columns starting at jb against the lane's kSymRows rows; the column values of
// column jb + c go to L[(c * kSymLdsStride + lane) * 2 + {0, 1}].
template <class V, int MASK>
__device__ __forceinline__ void sym_block(const StepSymArgs &A,
                                          const typename StepRec<V>::I (&rows)[kSymRows],
                                          const typename V::F (&wr)[kSymRows],
                                          const typename V::F (&er)[kSymRows],
                                          const int (&k)[kSymRows], int64_t jb,
                                          typename V::F eps2, typename V::F (&qmax)[kSymRows],
                                          typename V::F (&swmin)[kSymRows], typename V::F *L,
                                          int lane) {
  using F = typename V::F;
  // unrolled so that the column records of consecutive columns merge into wide scalar loads
  // (float64 records by two: eight would not fit the scalar registers)
  constexpr int UNR = sizeof(F) == 4 ? 4 : 2;
#pragma unroll UNR
  for (int c = 0; c < kSymBlock; ++c) {
    const int64_t j = jb + c;
    const typename StepRec<V>::J Jr = load_jv<V>(A, j);
    F cq = F(0), cs = inf_of<F>();
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
      const bool skip = MASK && (j <= k[r] || j >= A.n || k[r] >= A.n);
      if constexpr (sizeof(F) == 4)
        pair_step_sym<V>(rows[r], wr[r], er[r], Jr, eps2, skip, qmax[r], swmin[r], cq, cs);
      else
        pair_step_sym(rows[r], wr[r], er[r], Jr, eps2, skip, qmax[r], swmin[r], cq, cs);
    }
    L[(c * kSymLdsStride + lane) * 2] = cq;
    L[(c * kSymLdsStride + lane) * 2 + 1] = cs;
  }
}

// The particle planes and the partials come as separate restrict-qualified arguments:
// with stores to the partials inside the column loop, only the no-alias guarantee lets the
// compiler keep the column records on scalar loads.
template <class V>
__global__ __launch_bounds__(kWG) void k_timestep_sym(StepSymArgs A0,
                                                      const float *__restrict__ p32,
                                                      const double *__restrict__ p64,
                                                      const double *__restrict__ v64,
                                                      typename V::F *__restrict__ col_part,
                                                      typename V::F *__restrict__ row_part) {
  using F = typename V::F;
  StepSymArgs A = A0;
  A.p32 = p32;
  A.p64 = p64;
  A.v64 = v64;
  __shared__ F lds[kWG / 64][kSymBlock * kSymLdsStride * 2];
  __shared__ F xs[2][kSymWaves][2][kSymBlock];
  // the wave index is uniform over the wave: say so, so that the row tile and the column
  // index are scalar and the column records arrive through scalar loads
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int4 it = A.plan.items[blockIdx.x];  // one work item per workgroup
  const F eps2 = static_cast<F>(A.eps2);
  F *L = lds[wv];
  F *colq = col_part + static_cast<int64_t>(it.x) * 2 * A.npad;
  F *rq = row_part + static_cast<int64_t>(it.w) * 2 * A.plan.npad_rows;
  F *rs = rq + A.plan.npad_rows;
  int buf = 0;
  SymSub sg;
  for (int sub = 0; sym_sub(A.plan, it, sub, sg); ++sub) {
    const int64_t row0 = sg.grow0 + static_cast<int64_t>(wv) * kSymWaveRows;
    typename StepRec<V>::I rows[kSymRows];
    F wr[kSymRows], er[kSymRows], qmax[kSymRows], swmin[kSymRows];
    int k[kSymRows];  // row particles (fewer than 2^31)
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
      k[r] = static_cast<int>(row0) + r * 64 + lane;
      const int64_t kk = k[r] < A.npad ? k[r] : A.npad - 1;
      rows[r] = load_iv<V>(A, kk);
      col_weights<V>(A, kk, wr[r], er[r]);
      qmax[r] = F(0);
      swmin[r] = inf_of<F>();
    }
    const bool rows_pad = row0 + kSymWaveRows > A.n;
    for (int64_t jb = sg.j0; jb < it.z; jb += kSymBlock) {
      if (rows_pad || jb < row0 + kSymWaveRows || jb + kSymBlock > A.n)
        sym_block<V, 1>(A, rows, wr, er, k, jb, eps2, qmax, swmin, L, lane);
      else
        sym_block<V, 0>(A, rows, wr, er, k, jb, eps2, qmax, swmin, L, lane);
      wave_lds_sync();
      // column c = lane & 15 over the 16 lanes' entries of this lane's quarter, then the
      // four quarters
      const int c = lane & 15, quarter = lane >> 4;
      F cq = F(0), cs = inf_of<F>();
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e = (c * kSymLdsStride + quarter * 16 + i) * 2;
        cq = fmax(cq, L[e]);
        cs = fmin(cs, L[e + 1]);
      }
      cq = fmax(cq, __shfl_xor(cq, 16, 64));
      cs = fmin(cs, __shfl_xor(cs, 16, 64));
      cq = fmax(cq, __shfl_xor(cq, 32, 64));
      cs = fmin(cs, __shfl_xor(cs, 32, 64));
      // over the four waves (and the band's row groups): maxima of the first value,
      // minima of the second
      const F both[2] = {cq, -cs};
      sym_group_store<kSymBlock, 2>(xs, buf, wv, lane, both, colq + jb, A.npad,
                                    [](F x, F y) { return fmax(x, y); }, sub > 0);
      wave_lds_sync();
    }
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
      rq[k[r]] = qmax[r];
      rs[k[r]] = swmin[r];
    }
  }
}

// Particle p (target q = inv[p]): the row partials of the items of its band that reach
// its row group, in slot order, then the column partials of the bands 0 .. its own (the
// minima stored negated, so that the four waves and the band's row groups combine both
// values by maxima).
template <class V>
__global__ __launch_bounds__(kWG) void k_timestep_sym_reduce(StepSymArgs A) {
  using F = typename V::F;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (p >= A.n) return;
  const int q = A.plan.inv[p];
  if (q < 0 || q >= A.n_act) return;  // not in the list
  int band, s0, s1;
  sym_row_slots(A.plan, A.npad, p, band, s0, s1);
  double qm = 0.0, sm = __builtin_inf();
  // the loads of kSymBatch slots (bands) are issued before they are combined (the kernel
  // is bound by reading the partials)
  const int64_t rs = A.plan.npad_rows;
  const F *r = static_cast<const F *>(A.plan.row_part) + 2 * s0 * rs + p;
  int s = s0;
  for (; s + kSymBatch <= s1; s += kSymBatch, r += 2 * kSymBatch * rs) {
    F y[kSymBatch][2];
#pragma unroll
    for (int b = 0; b < kSymBatch; ++b) {
      y[b][0] = r[(2 * b) * rs];
      y[b][1] = r[(2 * b + 1) * rs];
    }
#pragma unroll
    for (int b = 0; b < kSymBatch; ++b) {
      qm = fmax(qm, static_cast<double>(y[b][0]));
      sm = fmin(sm, static_cast<double>(y[b][1]));
    }
  }
  for (; s < s1; ++s, r += 2 * rs) {
    qm = fmax(qm, static_cast<double>(r[0]));
    sm = fmin(sm, static_cast<double>(r[rs]));
  }
  const F *c = static_cast<const F *>(A.plan.col_part) + p;
  int u = 0;
  for (; u + kSymBatch <= band + 1; u += kSymBatch, c += 2 * kSymBatch * A.npad) {
    F y[kSymBatch][2];
#pragma unroll
    for (int b = 0; b < kSymBatch; ++b) {
      y[b][0] = c[(2 * b) * A.npad];
      y[b][1] = c[(2 * b + 1) * A.npad];
    }
#pragma unroll
    for (int b = 0; b < kSymBatch; ++b) {
      qm = fmax(qm, static_cast<double>(y[b][0]));
      sm = fmin(sm, -static_cast<double>(y[b][1]));  // stored negated
    }
  }
  for (; u <= band; ++u, c += 2 * A.npad) {
    qm = fmax(qm, static_cast<double>(c[0]));
    sm = fmin(sm, -static_cast<double>(c[A.npad]));
  }
  if (A.raw) {
    A.raw[q] = qm;
    A.raw[A.n_act + q] = sm;
  } else {
    A.dtc[q] = finish_dt(A.eta, qm, sm);
  }
}

template <class V>
hipError_t run(StepSymArgs &A, hipStream_t st) {
  const int nb = A.plan.n_items;  // one work item per workgroup
  using F = typename V::F;
  hipLaunchKernelGGL((k_timestep_sym<V>), dim3(nb), dim3(kWG), 0, st, A, A.p32, A.p64, A.v64,
                     static_cast<F *>(A.plan.col_part), static_cast<F *>(A.plan.row_part));
  // its error check clears the launch error state: keep what it found
  const hipError_t e = launch_sym_inverse(A.plan, A.idx, A.n_act, A.n, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_timestep_sym_reduce<V>), dim3(static_cast<unsigned>((A.n + kWG - 1) / kWG)),
                     dim3(kWG), 0, st, A);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_timestep_sym(tsbts_ctx *c, const SymPlan &plan, const int32_t *idx,
                               int n_act, double eta, double *dtc, hipStream_t st,
                               const SymSet *set, double *raw) {
  StepSymArgs A;
  A.n = set ? set->n : c->n;
  A.npad = set ? set->npad : c->npad;
  A.p32 = set ? set->p32 : c->p32;
  A.p64 = set ? set->p64 : c->p64;
  A.v64 = set ? set->v64 : c->v64;
  A.raw = raw;
  A.eps2 = c->eps * c->eps;
  A.plan = plan;
  A.idx = idx;
  A.n_act = n_act;
  A.eta = eta;
  A.dtc = dtc;
  if (c->precision == TSBTS_FP64) return run<Fp64>(A, st);
  if (c->flags & TSBTS_FLAG_HILO_SEPARATION) return run<MixHiLo>(A, st);
  return run<MixSep64>(A, st);
}

}  // namespace tsbts
