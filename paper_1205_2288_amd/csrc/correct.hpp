// Leapfrog corrector of one active particle (Section 2, Eq. leapfrog; Algorithm 2,
// step 6) and its era-history record, shared by the corrector kernel and by the force
// reductions that apply it directly (the native scheduler's fused force + corrector).
#pragma once

#include "internal.hpp"

namespace tsbts {

struct CorrectArgs {
  int64_t n, npad;
  const int32_t *idx;
  int n_act;
  double tb;
  const double *acc_new;
  const double *p64;
  double *v64;
  float *p32;  // mixed precision: float32 velocity planes refreshed too (else null)
  double *r, *v, *a, *t_last;
  int record;
  int64_t base;    // first free record slot
  int64_t cap;
  int32_t *pid, *rank, *cnt;
  double *rt, *rs;
  // native scheduler: each target g tagged (step << 32) | q, so that the next block step's
  // predictor finds its new step (PendingSteps); null: no tags
  int64_t *tag;
  int64_t step;
};

// The corrector's inputs of one target: its last time, its predicted position, the
// velocity and acceleration of its last step, and its record count (when recording).
struct TargetState {
  double tl, rn[3], v[3], a[3];
  int32_t cnt;
};

__device__ __forceinline__ TargetState load_target(const CorrectArgs &p, int64_t g) {
  const int64_t n = p.n, P = p.npad;
  TargetState s;
  s.tl = p.t_last[g];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s.rn[c] = p.p64[c * P + g];  // predicted position = r + v h + a h^2/2
    s.v[c] = p.v[c * n + g];
    s.a[c] = p.a[c * n + g];
  }
  s.cnt = p.record ? p.cnt[g] : 0;
  return s;
}

// Target q (particle g, inputs s) with new acceleration an: r <- predicted position,
// v <- v + (a + an) h / 2, a <- an, t_last <- t_block; append the record when recording.
// Writes only the bound state, the float64 / float32 velocity planes and the record of g,
// none of which a force kernel reads.
__device__ __forceinline__ void correct_target(const CorrectArgs &p, int q, int64_t g,
                                               const double an[3], const TargetState &s) {
  const int64_t n = p.n, P = p.npad;
  const double h = p.tb - s.tl;
  double st[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double rn = s.rn[c];
    const double vn = s.v[c] + 0.5 * (s.a[c] + an[c]) * h;
    p.r[c * n + g] = rn;
    p.v[c * n + g] = vn;
    p.a[c * n + g] = an[c];
    p.v64[c * P + g] = vn;
    if (p.p32) p.p32[(P32_VX + c) * P + g] = static_cast<float>(vn);
    st[c] = rn;
    st[c + 3] = vn;
    st[c + 6] = an[c];
  }
  p.t_last[g] = p.tb;
  if (p.tag) p.tag[g] = (p.step << 32) | static_cast<int64_t>(q);
  if (p.record) {
    const int64_t slot = p.base + q;
    p.pid[slot] = static_cast<int32_t>(g);
    p.rank[slot] = s.cnt;
    p.cnt[g] = s.cnt + 1;
    p.rt[slot] = p.tb;
#pragma unroll
    for (int c = 0; c < 9; ++c) p.rs[c * p.cap + slot] = st[c];
  }
}

// The same with the inputs read from the context.
__device__ __forceinline__ void correct_one(const CorrectArgs &p, int q, int64_t g,
                                            const double an[3]) {
  correct_target(p, q, g, an, load_target(p, g));
}

// Arguments of a corrector call on the context's bound state and era log.
CorrectArgs correct_args(tsbts_ctx *c, const int32_t *idx, int n_act, double t_block,
                         const double *acc_new);

}  // namespace tsbts
