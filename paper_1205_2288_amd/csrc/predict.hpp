// Prediction of a particle to a block time (Section 2 predictor; Algorithm 2, step 4) and
// the time-symmetric (cubic Hermite) interpolation of stored era data used from the
// second pass on: the per-particle arithmetic and the stores of the predicted planes,
// shared by the predictor kernel and by the small-set force kernel that predicts its
// sources as it loads them.
#pragma once

#include "hermite.hpp"

namespace tsbts {

struct Out {
  double *p64;  // [5][npad]
  double *v64;  // [3][npad]
  float *p32;   // [12][npad] or null
  int64_t npad;
  double eps2;
};

__device__ __forceinline__ void store_particle(const Out &o, int64_t j, double x, double y,
                                               double z, double vx, double vy, double vz,
                                               double m) {
  const int64_t P = o.npad;
  const double w = ff_weight(m);
  o.p64[0 * P + j] = x;
  o.p64[1 * P + j] = y;
  o.p64[2 * P + j] = z;
  o.p64[3 * P + j] = m;
  o.p64[4 * P + j] = w;
  o.v64[0 * P + j] = vx;
  o.v64[1 * P + j] = vy;
  o.v64[2 * P + j] = vz;
  if (o.p32) {
    float h, l;
    split_hilo(x, h, l);
    o.p32[(P32_XH + 0) * P + j] = h;
    o.p32[(P32_XL + 0) * P + j] = l;
    split_hilo(y, h, l);
    o.p32[(P32_XH + 1) * P + j] = h;
    o.p32[(P32_XL + 1) * P + j] = l;
    split_hilo(z, h, l);
    o.p32[(P32_XH + 2) * P + j] = h;
    o.p32[(P32_XL + 2) * P + j] = l;
    o.p32[P32_M * P + j] = static_cast<float>(m);
    o.p32[P32_W * P + j] = static_cast<float>(w);
    o.p32[(P32_VX + 0) * P + j] = static_cast<float>(vx);
    o.p32[(P32_VX + 1) * P + j] = static_cast<float>(vy);
    o.p32[(P32_VX + 2) * P + j] = static_cast<float>(vz);
    // criterion term eps^2 m^(-2/3) (0 when eps = 0, where a massless weight is infinite)
    o.p32[P32_E * P + j] = o.eps2 > 0.0 ? static_cast<float>(o.eps2 * w) : 0.0f;
  }
}

// Padding particles: far away, at rest, massless.  Their contributions to every sum
// vanish and they never win a minimum.
__device__ __forceinline__ void store_pad(const Out &o, int64_t j) {
  store_particle(o, j, kFar, kFar, kFar, 0.0, 0.0, 0.0, 0.0);
}

// Records of particle j in the finished history: times ht[k], state planes hs[c*hcap+k]
// (c = 0..2 position, 3..5 velocity, 6..8 acceleration).
__device__ __forceinline__ void from_records(const double *ht, const double *hs, int64_t hcap,
                                             int k, double t, bool exact, double out[6]) {
  if (exact) {
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = hs[c * hcap + k];
    return;
  }
  const Herm H(ht[k], ht[k + 1], t);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    out[c] = H(hs[c * hcap + k], hs[(c + 3) * hcap + k], hs[c * hcap + k + 1],
               hs[(c + 3) * hcap + k + 1]);
    out[c + 3] = H(hs[(c + 3) * hcap + k], hs[(c + 6) * hcap + k], hs[(c + 3) * hcap + k + 1],
                   hs[(c + 6) * hcap + k + 1]);
  }
}

// Pending new steps of at most this many targets travel by value (PredictArgs).
constexpr int kInlinePend = 256;

struct PredictArgs {
  Out o;
  int64_t n;
  const double *r, *v, *a, *m, *t_last, *dt;
  double tb;
  int use_hist;
  const double *ht, *hs;
  const int32_t *off;
  int32_t *cur;
  int64_t hcap;
  // Pending new steps of the previous block step (native scheduler): the corrector of
  // that step tagged each target g with pend_tag[g] = (step << 32) | q, q its position
  // in that step's active list, whose new steps pend_dt[q] the host chose after it.  A
  // particle whose tag names pend_step takes pend_dt[q] as its step; the thread that owns
  // it also stores it in dt_w.  Null pend_tag: no pending steps.
  // With pend_inline, the steps arrive by value instead: pend_dt[q] = 2^pend_exp[q] (every
  // step of the scheduler is a power of two), so no kernel reads them from host memory.
  const int64_t *pend_tag;
  const double *pend_dt;
  int64_t pend_step;
  double *dt_w;
  int pend_inline;
  int8_t pend_exp[kInlinePend];
};

// An active list of at most kInlineIdx particles passed by value to the first kernel of
// a block step, which writes it to `out` for the later kernels (no separate copy).
constexpr int kInlineIdx = 256;
struct InlineIdx {
  int32_t *out;
  int32_t k;  // 0: the list is already in device memory
  int32_t v[kInlineIdx];
};

__device__ __forceinline__ void store_inline_idx(const InlineIdx &in, int64_t t) {
  if (t < in.k) in.out[t] = in.v[t];
}

// Step of particle j at p.tb: its pending new step, else the stored one.
__device__ __forceinline__ double step_of(const PredictArgs &p, int64_t j, bool owner) {
  const double stored = p.dt[j];  // read with the tag, not after it
  if (p.pend_tag) {
    const int64_t e = p.pend_tag[j];
    if ((e >> 32) == p.pend_step) {
      const int32_t q = static_cast<int32_t>(e & 0xffffffff);
      const double d = p.pend_inline ? ldexp(1.0, p.pend_exp[q]) : p.pend_dt[q];
      if (owner) p.dt_w[j] = d;
      return d;
    }
  }
  return stored;
}

// Taylor polynomial of particle j from its last time tl to p.tb (Section 2 predictor).
__device__ __forceinline__ void predict_taylor(const PredictArgs &p, int64_t j, double tl,
                                               double s[6]) {
  const int64_t n = p.n;
  const double h = p.tb - tl;
  const double hh = 0.5 * h * h;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double rr = p.r[c * n + j], vv = p.v[c * n + j], aa = p.a[c * n + j];
    s[c] = rr + vv * h + aa * hh;
    s[c + 3] = vv + aa * h;
  }
}

// Predicted position and velocity of particle j < n at p.tb (Section 2 predictor;
// Algorithm 2, step 4): an active particle (t_last + dt = t_b) and, without a usable
// history, every particle by its Taylor polynomial; otherwise the stored record at t_b or
// the cubic Hermite interpolant of the two bracketing records.  The history cursor of j
// follows the block time in either direction (a reverse sweep predicts at decreasing
// times) and stops at the particle's first record; only the thread that owns j may move
// it (update_cursor); that thread also stores a pending new step (step_of).
__device__ __forceinline__ void predict_state(const PredictArgs &p, int64_t j,
                                              bool update_cursor, double s[6]) {
  const double tl = p.t_last[j];
  // the record range and cursor are read with the activity test's inputs, and the two
  // records at the cursor together: the loads overlap instead of following one another
  int lo = 0, hi = 0, k = 0;
  if (p.use_hist) {
    lo = p.off[j];
    hi = p.off[j + 1];
    k = p.cur[j];
  }
  const bool active = (tl + step_of(p, j, update_cursor) == p.tb);
  if (p.use_hist && !active) {
    // every particle has a record at its era start, so lo < hi and ht[k] exists
    const int k0 = k;
    double tk = p.ht[k];
    double tn = k + 1 < hi ? p.ht[k + 1] : 0.0;
    while (k > lo && tk > p.tb) {
      tn = tk;
      tk = p.ht[--k];
    }
    while (k + 1 < hi && tn <= p.tb) {
      tk = tn;
      ++k;
      tn = k + 1 < hi ? p.ht[k + 1] : 0.0;
    }
    if (update_cursor && k != k0) p.cur[j] = k;
    const bool exact = (tk == p.tb);
    if (exact || k + 1 < hi) {
      from_records(p.ht, p.hs, p.hcap, k, p.tb, exact, s);
      return;
    }
  }
  predict_taylor(p, j, tl, s);
}

// Predictor arguments for the context at t_block (history source of the context), with
// no pending steps.
PredictArgs predict_args(tsbts_ctx *c, double t_block, int use_history);
// The pending steps `pend` (may be null) in p: by value when they come as exponents.
void set_pending(PredictArgs &p, const PendingSteps *pend);

}  // namespace tsbts
