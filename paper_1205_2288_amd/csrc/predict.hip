// Prediction of all particles to a block time (Section 2 predictor; Algorithm 2, step 4)
// and the time-symmetric (cubic Hermite) interpolation of stored era data used from the
// second pass on and for era-end synchronisation.
//
// One thread per particle; float64 structure-of-arrays loads and stores, all coalesced.
// Bandwidth-bound: per particle, Taylor reads r, v, a, t_last, dt, m (88 B) and writes the
// float64 position/mass/weight planes (40 B), float64 velocities (24 B) and, in mixed
// precision, the float32 hi/lo, mass, weight, velocity and eps^2-weight planes (48 B).
#include <algorithm>

#include "predict.hpp"

namespace tsbts {
namespace {

__global__ __launch_bounds__(kWG) void k_predict(PredictArgs p, InlineIdx in) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  store_inline_idx(in, j);
  if (j >= p.o.npad) return;
  if (j >= p.n) {
    store_pad(p.o, j);
    return;
  }
  double s[6];
  predict_state(p, j, true, s);
  store_particle(p.o, j, s[0], s[1], s[2], s[3], s[4], s[5], p.m[j]);
}

__global__ __launch_bounds__(kWG) void k_load_positions(Out o, int64_t n, const double *r,
                                                        const double *m) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (j >= o.npad) return;
  if (j >= n) {
    store_pad(o, j);
    return;
  }
  store_particle(o, j, r[j], r[n + j], r[2 * n + j], 0.0, 0.0, 0.0, m[j]);
}

struct SnapArgs {
  int64_t n;
  const double *r, *v, *a, *t_last;
  double T;
  int use_hist;
  const double *ht, *hs;
  const int32_t *off;
  int64_t hcap;
  double *r_out, *v_out;
};

__global__ __launch_bounds__(kWG) void k_snapshot(SnapArgs p) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (j >= p.n) return;
  const int64_t n = p.n;
  const double tl = p.t_last[j];
  double s[6];
  bool done = false;
  if (tl == p.T) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s[c] = p.r[c * n + j];
      s[c + 3] = p.v[c * n + j];
    }
    done = true;
  } else if (p.use_hist) {
    // binary search: last record with time <= T
    int lo = p.off[j], hi = p.off[j + 1] - 1;
    if (hi >= lo && p.ht[lo] <= p.T) {
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.ht[mid] <= p.T) lo = mid; else hi = mid - 1;
      }
      const bool exact = (p.ht[lo] == p.T);
      if (exact || lo + 1 < p.off[j + 1]) {
        from_records(p.ht, p.hs, p.hcap, lo, p.T, exact, s);
        done = true;
      }
    }
  }
  if (!done) {
    const double h = p.T - tl;
    const double hh = 0.5 * h * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double rr = p.r[c * n + j], vv = p.v[c * n + j], aa = p.a[c * n + j];
      s[c] = rr + vv * h + aa * hh;
      s[c + 3] = vv + aa * h;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    p.r_out[c * n + j] = s[c];
    p.v_out[c * n + j] = s[c + 3];
  }
}

Out make_out(tsbts_ctx *c) {
  Out o;
  o.p64 = c->p64;
  o.v64 = c->v64;
  o.p32 = c->precision == TSBTS_MIXED ? c->p32 : nullptr;
  o.npad = c->npad;
  o.eps2 = c->eps * c->eps;
  return o;
}

}  // namespace

PredictArgs predict_args(tsbts_ctx *c, double t_block, int use_history) {
  PredictArgs p;
  p.o = make_out(c);
  p.n = c->n;
  p.r = c->r;
  p.v = c->v;
  p.a = c->a;
  p.m = c->m;
  p.t_last = c->t_last;
  p.dt = c->dt;
  p.tb = t_block;
  p.use_hist = use_history;
  p.ht = c->h.ht;
  p.hs = c->h.hs;
  p.off = c->h.off;
  p.cur = c->h.cur;
  p.hcap = c->h.hcap;
  p.pend_tag = nullptr;
  p.pend_dt = nullptr;
  p.pend_step = 0;
  p.dt_w = c->dt;
  p.pend_inline = 0;
  return p;
}

void set_pending(PredictArgs &p, const PendingSteps *pend) {
  if (!pend) return;
  p.pend_tag = pend->tag;
  p.pend_dt = pend->dt;
  p.pend_step = pend->step;
  if (pend->exp && pend->k <= kInlinePend) {
    p.pend_inline = 1;
    std::copy(pend->exp, pend->exp + pend->k, p.pend_exp);
  }
}

hipError_t launch_predict(tsbts_ctx *c, double t_block, int use_history, hipStream_t st,
                          const PendingSteps *pend, const InlineIdx *in) {
  PredictArgs p = predict_args(c, t_block, use_history);
  set_pending(p, pend);
  InlineIdx none;
  none.out = nullptr;
  none.k = 0;
  // the inline list is written by the first threads of the grid
  const int64_t threads = std::max<int64_t>(c->npad, in ? in->k : 0);
  const int nb = static_cast<int>((threads + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_predict, dim3(nb), dim3(kWG), 0, st, p, in ? *in : none);
  return hipGetLastError();
}

hipError_t launch_load_positions(tsbts_ctx *c, const double *r, const double *m,
                                 hipStream_t st) {
  const int nb = static_cast<int>((c->npad + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_load_positions, dim3(nb), dim3(kWG), 0, st, make_out(c), c->n, r, m);
  return hipGetLastError();
}

hipError_t launch_snapshot(tsbts_ctx *c, double T, double *r_out, double *v_out,
                           hipStream_t st) {
  SnapArgs p;
  p.n = c->n;
  p.r = c->r;
  p.v = c->v;
  p.a = c->a;
  p.t_last = c->t_last;
  p.T = T;
  p.use_hist = c->h.valid ? 1 : 0;
  p.ht = c->h.ht;
  p.hs = c->h.hs;
  p.off = c->h.off;
  p.hcap = c->h.hcap;
  p.r_out = r_out;
  p.v_out = v_out;
  const int nb = static_cast<int>((c->n + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_snapshot, dim3(nb), dim3(kWG), 0, st, p);
  return hipGetLastError();
}

}  // namespace tsbts
