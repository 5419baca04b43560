// Prediction of all particles to a block time (Section 2 predictor; Algorithm 2, step 4)
// and the time-symmetric (cubic Hermite) interpolation of stored era data used from the
// second pass on and for era-end synchronisation.
//
// One thread per particle; float64 structure-of-arrays loads and stores, all coalesced.
// Bandwidth-bound: per particle, Taylor reads r, v, a, t_last, dt, m (88 B) and writes the
// float64 position/mass/weight planes (40 B), float64 velocities (24 B) and, in mixed
// precision, the float32 hi/lo, mass, weight, velocity and eps^2-weight planes (48 B).
#include "hermite.hpp"

namespace tsbts {
namespace {

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
};

__global__ __launch_bounds__(kWG) void k_predict(PredictArgs p) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (j >= p.o.npad) return;
  if (j >= p.n) {
    store_pad(p.o, j);
    return;
  }
  const int64_t n = p.n;
  const double tl = p.t_last[j];
  const bool active = (tl + p.dt[j] == p.tb);
  double s[6];
  bool done = false;
  if (p.use_hist && !active) {
    // the cursor follows the block time in either direction (a reverse sweep predicts
    // at decreasing times); it stops at the particle's first record
    const int lo = p.off[j], hi = p.off[j + 1];
    int k = p.cur[j];
    const int k0 = k;
    while (k > lo && p.ht[k] > p.tb) --k;
    while (k + 1 < hi && p.ht[k + 1] <= p.tb) ++k;
    if (k != k0) p.cur[j] = k;
    const bool exact = (p.ht[k] == p.tb);
    if (exact || k + 1 < hi) {
      from_records(p.ht, p.hs, p.hcap, k, p.tb, exact, s);
      done = true;
    }
  }
  if (!done) {
    const double h = p.tb - tl;
    const double hh = 0.5 * h * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double rr = p.r[c * n + j], vv = p.v[c * n + j], aa = p.a[c * n + j];
      s[c] = rr + vv * h + aa * hh;
      s[c + 3] = vv + aa * h;
    }
  }
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

hipError_t launch_predict(tsbts_ctx *c, double t_block, int use_history, hipStream_t st) {
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
  const int nb = static_cast<int>((c->npad + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_predict, dim3(nb), dim3(kWG), 0, st, p);
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
