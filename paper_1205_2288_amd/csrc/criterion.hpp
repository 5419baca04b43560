// Time-step criterion pair arithmetic (Eq. nbdt of Section 2), shared by the criterion
// kernels and the fused force + criterion kernel.  Per pair: max |v_ij|^2 / |r_ij|^2 (the
// collision term) and min s m_j^(-2/3) (the free-fall term, s = |r_ij|^2 + eps^2); the
// square root and the 3/4 power are taken once per target in finish_dt.
#pragma once

#include "pair.hpp"

namespace tsbts {

template <class V> struct StepRec;

template <> struct StepRec<MixHiLo> {
  struct __align__(16) J { MixHiLo::J p; float4 v; };
  struct I { MixHiLo::I p; float vx, vy, vz; };
};
template <> struct StepRec<MixSep64> {
  struct __align__(16) J { MixSep64::J p; float4 v; };
  struct I { MixSep64::I p; float vx, vy, vz; };
};
template <> struct StepRec<Fp64> {
  struct __align__(16) J { Fp64::J p; double vx, vy, vz, w; };
  struct I { Fp64::I p; double vx, vy, vz; };
};

template <class V, class Args>
__device__ __forceinline__ typename StepRec<V>::J load_jv(const Args &A, int64_t j) {
  typename StepRec<V>::J r;
  const int64_t P = A.npad;
  r.p = V::load_j(A.p32, A.p64, P, j, 1.0f);
  if constexpr (sizeof(typename V::F) == 4) {
    // float32 velocities, and in the fourth lane eps^2 m_j^(-2/3) so that s m_j^(-2/3) is
    // one fma per pair (both planes written by the predictor)
    r.v = make_float4(A.p32[(P32_VX + 0) * P + j], A.p32[(P32_VX + 1) * P + j],
                      A.p32[(P32_VX + 2) * P + j], A.p32[P32_E * P + j]);
  } else {
    r.vx = A.v64[j];
    r.vy = A.v64[P + j];
    r.vz = A.v64[2 * P + j];
    r.w = A.p64[P64_W * P + j];
  }
  return r;
}

template <class V, class Args>
__device__ __forceinline__ typename StepRec<V>::I load_iv(const Args &A, int64_t g) {
  typename StepRec<V>::I r;
  const int64_t P = A.npad;
  r.p = V::load_i(A.p32, A.p64, P, g);
  r.vx = A.v64[g];
  r.vy = A.v64[P + g];
  r.vz = A.v64[2 * P + g];
  return r;
}

__device__ __forceinline__ void pair_step(const StepRec<MixHiLo>::I &i,
                                          const StepRec<MixHiLo>::J &j, float eps2, bool self,
                                          float &qmax, float &swmin) {
  float dx, dy, dz;
  MixHiLo::sep(i.p, j.p, dx, dy, dz);
  const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  const float ux = j.v.x - i.vx, uy = j.v.y - i.vy, uz = j.v.z - i.vz;
  const float v2 = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
  float q = v2 * __builtin_amdgcn_rcpf(r2);
  float sw = fmaf(r2, MixHiLo::weight(j.p), j.v.w);
  if (self) {
    q = 0.0f;
    sw = __builtin_inff();
  }
  qmax = fmaxf(qmax, q);
  swmin = fminf(swmin, sw);
}

__device__ __forceinline__ void pair_step(const StepRec<MixSep64>::I &i,
                                          const StepRec<MixSep64>::J &j, float eps2, bool self,
                                          float &qmax, float &swmin) {
  float dx, dy, dz;
  MixSep64::sep(i.p, j.p, dx, dy, dz);
  const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  const float ux = j.v.x - i.vx, uy = j.v.y - i.vy, uz = j.v.z - i.vz;
  const float v2 = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
  float q = v2 * __builtin_amdgcn_rcpf(r2);
  float sw = fmaf(r2, MixSep64::weight(j.p), j.v.w);
  if (self) {
    q = 0.0f;
    sw = __builtin_inff();
  }
  qmax = fmaxf(qmax, q);
  swmin = fminf(swmin, sw);
}

__device__ __forceinline__ void pair_step(const StepRec<Fp64>::I &i, const StepRec<Fp64>::J &j,
                                          double eps2, bool self, double &qmax,
                                          double &swmin) {
  double dx, dy, dz;
  Fp64::sep(i.p, j.p, dx, dy, dz);
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ux = j.vx - i.vx, uy = j.vy - i.vy, uz = j.vz - i.vz;
  const double v2 = ux * ux + uy * uy + uz * uz;
  // v2 / r2 through the hardware reciprocal estimate and two Newton steps
  double rr = __builtin_amdgcn_rcp(r2);
  rr = fma(rr, fma(-r2, rr, 1.0), rr);
  rr = fma(rr, fma(-r2, rr, 1.0), rr);
  double q = v2 * rr;
  double sw = (r2 + eps2) * j.w;
  if (self) {
    q = 0.0;
    sw = __builtin_inf();
  }
  qmax = fmax(qmax, q);
  swmin = fmin(swmin, sw);
}

// Both directions of one pair for the symmetric all-targets kernel: the row particle i
// gets the terms pair_step gives it against j, and the column particle j the terms
// pair_step would give it against i (cq, cs).  The separation and the velocity difference
// only change sign between the two directions, so r^2, v^2 and q are the same values and
// every result equals the gather kernel's bit for bit.  wi, ei: i's weight m^(-2/3) and
// eps^2 m^(-2/3) (mixed precision) or its weight alone (float64).
template <class V>
__device__ __forceinline__ void pair_step_sym(const typename StepRec<V>::I &i, float wi,
                                              float ei, const typename StepRec<V>::J &j,
                                              float eps2, bool skip, float &qmax,
                                              float &swmin, float &cq, float &cs) {
  float dx, dy, dz;
  V::sep(i.p, j.p, dx, dy, dz);
  const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  const float ux = j.v.x - i.vx, uy = j.v.y - i.vy, uz = j.v.z - i.vz;
  const float v2 = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
  float q = v2 * __builtin_amdgcn_rcpf(r2);
  float sw = fmaf(r2, V::weight(j.p), j.v.w);
  float swj = fmaf(r2, wi, ei);
  if (skip) {
    q = 0.0f;
    sw = __builtin_inff();
    swj = __builtin_inff();
  }
  qmax = fmaxf(qmax, q);
  swmin = fminf(swmin, sw);
  cq = fmaxf(cq, q);
  cs = fminf(cs, swj);
}

__device__ __forceinline__ void pair_step_sym(const StepRec<Fp64>::I &i, double wi, double,
                                              const StepRec<Fp64>::J &j, double eps2,
                                              bool skip, double &qmax, double &swmin,
                                              double &cq, double &cs) {
  double dx, dy, dz;
  Fp64::sep(i.p, j.p, dx, dy, dz);
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ux = j.vx - i.vx, uy = j.vy - i.vy, uz = j.vz - i.vz;
  const double v2 = ux * ux + uy * uy + uz * uz;
  double rr = __builtin_amdgcn_rcp(r2);
  rr = fma(rr, fma(-r2, rr, 1.0), rr);
  rr = fma(rr, fma(-r2, rr, 1.0), rr);
  double q = v2 * rr;
  double sw = (r2 + eps2) * j.w;
  double swj = (r2 + eps2) * wi;
  if (skip) {
    q = 0.0;
    sw = __builtin_inf();
    swj = __builtin_inf();
  }
  qmax = fmax(qmax, q);
  swmin = fmin(swmin, sw);
  cq = fmax(cq, q);
  cs = fmin(cs, swj);
}

__device__ __forceinline__ double finish_dt(double eta, double qmax, double swmin) {
  const double tcol = qmax > 0.0 ? sqrt(1.0 / qmax) : __builtin_inf();
  const double tff = pow(swmin, 0.75);
  return eta * fmin(tcol, tff);
}

}  // namespace tsbts
