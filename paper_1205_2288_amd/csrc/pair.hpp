// Pair arithmetic policies shared by the force, criterion and adjoint kernels.
//
// A policy defines how the j-particles of a tile are held in LDS (J), how a target particle
// is held in registers (I), and how a separation d = r_j - r_i is formed:
//   MixHiLo  : positions as float32 hi/lo pairs; d = (xj_hi - xi_hi) + (xj_lo - xi_lo),
//              exact in the hi difference for nearby pairs, then float32 arithmetic.
//   MixSep64 : positions in float64; d formed in float64 and rounded once to float32.
//   Fp64     : everything in float64.
#pragma once

#include "internal.hpp"

namespace tsbts {

// Float32 1/sqrt(s).  With NEWTON, one Newton step on the hardware estimate is folded
// into a result scaled by 2: z = y (3 - s y^2) = 2/sqrt(s) (the factor is removed by the
// callers through pre-scaled masses), so the refinement costs three operations.
template <int NEWTON>
__device__ __forceinline__ float rsq_refined(float s) {
  const float y = rsq_f32(s);
  if (NEWTON) return y * fmaf(-s * y, y, 3.0f);
  return y;
}

struct MixHiLo {
  struct __align__(16) J { float4 a, b; };  // a = (x_hi, y_hi, z_hi, m'), b = (x_lo, y_lo, z_lo, w)
  struct I { float xh, yh, zh, xl, yl, zl; };
  using F = float;
  __device__ static J load_j(const float *p32, const double *, int64_t P, int64_t j, float ms) {
    J r;
    r.a = make_float4(p32[(P32_XH + 0) * P + j], p32[(P32_XH + 1) * P + j],
                      p32[(P32_XH + 2) * P + j], p32[P32_M * P + j] * ms);
    r.b = make_float4(p32[(P32_XL + 0) * P + j], p32[(P32_XL + 1) * P + j],
                      p32[(P32_XL + 2) * P + j], p32[P32_W * P + j]);
    return r;
  }
  __device__ static I load_i(const float *p32, const double *, int64_t P, int64_t g) {
    I r;
    r.xh = p32[(P32_XH + 0) * P + g];
    r.yh = p32[(P32_XH + 1) * P + g];
    r.zh = p32[(P32_XH + 2) * P + g];
    r.xl = p32[(P32_XL + 0) * P + g];
    r.yl = p32[(P32_XL + 1) * P + g];
    r.zl = p32[(P32_XL + 2) * P + g];
    return r;
  }
  // separation r_j - r_i
  __device__ static void sep(const I &i, const J &j, float &dx, float &dy, float &dz) {
    dx = (j.a.x - i.xh) + (j.b.x - i.xl);
    dy = (j.a.y - i.yh) + (j.b.y - i.yl);
    dz = (j.a.z - i.zh) + (j.b.z - i.zl);
  }
  __device__ static float mass(const J &j) { return j.a.w; }
  __device__ static float weight(const J &j) { return j.b.w; }
};

struct MixSep64 {
  struct __align__(16) J { double x, y, z; float m, w; };
  struct I { double x, y, z; };
  using F = float;
  __device__ static J load_j(const float *p32, const double *p64, int64_t P, int64_t j,
                             float ms) {
    J r;
    r.x = p64[(P64_X + 0) * P + j];
    r.y = p64[(P64_X + 1) * P + j];
    r.z = p64[(P64_X + 2) * P + j];
    r.m = p32[P32_M * P + j] * ms;
    r.w = p32[P32_W * P + j];
    return r;
  }
  __device__ static I load_i(const float *, const double *p64, int64_t P, int64_t g) {
    I r;
    r.x = p64[(P64_X + 0) * P + g];
    r.y = p64[(P64_X + 1) * P + g];
    r.z = p64[(P64_X + 2) * P + g];
    return r;
  }
  __device__ static void sep(const I &i, const J &j, float &dx, float &dy, float &dz) {
    dx = static_cast<float>(j.x - i.x);
    dy = static_cast<float>(j.y - i.y);
    dz = static_cast<float>(j.z - i.z);
  }
  __device__ static float mass(const J &j) { return j.m; }
  __device__ static float weight(const J &j) { return j.w; }
};

struct Fp64 {
  struct __align__(16) J { double x, y, z, m; };
  struct I { double x, y, z; };
  using F = double;
  __device__ static J load_j(const float *, const double *p64, int64_t P, int64_t j, float) {
    J r;
    r.x = p64[(P64_X + 0) * P + j];
    r.y = p64[(P64_X + 1) * P + j];
    r.z = p64[(P64_X + 2) * P + j];
    r.m = p64[P64_M * P + j];
    return r;
  }
  __device__ static I load_i(const float *, const double *p64, int64_t P, int64_t g) {
    I r;
    r.x = p64[(P64_X + 0) * P + g];
    r.y = p64[(P64_X + 1) * P + g];
    r.z = p64[(P64_X + 2) * P + g];
    return r;
  }
  __device__ static void sep(const I &i, const J &j, double &dx, double &dy, double &dz) {
    dx = j.x - i.x;
    dy = j.y - i.y;
    dz = j.z - i.z;
  }
  __device__ static double mass(const J &j) { return j.m; }
};

}  // namespace tsbts
