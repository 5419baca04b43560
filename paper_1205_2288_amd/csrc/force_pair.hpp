// Softened pair force and potential (Section 2 force law with Plummer softening), shared
// by the force kernels and the fused force + criterion kernel.
#pragma once

#include "pair.hpp"

namespace tsbts {

// ----- pair contributions -------------------------------------------------------------
// acc += m r^-3 d (times a constant scale), pot += m r^-1.

template <class V, int NEWTON, int MASK, int POT>
__device__ __forceinline__ void pair_acc(const typename V::I &i, const typename V::J &j,
                                         float eps2, bool self, float &ax, float &ay,
                                         float &az, float &pp) {
  float dx, dy, dz;
  V::sep(i, j, dx, dy, dz);
  float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
  float m = V::mass(j);
  if (MASK && self) {
    s = 1.0f;
    m = 0.0f;
  }
  const float y = rsq_refined<NEWTON>(s);
  const float mr1 = m * y;
  const float mr3 = mr1 * (y * y);
  ax = fmaf(mr3, dx, ax);
  ay = fmaf(mr3, dy, ay);
  az = fmaf(mr3, dz, az);
  if (POT) pp += mr1;
}

template <class V, int NEWTON, int MASK, int POT>
__device__ __forceinline__ void pair_acc(const typename V::I &i, const typename V::J &j,
                                         double eps2, bool self, double &ax, double &ay,
                                         double &az, double &pp) {
  double dx, dy, dz;
  V::sep(i, j, dx, dy, dz);
  double s = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
  double m = V::mass(j);
  if (MASK && self) {
    s = 1.0;
    m = 0.0;
  }
  const double y = rsqrt_f64<2>(s);
  const double mr1 = m * y;
  const double mr3 = mr1 * (y * y);
  ax = fma(mr3, dx, ax);
  ay = fma(mr3, dy, ay);
  az = fma(mr3, dz, az);
  if (POT) pp += mr1;
}

// Mass scale held in LDS and the final acceleration scale (see rsq_refined).
template <class V, int NEWTON>
struct Scale {
  static constexpr float kMass = (NEWTON && sizeof(typename V::F) == 4) ? 0.5f : 1.0f;
  static constexpr double kAcc = (NEWTON && sizeof(typename V::F) == 4) ? 0.25 : 1.0;
};

}  // namespace tsbts
