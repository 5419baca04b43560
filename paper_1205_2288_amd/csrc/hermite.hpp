// Cubic Hermite interpolation between two stored states of a particle (the time-symmetric
// interpolation of Section 2 used from the second pass on), shared by the predictor and
// by its adjoint.
#pragma once

#include "internal.hpp"

namespace tsbts {

// Between records (t0; r0, v0, a0) and (t1; r1, v1, a1): positions from (r, v) at both
// ends, velocities from (v, a):
//   tau = (t - t0)/h, H00 = 2tau^3 - 3tau^2 + 1, H10 = tau^3 - 2tau^2 + tau,
//   H01 = -2tau^3 + 3tau^2, H11 = tau^3 - tau^2,
//   x(t) = H00 x0 + h H10 x0' + H01 x1 + h H11 x1'.
// The interpolant is linear in the stored values with these four weights, which are also
// the weights of its adjoint.
struct Herm {
  double h00, h10h, h01, h11h;
  __device__ Herm(double t0, double t1, double t) {
    const double h = t1 - t0;
    const double tau = (t - t0) / h;
    const double tau2 = tau * tau, tau3 = tau2 * tau;
    h00 = 2.0 * tau3 - 3.0 * tau2 + 1.0;
    h10h = (tau3 - 2.0 * tau2 + tau) * h;
    h01 = -2.0 * tau3 + 3.0 * tau2;
    h11h = (tau3 - tau2) * h;
  }
  __device__ double operator()(double p0, double d0, double p1, double d1) const {
    return h00 * p0 + h10h * d0 + h01 * p1 + h11h * d1;
  }
};

// Record of particle j that the interpolation at time t starts from: the last record in
// [lo, hi) with time <= t, or lo when there is none (records are in time order).
__device__ __forceinline__ int bracket_search(const double *ht, int lo, int hi, double t) {
  int a = lo, b = hi - 1;
  while (a < b) {
    const int mid = (a + b + 1) >> 1;
    if (ht[mid] <= t) a = mid; else b = mid - 1;
  }
  return a;
}

}  // namespace tsbts
