// Total energy E = K + W for the energy-error diagnostic (Section 3), in float64:
//   K =  1/2 sum_i m_i |v_i|^2,   W = -sum_{i<j} m_i m_j (|r_i - r_j|^2 + eps^2)^(-1/2).
// The upper triangle of 256x256 particle tiles (I <= J) is enumerated in row order and cut
// into at most kMaxEB contiguous ranges of tile pairs, one per workgroup: for each pair,
// target i = 256 I + lane in registers, the 256 sources of tile J in LDS, and on diagonal
// tiles only j > i counts.  Each lane sums its pairs in range order, the workgroup
// reduces its lanes in a fixed order into one partial, and a single workgroup then adds
// the partials in a fixed order, so the result is bit-reproducible and the partials take
// at most 2 kMaxEB float64 values whatever N.  1/sqrt uses the hardware float64 estimate
// refined by kNewton Newton steps.
#include <algorithm>

#include "internal.hpp"

namespace tsbts {
namespace {

constexpr int kTE = 256;
constexpr int kNewton = 1;
constexpr int64_t kMaxEB = 8192;  // workgroups (and partials) of the pair kernel

struct EnergyArgs {
  int64_t n;
  const double *r, *v, *m;
  double eps2;
  int64_t T;       // tile rows
  int64_t ntp;     // tile pairs T (T + 1) / 2
  int64_t nb;      // workgroups: min(ntp, kMaxEB)
  double *part;    // [nb][2]
  double *out;
};

struct __align__(16) SRec { double x, y, z, m; };

// Tile pair b -> (I, J), I <= J, rows enumerated I = 0, 1, ... with T - I pairs each.
__device__ __forceinline__ void tile_pair(int64_t b, int64_t T, int64_t &I, int64_t &J) {
  const double a = 2.0 * static_cast<double>(T) + 1.0;
  int64_t i = static_cast<int64_t>((a - sqrt(a * a - 8.0 * static_cast<double>(b))) * 0.5);
  auto first = [T](int64_t r) { return r * T - r * (r - 1) / 2; };
  while (i > 0 && first(i) > b) --i;
  while (first(i + 1) <= b) ++i;
  I = i;
  J = i + (b - first(i));
}

__global__ __launch_bounds__(kWG) void k_energy_pairs(EnergyArgs A) {
  __shared__ SRec sj[kTE];
  __shared__ double red[2][kWG / 64];
  const int tid = threadIdx.x;
  const int64_t n = A.n;
  // this workgroup's contiguous range of tile pairs
  const int64_t b0 = blockIdx.x * A.ntp / A.nb, b1 = (blockIdx.x + 1) * A.ntp / A.nb;
  double pw = 0.0, pk = 0.0;
  for (int64_t b = b0; b < b1; ++b) {
    int64_t I, J;
    tile_pair(b, A.T, I, J);
    const int64_t i = I * kTE + tid;
    const int64_t j = J * kTE + tid;
    SRec rec;
    if (j < n) {
      rec.x = A.r[j];
      rec.y = A.r[n + j];
      rec.z = A.r[2 * n + j];
      rec.m = A.m[j];
    } else {
      rec.x = rec.y = rec.z = kFar;
      rec.m = 0.0;
    }
    __syncthreads();  // the previous pair's sources are no longer read
    sj[tid] = rec;
    double xi = kFar, yi = kFar, zi = kFar, mi = 0.0;
    if (i < n) {
      xi = A.r[i];
      yi = A.r[n + i];
      zi = A.r[2 * n + i];
      mi = A.m[i];
      if (I == J) {
        const double vx = A.v[i], vy = A.v[n + i], vz = A.v[2 * n + i];
        pk += 0.5 * mi * (vx * vx + vy * vy + vz * vz);
      }
    }
    __syncthreads();
    double w = 0.0;
    if (i >= n) {
      // padding target: contributes nothing (and must not meet padding sources at d = 0)
    } else if (I != J) {
#pragma unroll 4
      for (int jj = 0; jj < kTE; ++jj) {
        const SRec s = sj[jj];
        const double dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
        const double q = fma(dx, dx, fma(dy, dy, fma(dz, dz, A.eps2)));
        w = fma(s.m, rsqrt_f64<kNewton>(q), w);
      }
    } else {
      for (int jj = 0; jj < kTE; ++jj) {
        const SRec s = sj[jj];
        const double dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
        double q = fma(dx, dx, fma(dy, dy, fma(dz, dz, A.eps2)));
        const bool upper = jj > tid;
        q = upper ? q : 1.0;
        const double mj = upper ? s.m : 0.0;
        w = fma(mj, rsqrt_f64<kNewton>(q), w);
      }
    }
    pw = fma(mi, w, pw);
  }
  pw = wave_sum(pw);
  pk = wave_sum(pk);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = pw;
    red[1][tid >> 6] = pk;
  }
  __syncthreads();
  if (tid == 0) {
    double sw = 0.0, sk = 0.0;
    for (int k = 0; k < kWG / 64; ++k) {
      sw += red[0][k];
      sk += red[1][k];
    }
    A.part[2 * blockIdx.x] = sw;
    A.part[2 * blockIdx.x + 1] = sk;
  }
}

constexpr int kRedWG = 1024;
__global__ __launch_bounds__(kRedWG) void k_energy_reduce(EnergyArgs A) {
  __shared__ double sw[kRedWG], sk[kRedWG];
  const int t = threadIdx.x;
  double w = 0.0, k = 0.0;
  for (int64_t b = t; b < A.nb; b += kRedWG) {
    w += A.part[2 * b];
    k += A.part[2 * b + 1];
  }
  sw[t] = w;
  sk[t] = k;
  __syncthreads();
  for (int s = kRedWG / 2; s > 0; s >>= 1) {
    if (t < s) {
      sw[t] += sw[t + s];
      sk[t] += sk[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    A.out[0] = sk[0];
    A.out[1] = -sw[0];
  }
}

}  // namespace

int64_t energy_partials_needed(const tsbts_ctx *c) {
  const int64_t T = (c->n + kTE - 1) / kTE;
  return 2 * std::min<int64_t>(T * (T + 1) / 2, kMaxEB);  // two doubles per workgroup
}

hipError_t launch_energy(tsbts_ctx *c, const double *r, const double *v, const double *m,
                         double *out, hipStream_t st) {
  EnergyArgs A;
  A.n = c->n;
  A.r = r;
  A.v = v;
  A.m = m;
  A.eps2 = c->eps * c->eps;
  A.T = (c->n + kTE - 1) / kTE;
  A.ntp = A.T * (A.T + 1) / 2;
  A.nb = std::min<int64_t>(A.ntp, kMaxEB);
  A.part = c->epart;
  A.out = out;
  hipLaunchKernelGGL(k_energy_pairs, dim3(static_cast<unsigned>(A.nb)), dim3(kWG), 0, st, A);
  hipLaunchKernelGGL(k_energy_reduce, dim3(1), dim3(kRedWG), 0, st, A);
  return hipGetLastError();
}

}  // namespace tsbts
