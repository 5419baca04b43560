// Adjoint of the force (vector-Jacobian product; not in the paper): from g_c = dL/dacc_c
// and gp_c = dL/dpot_c of the active targets c, accumulate dL/dr and dL/dm of all
// particles.  With e = r_source - r_target, s = |e|^2 + eps^2, y = s^(-1/2) and
// u = e . g, the two parts are
//
//   source part, every particle k (rows) against every active target c (columns), k != c:
//     dL/dr_k += m_k sum_c [ y^3 g_c - (3 y^5 u + gp_c y^3) e ],   e = r_c - r_k
//     dL/dm_k +=     sum_c [ -y^3 u - gp_c y ]
//   target part, every active k (rows) against every particle j (columns), j != k:
//     dL/dr_k += sum_j m_j [ -y^3 g_k + (3 y^5 u - gp_k y^3) e ],  e = r_j - r_k
//
// Both are gathers (each row owns its sums), with the same register/LDS tiling and
// split-column scheme as the force kernel: no scatter, no atomics, fixed-order float64
// combination.  When every particle is active the two parts run over the same pairs and
// are fused into one kernel that shares each pair's separation, 1/sqrt(s) and its powers
// (the adjoint seeds are first put in particle order).  The self pair is masked by index,
// only in tiles that can contain it (wave-uniform vote).
#include "pair.hpp"
#include "sym.hpp"

namespace tsbts {
namespace {

template <class V> struct GradT { using T = float4; };
template <> struct GradT<Fp64> { struct __align__(16) T { double x, y, z, w; }; };

// Column record of the source part: an active target's position, (g, gp) and index.
template <class V>
struct __align__(16) Col {
  typename V::J p;
  typename GradT<V>::T g;
  int idx;
  int pad[3];
};

// Column record of the fused kernel: a particle's position and mass, and its (g, gp).
template <class V>
struct __align__(16) ColAll {
  typename V::J p;
  typename GradT<V>::T g;
};

struct BwdArgs {
  const float *p32;
  const double *p64;
  int64_t n, npad;
  const int32_t *idx;
  int n_act;
  const double *ga, *gp;
  double *gr, *gm;
  SplitPlan plan;
  int n_ctiles;
  double eps2;
  double *part;
  double *gord;  // [4][npad] seeds in particle order (fused kernel)
  int blocks;
  int scalar_j;  // fused kernel reads its columns through scalar loads
};

template <class V, int NEWTON>
__device__ __forceinline__ typename V::F inv_r(typename V::F s) {
  if constexpr (sizeof(typename V::F) == 4) {
    return NEWTON ? 0.5f * rsq_refined<1>(s) : rsq_refined<0>(s);
  } else {
    return rsqrt_f64<2>(s);
  }
}

template <class V, int NEWTON, int MASK>
__device__ __forceinline__ void pair_src(const typename V::I &row, const Col<V> &c,
                                         typename V::F eps2, bool self,
                                         typename V::F acc[4]) {
  using F = typename V::F;
  F ex, ey, ez;
  V::sep(row, c.p, ex, ey, ez);
  const F s = fma(ex, ex, fma(ey, ey, fma(ez, ez, eps2)));
  F y = inv_r<V, NEWTON>(s);
  if (MASK && self) y = F(0);
  // 3 y^5 u + gp y^3 = y^3 (3 y^2 u + gp) and y^3 u + gp y = y (y^2 u + gp)
  const F y2 = y * y;
  const F y3 = y2 * y;
  const F u = fma(ex, F(c.g.x), fma(ey, F(c.g.y), ez * F(c.g.z)));
  const F gpc = F(c.g.w);
  const F coef = y3 * fma(F(3) * y2, u, gpc);
  acc[0] = fma(y3, F(c.g.x), fma(-coef, ex, acc[0]));
  acc[1] = fma(y3, F(c.g.y), fma(-coef, ey, acc[1]));
  acc[2] = fma(y3, F(c.g.z), fma(-coef, ez, acc[2]));
  acc[3] = fma(-y, fma(y2, u, gpc), acc[3]);
}

template <class V, int NEWTON, int MASK>
__device__ __forceinline__ void pair_tgt(const typename V::I &row, const typename V::J &j,
                                         const typename V::F g[4], typename V::F eps2,
                                         bool self, typename V::F acc[3]) {
  using F = typename V::F;
  F ex, ey, ez;
  V::sep(row, j, ex, ey, ez);
  const F s = fma(ex, ex, fma(ey, ey, fma(ez, ez, eps2)));
  F y = inv_r<V, NEWTON>(s);
  if (MASK && self) y = F(0);
  const F m = V::mass(j);
  const F y2 = y * y;
  const F my3 = m * (y2 * y);
  const F u = fma(ex, g[0], fma(ey, g[1], ez * g[2]));
  // 3 m y^5 u - gp m y^3 = m y^3 (3 y^2 u - gp)
  const F coef = my3 * fma(F(3) * y2, u, -g[3]);
  acc[0] = fma(-my3, g[0], fma(coef, ex, acc[0]));
  acc[1] = fma(-my3, g[1], fma(coef, ey, acc[1]));
  acc[2] = fma(-my3, g[2], fma(coef, ez, acc[2]));
}

// Both parts for one pair (row k, column j): acc[0..2] source sum P, acc[3] mass sum Q,
// acc[4..6] target sum R.
template <class V, int NEWTON, int MASK>
__device__ __forceinline__ void pair_all(const typename V::I &row, const typename V::F gk[4],
                                         const ColAll<V> &c, typename V::F eps2, bool self,
                                         typename V::F acc[7]) {
  using F = typename V::F;
  F ex, ey, ez;
  V::sep(row, c.p, ex, ey, ez);
  const F s = fma(ex, ex, fma(ey, ey, fma(ez, ez, eps2)));
  F y = inv_r<V, NEWTON>(s);
  if (MASK && self) y = F(0);
  const F y2 = y * y;
  const F y3 = y2 * y;
  const F z = F(3) * y2;
  // source part: k pulls on target j
  const F gx = F(c.g.x), gy = F(c.g.y), gz = F(c.g.z), gpj = F(c.g.w);
  const F us = fma(ex, gx, fma(ey, gy, ez * gz));
  const F cs = y3 * fma(z, us, gpj);
  acc[0] = fma(y3, gx, fma(-cs, ex, acc[0]));
  acc[1] = fma(y3, gy, fma(-cs, ey, acc[1]));
  acc[2] = fma(y3, gz, fma(-cs, ez, acc[2]));
  acc[3] = fma(-y, fma(y2, us, gpj), acc[3]);
  // target part: j pulls on target k
  const F m = V::mass(c.p);
  const F my3 = m * y3;
  const F ut = fma(ex, gk[0], fma(ey, gk[1], ez * gk[2]));
  const F ct = my3 * fma(z, ut, -gk[3]);
  acc[4] = fma(-my3, gk[0], fma(ct, ex, acc[4]));
  acc[5] = fma(-my3, gk[1], fma(ct, ey, acc[5]));
  acc[6] = fma(-my3, gk[2], fma(ct, ez, acc[6]));
}

__device__ __forceinline__ int wave_min_i(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = min(x, __shfl_xor(x, off, 64));
  return x;
}
__device__ __forceinline__ int wave_max_i(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

// ---------------------------------------------------------------- source part
template <class V, int NEWTON, int MASK>
__device__ __forceinline__ void src_tile(const typename V::I &row, const Col<V> *sc, int cnt,
                                         int64_t k, typename V::F eps2, typename V::F acc[4]) {
  for (int cc = 0; cc < cnt; ++cc) {
    const Col<V> c = sc[cc];
    pair_src<V, NEWTON, MASK>(row, c, eps2, MASK && c.idx == k, acc);
  }
}

template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_bwd_src(BwdArgs A) {
  using F = typename V::F;
  __shared__ Col<V> sc[kTJ];
  __shared__ int srange[2][kWG / 64];
  const int tid = threadIdx.x;
  int rtile, slice;
  split_tile(blockIdx.x, A.plan, rtile, slice);
  if (slice >= A.plan.n_slices) return;
  const int ct0 = slice * A.plan.tiles_per_slice;
  const int ct1 = min(ct0 + A.plan.tiles_per_slice, A.n_ctiles);
  const int64_t P = A.npad;
  const int64_t k = static_cast<int64_t>(rtile) * kWG + tid;  // row particle (< npad)
  const typename V::I row = V::load_i(A.p32, A.p64, P, k);
  const F eps2 = static_cast<F>(A.eps2);
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  for (int ct = ct0; ct < ct1; ++ct) {
    const int q = ct * kTJ + tid;
    Col<V> rec;
    int lo, hi;
    if (q < A.n_act) {
      const int64_t c = A.idx[q];
      rec.p = V::load_j(A.p32, A.p64, P, c, 1.0f);
      rec.g.x = A.ga[q];
      rec.g.y = A.ga[A.n_act + q];
      rec.g.z = A.ga[2 * A.n_act + q];
      rec.g.w = A.gp ? A.gp[q] : 0.0;
      rec.idx = static_cast<int>(c);
      lo = hi = rec.idx;
    } else {
      rec.p = V::load_j(A.p32, A.p64, P, P - 1, 1.0f);  // never used (beyond cnt)
      rec.g.x = rec.g.y = rec.g.z = rec.g.w = 0.0f;
      rec.idx = -1;
      lo = 0x7fffffff;
      hi = -1;
    }
    // index range of this tile's columns: rows outside it cannot meet themselves
    lo = wave_min_i(lo);
    hi = wave_max_i(hi);
    const int cnt = min(kTJ, A.n_act - ct * kTJ);
    __syncthreads();
    sc[tid] = rec;
    if ((tid & 63) == 0) {
      srange[0][tid >> 6] = lo;
      srange[1][tid >> 6] = hi;
    }
    __syncthreads();
    int tlo = srange[0][0], thi = srange[1][0];
#pragma unroll
    for (int w = 1; w < kWG / 64; ++w) {
      tlo = min(tlo, srange[0][w]);
      thi = max(thi, srange[1][w]);
    }
    F acc[4] = {F(0), F(0), F(0), F(0)};
    if (__ballot(k >= tlo && k <= thi) != 0)
      src_tile<V, NEWTON, 1>(row, sc, cnt, k, eps2, acc);
    else
      src_tile<V, NEWTON, 0>(row, sc, cnt, k, eps2, acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) tot[e] += static_cast<double>(acc[e]);
  }
  if (k >= A.n) return;
  if (A.plan.n_slices == 1) {
    const double mk = A.p64[P64_M * P + k];
#pragma unroll
    for (int e = 0; e < 3; ++e) A.gr[e * A.n + k] += mk * tot[e];
    A.gm[k] += tot[3];
  } else {
    double *out = A.part + static_cast<int64_t>(slice) * 4 * A.n;
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e * A.n + k] = tot[e];
  }
}

// Combine the source part's slices; SCALE_R multiplies the position sums by m_k.
template <int SCALE_R>
__global__ __launch_bounds__(kWG) void k_bwd_rows_reduce(BwdArgs A) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (k >= A.n) return;
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < A.plan.n_slices; ++s) {
    const double *in = A.part + static_cast<int64_t>(s) * 4 * A.n;
#pragma unroll
    for (int e = 0; e < 4; ++e) tot[e] += in[e * A.n + k];
  }
  const double mk = SCALE_R ? A.p64[P64_M * A.npad + k] : 1.0;
#pragma unroll
  for (int e = 0; e < 3; ++e) A.gr[e * A.n + k] += mk * tot[e];
  A.gm[k] += tot[3];
}

template <int SCALE_R>
__global__ __launch_bounds__(kWG) void k_bwd_rows_reduce_wave(BwdArgs A) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * (kWG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= A.n) return;
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = lane; s < A.plan.n_slices; s += 64) {
    const double *in = A.part + static_cast<int64_t>(s) * 4 * A.n;
#pragma unroll
    for (int e = 0; e < 4; ++e) tot[e] += in[e * A.n + k];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) tot[e] = wave_sum(tot[e]);
  if (lane != 0) return;
  const double mk = SCALE_R ? A.p64[P64_M * A.npad + k] : 1.0;
#pragma unroll
  for (int e = 0; e < 3; ++e) A.gr[e * A.n + k] += mk * tot[e];
  A.gm[k] += tot[3];
}

// ---------------------------------------------------------------- target part
template <class V, int NEWTON, int MASK>
__device__ __forceinline__ void tgt_tile(const typename V::I &row, const typename V::J *sj,
                                         const typename V::F gk[4], int64_t jbase, int64_t g,
                                         typename V::F eps2, typename V::F acc[3]) {
#pragma unroll 2
  for (int jj = 0; jj < kTJ; ++jj)
    pair_tgt<V, NEWTON, MASK>(row, sj[jj], gk, eps2, MASK && (jbase + jj == g), acc);
}

template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_bwd_tgt(BwdArgs A) {
  using F = typename V::F;
  __shared__ typename V::J sj[kTJ];
  const int tid = threadIdx.x;
  int itile, slice;
  split_tile(blockIdx.x, A.plan, itile, slice);
  if (slice >= A.plan.n_slices) return;
  const int jt0 = slice * A.plan.tiles_per_slice;
  const int jt1 = min(jt0 + A.plan.tiles_per_slice, A.n_ctiles);
  const int64_t P = A.npad;
  const int q = itile * kWG + tid;
  const int qq = min(q, A.n_act - 1);
  const int64_t g = A.idx[qq];
  const typename V::I row = V::load_i(A.p32, A.p64, P, g);
  const F gk[4] = {static_cast<F>(A.ga[qq]), static_cast<F>(A.ga[A.n_act + qq]),
                   static_cast<F>(A.ga[2 * A.n_act + qq]),
                   static_cast<F>(A.gp ? A.gp[qq] : 0.0)};
  const F eps2 = static_cast<F>(A.eps2);
  double tot[3] = {0.0, 0.0, 0.0};
  for (int jt = jt0; jt < jt1; ++jt) {
    const int64_t jbase = static_cast<int64_t>(jt) * kTJ;
    const typename V::J rec = V::load_j(A.p32, A.p64, P, jbase + tid, 1.0f);
    __syncthreads();
    sj[tid] = rec;
    __syncthreads();
    F acc[3] = {F(0), F(0), F(0)};
    if (__ballot(g >= jbase && g < jbase + kTJ) != 0)
      tgt_tile<V, NEWTON, 1>(row, sj, gk, jbase, g, eps2, acc);
    else
      tgt_tile<V, NEWTON, 0>(row, sj, gk, jbase, g, eps2, acc);
#pragma unroll
    for (int e = 0; e < 3; ++e) tot[e] += static_cast<double>(acc[e]);
  }
  if (q >= A.n_act) return;
  if (A.plan.n_slices == 1) {
#pragma unroll
    for (int e = 0; e < 3; ++e) A.gr[e * A.n + g] += tot[e];
  } else {
    double *out = A.part + static_cast<int64_t>(slice) * 3 * A.n_act;
#pragma unroll
    for (int e = 0; e < 3; ++e) out[e * A.n_act + q] = tot[e];
  }
}

__global__ __launch_bounds__(kWG) void k_bwd_tgt_reduce(BwdArgs A) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q >= A.n_act) return;
  double tot[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < A.plan.n_slices; ++s) {
    const double *in = A.part + static_cast<int64_t>(s) * 3 * A.n_act;
#pragma unroll
    for (int e = 0; e < 3; ++e) tot[e] += in[e * A.n_act + q];
  }
  const int64_t g = A.idx[q];
#pragma unroll
  for (int e = 0; e < 3; ++e) A.gr[e * A.n + g] += tot[e];
}

__global__ __launch_bounds__(kWG) void k_bwd_tgt_reduce_wave(BwdArgs A) {
  const int q = blockIdx.x * (kWG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= A.n_act) return;
  double tot[3] = {0.0, 0.0, 0.0};
  for (int s = lane; s < A.plan.n_slices; s += 64) {
    const double *in = A.part + static_cast<int64_t>(s) * 3 * A.n_act;
#pragma unroll
    for (int e = 0; e < 3; ++e) tot[e] += in[e * A.n_act + q];
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) tot[e] = wave_sum(tot[e]);
  if (lane != 0) return;
  const int64_t g = A.idx[q];
#pragma unroll
  for (int e = 0; e < 3; ++e) A.gr[e * A.n + g] += tot[e];
}

// ---------------------------------------------------------------- fused, all active
// Seeds in particle order: gord[c][idx[q]] = g[c][q]; padding particles get zero.
__global__ __launch_bounds__(kWG) void k_bwd_order(BwdArgs A) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  const int64_t P = A.npad;
  if (t < A.n_act) {
    const int64_t j = A.idx[t];
#pragma unroll
    for (int c = 0; c < 3; ++c) A.gord[c * P + j] = A.ga[c * A.n_act + t];
    A.gord[3 * P + j] = A.gp ? A.gp[t] : 0.0;
  } else if (t < A.n_act + (P - A.n)) {
    const int64_t j = A.n + (t - A.n_act);
#pragma unroll
    for (int c = 0; c < 4; ++c) A.gord[c * P + j] = 0.0;
  }
}

// Column (g, gp) of the fused kernel read straight from the ordered seed planes.
template <class V>
__device__ __forceinline__ typename GradT<V>::T load_g(const BwdArgs &A, int64_t j) {
  typename GradT<V>::T g;
  const int64_t P = A.npad;
  g.x = A.gord[j];
  g.y = A.gord[P + j];
  g.z = A.gord[2 * P + j];
  g.w = A.gord[3 * P + j];
  return g;
}

template <class V, int NEWTON, int MASK>
__device__ __forceinline__ void all_tile(const typename V::I &row, const typename V::F gk[4],
                                         const ColAll<V> *sc, int64_t jbase, int64_t k,
                                         typename V::F eps2, typename V::F acc[7]) {
#pragma unroll 2
  for (int jj = 0; jj < kTJ; ++jj)
    pair_all<V, NEWTON, MASK>(row, gk, sc[jj], eps2, MASK && (jbase + jj == k), acc);
}

template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_bwd_all(BwdArgs A) {
  using F = typename V::F;
  __shared__ ColAll<V> sc[kTJ];
  const int tid = threadIdx.x;
  int rtile, slice;
  split_tile(blockIdx.x, A.plan, rtile, slice);
  if (slice >= A.plan.n_slices) return;
  const int jt0 = slice * A.plan.tiles_per_slice;
  const int jt1 = min(jt0 + A.plan.tiles_per_slice, A.n_ctiles);
  const int64_t P = A.npad;
  const int64_t k = static_cast<int64_t>(rtile) * kWG + tid;  // row particle (< npad)
  const typename V::I row = V::load_i(A.p32, A.p64, P, k);
  const F gk[4] = {static_cast<F>(A.gord[k]), static_cast<F>(A.gord[P + k]),
                   static_cast<F>(A.gord[2 * P + k]), static_cast<F>(A.gord[3 * P + k])};
  const F eps2 = static_cast<F>(A.eps2);
  double tot[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int jt = jt0; jt < jt1; ++jt) {
    const int64_t jbase = static_cast<int64_t>(jt) * kTJ;
    const int64_t j = jbase + tid;
    ColAll<V> rec;
    rec.p = V::load_j(A.p32, A.p64, P, j, 1.0f);
    rec.g.x = A.gord[j];
    rec.g.y = A.gord[P + j];
    rec.g.z = A.gord[2 * P + j];
    rec.g.w = A.gord[3 * P + j];
    __syncthreads();
    sc[tid] = rec;
    __syncthreads();
    F acc[7] = {F(0), F(0), F(0), F(0), F(0), F(0), F(0)};
    if (__ballot(k >= jbase && k < jbase + kTJ) != 0)
      all_tile<V, NEWTON, 1>(row, gk, sc, jbase, k, eps2, acc);
    else
      all_tile<V, NEWTON, 0>(row, gk, sc, jbase, k, eps2, acc);
#pragma unroll
    for (int e = 0; e < 7; ++e) tot[e] += static_cast<double>(acc[e]);
  }
  if (k >= A.n) return;
  const double mk = A.p64[P64_M * P + k];
  double out4[4] = {mk * tot[0] + tot[4], mk * tot[1] + tot[5], mk * tot[2] + tot[6], tot[3]};
  if (A.plan.n_slices == 1) {
#pragma unroll
    for (int e = 0; e < 3; ++e) A.gr[e * A.n + k] += out4[e];
    A.gm[k] += out4[3];
  } else {
    double *out = A.part + static_cast<int64_t>(slice) * 4 * A.n;
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e * A.n + k] = out4[e];
  }
}

// The fused kernel with its columns read through wave-uniform (scalar) loads straight
// from the predicted and seed planes: no LDS staging, no barriers; same tiles, vote and
// sums as k_bwd_all.  Used in float64 mode, where it measured ~4% faster than the LDS
// form at N = 131072; in mixed precision it measured ~6% slower (eight scalar streams per
// column against a single staged record), so the LDS form stays the default there.
template <class V, int NEWTON, int MASK>
__device__ __forceinline__ void all_tile_scalar(const BwdArgs &A, const typename V::I &row,
                                                const typename V::F gk[4], int64_t jbase,
                                                int64_t k, typename V::F eps2,
                                                typename V::F acc[7]) {
#pragma unroll 4
  for (int jj = 0; jj < kTJ; ++jj) {
    ColAll<V> c;
    c.p = V::load_j(A.p32, A.p64, A.npad, jbase + jj, 1.0f);
    c.g = load_g<V>(A, jbase + jj);
    pair_all<V, NEWTON, MASK>(row, gk, c, eps2, MASK && (jbase + jj == k), acc);
  }
}

template <class V, int NEWTON>
__global__ __launch_bounds__(kWG) void k_bwd_all_scalar(BwdArgs A) {
  using F = typename V::F;
  const int tid = threadIdx.x;
  int rtile, slice;
  split_tile(blockIdx.x, A.plan, rtile, slice);
  if (slice >= A.plan.n_slices) return;
  const int jt0 = slice * A.plan.tiles_per_slice;
  const int jt1 = min(jt0 + A.plan.tiles_per_slice, A.n_ctiles);
  const int64_t P = A.npad;
  const int64_t k = static_cast<int64_t>(rtile) * kWG + tid;  // row particle (< npad)
  const typename V::I row = V::load_i(A.p32, A.p64, P, k);
  const F gk[4] = {static_cast<F>(A.gord[k]), static_cast<F>(A.gord[P + k]),
                   static_cast<F>(A.gord[2 * P + k]), static_cast<F>(A.gord[3 * P + k])};
  const F eps2 = static_cast<F>(A.eps2);
  double tot[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int jt = jt0; jt < jt1; ++jt) {
    const int64_t jbase = static_cast<int64_t>(jt) * kTJ;
    F acc[7] = {F(0), F(0), F(0), F(0), F(0), F(0), F(0)};
    if (__ballot(k >= jbase && k < jbase + kTJ) != 0)
      all_tile_scalar<V, NEWTON, 1>(A, row, gk, jbase, k, eps2, acc);
    else
      all_tile_scalar<V, NEWTON, 0>(A, row, gk, jbase, k, eps2, acc);
#pragma unroll
    for (int e = 0; e < 7; ++e) tot[e] += static_cast<double>(acc[e]);
  }
  if (k >= A.n) return;
  const double mk = A.p64[P64_M * P + k];
  double out4[4] = {mk * tot[0] + tot[4], mk * tot[1] + tot[5], mk * tot[2] + tot[6], tot[3]};
  if (A.plan.n_slices == 1) {
#pragma unroll
    for (int e = 0; e < 3; ++e) A.gr[e * A.n + k] += out4[e];
    A.gm[k] += out4[3];
  } else {
    double *out = A.part + static_cast<int64_t>(slice) * 4 * A.n;
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e * A.n + k] = out4[e];
  }
}

SplitPlan plan_src(const BwdArgs &A) {
  return plan_split(A.npad, 1, (A.n_act + kTJ - 1) / kTJ, A.blocks);
}
SplitPlan plan_tgt(const BwdArgs &A) {
  return plan_split(A.n_act, 1, A.npad / kTJ, A.blocks);
}
SplitPlan plan_all(const BwdArgs &A) { return plan_split(A.npad, 1, A.npad / kTJ, A.blocks); }

template <int SCALE_R>
void reduce_rows(BwdArgs &A, hipStream_t st) {
  if (use_wave_reduce(A.plan.n_slices, A.n)) {
    const int nb = static_cast<int>((A.n + kWG / 64 - 1) / (kWG / 64));
    hipLaunchKernelGGL(k_bwd_rows_reduce_wave<SCALE_R>, dim3(nb), dim3(kWG), 0, st, A);
  } else if (A.plan.n_slices > 1) {
    const int nb = static_cast<int>((A.n + kWG - 1) / kWG);
    hipLaunchKernelGGL(k_bwd_rows_reduce<SCALE_R>, dim3(nb), dim3(kWG), 0, st, A);
  }
}

template <class V, int NEWTON>
hipError_t run(BwdArgs &A, hipStream_t st, tsbts_ctx *c) {
  if (A.n_act == A.n) {
    // every particle is active (the active set is a permutation of all particles)
    const int64_t cnt = A.n_act + (A.npad - A.n);
    hipLaunchKernelGGL(k_bwd_order, dim3(static_cast<unsigned>((cnt + kWG - 1) / kWG)),
                       dim3(kWG), 0, st, A);
    if (bwd_sym_applies(c, A.n_act)) {
      SymPlan plan;
      if (sym_plan(c, 4, 8, c->precision == TSBTS_FP64 ? 8 : 4, &plan))
        return launch_bwd_sym(c, plan, A.gr, A.gm, st);
    }
    A.plan = plan_all(A);
    A.n_ctiles = static_cast<int>(A.npad / kTJ);
    if (A.scalar_j)
      hipLaunchKernelGGL((k_bwd_all_scalar<V, NEWTON>), dim3(A.plan.nblk), dim3(kWG), 0, st,
                         A);
    else
      hipLaunchKernelGGL((k_bwd_all<V, NEWTON>), dim3(A.plan.nblk), dim3(kWG), 0, st, A);
    reduce_rows<0>(A, st);
    return hipGetLastError();
  }
  // source part over all particles
  A.plan = plan_src(A);
  A.n_ctiles = (A.n_act + kTJ - 1) / kTJ;
  hipLaunchKernelGGL((k_bwd_src<V, NEWTON>), dim3(A.plan.nblk), dim3(kWG), 0, st, A);
  reduce_rows<1>(A, st);
  // target part over the active set
  A.plan = plan_tgt(A);
  A.n_ctiles = static_cast<int>(A.npad / kTJ);
  hipLaunchKernelGGL((k_bwd_tgt<V, NEWTON>), dim3(A.plan.nblk), dim3(kWG), 0, st, A);
  if (use_wave_reduce(A.plan.n_slices, A.n_act)) {
    const int nb = (A.n_act + kWG / 64 - 1) / (kWG / 64);
    hipLaunchKernelGGL(k_bwd_tgt_reduce_wave, dim3(nb), dim3(kWG), 0, st, A);
  } else if (A.plan.n_slices > 1) {
    const int nb = (A.n_act + kWG - 1) / kWG;
    hipLaunchKernelGGL(k_bwd_tgt_reduce, dim3(nb), dim3(kWG), 0, st, A);
  }
  return hipGetLastError();
}

}  // namespace

int64_t backward_partials_needed(const tsbts_ctx *c, int n_act) {
  BwdArgs A;
  A.n = c->n;
  A.npad = c->npad;
  A.n_act = n_act;
  A.blocks = c->tune_blocks;
  int64_t need = 0;
  if (n_act == c->n) {
    const SplitPlan a = plan_all(A);
    if (a.n_slices > 1) need = static_cast<int64_t>(a.n_slices) * 4 * c->n;
    return need;
  }
  const SplitPlan s = plan_src(A);
  const SplitPlan t = plan_tgt(A);
  if (s.n_slices > 1) need = static_cast<int64_t>(s.n_slices) * 4 * c->n;
  if (t.n_slices > 1) need = std::max<int64_t>(need, static_cast<int64_t>(t.n_slices) * 3 * n_act);
  return need;
}

hipError_t launch_backward(tsbts_ctx *c, const int32_t *idx, int n_act, const double *ga,
                           const double *gp, double *gr, double *gm, hipStream_t st) {
  BwdArgs A;
  A.p32 = c->p32;
  A.p64 = c->p64;
  A.n = c->n;
  A.npad = c->npad;
  A.idx = idx;
  A.n_act = n_act;
  A.ga = ga;
  A.gp = gp;
  A.gr = gr;
  A.gm = gm;
  A.eps2 = c->eps * c->eps;
  A.part = c->part;
  A.gord = c->gord;
  A.blocks = c->tune_blocks;
  A.scalar_j = force_scalar_j(c) && c->precision == TSBTS_FP64 ? 1 : 0;
  if (c->precision == TSBTS_FP64) return run<Fp64, 0>(A, st, c);
  const bool newton = (c->flags & TSBTS_FLAG_NEWTON) != 0;
  if (c->flags & TSBTS_FLAG_HILO_SEPARATION)
    return newton ? run<MixHiLo, 1>(A, st, c) : run<MixHiLo, 0>(A, st, c);
  return newton ? run<MixSep64, 1>(A, st, c) : run<MixSep64, 0>(A, st, c);
}

}  // namespace tsbts
