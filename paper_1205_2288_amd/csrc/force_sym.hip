// Softened force and potential (Section 2 force law, Plummer softening; Algorithm 2,
// step 5) when every particle is a target: each unordered pair once for both particles
// (symmetric all-targets scheme of sym.hpp).  For the pair k < j with d = r_j - r_k and
// y = (|d|^2 + eps^2)^(-1/2), row k gets m_j y^3 d and m_j y, column j gets -m_k y^3 d and
// m_k y.  Mixed precision without the Newton step: float32 pair arithmetic on the float64
// separation (or the hi/lo one), float32 sums over a column tile of 64 (rows) or over one
// work item's rows (columns), float64 across them, combined in a fixed order.  The
// corrector can be applied as each target is finished, as in the gather kernels.
#include "correct.hpp"
#include "force_pair.hpp"
#include "sym.hpp"

namespace tsbts {
namespace {

// columns per LDS transposition and values per column: with the potential 8 columns of
// (x, y, z, potential), without it 16 columns of (x, y, z) (same LDS footprint per wave)
template <int POT> struct FCols {
  static constexpr int kBlock = POT ? 8 : 16;
  static constexpr int kNV = POT ? 4 : 3;
};

struct ForceSymArgs {
  int64_t n, npad;
  const float *p32;
  const double *p64;
  float eps2;
  double eps2_64;
  SymPlan plan;
  const int32_t *idx;
  int n_act;
  double *acc;  // [3][n_act]
  double *pot;  // [n_act] or null
  int correct;
  CorrectArgs corr;
};

// Both directions of pair (row i, column j): row sums (ax, ay, az, pp), column sums
// (cx, cy, cz, cp).
template <class V, int POT>
__device__ __forceinline__ void pair_acc_sym(const typename V::I &i, float mi,
                                             const typename V::J &j, float eps2, bool skip,
                                             float &ax, float &ay, float &az, float &pp,
                                             float &cx, float &cy, float &cz, float &cp) {
  float dx, dy, dz;
  V::sep(i, j, dx, dy, dz);
  const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
  float y = rsq_f32(s);
  if (skip) y = 0.0f;
  const float y3 = y * (y * y);
  const float mj = V::mass(j);
  const float mj3 = mj * y3;
  const float mi3 = mi * y3;
  ax = fmaf(mj3, dx, ax);
  ay = fmaf(mj3, dy, ay);
  az = fmaf(mj3, dz, az);
  cx = fmaf(-mi3, dx, cx);
  cy = fmaf(-mi3, dy, cy);
  cz = fmaf(-mi3, dz, cz);
  if (POT) {
    pp = fmaf(mj, y, pp);
    cp = fmaf(mi, y, cp);
  }
}

template <class V, int POT>
__device__ __forceinline__ void pair_acc_sym(const typename V::I &i, double mi,
                                             const typename V::J &j, double eps2, bool skip,
                                             double &ax, double &ay, double &az, double &pp,
                                             double &cx, double &cy, double &cz,
                                             double &cp) {
  double dx, dy, dz;
  V::sep(i, j, dx, dy, dz);
  const double s = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
  double y = rsqrt_f64<2>(s);
  if (skip) y = 0.0;
  const double y3 = y * (y * y);
  const double mj = V::mass(j);
  const double mj3 = mj * y3;
  const double mi3 = mi * y3;
  ax = fma(mj3, dx, ax);
  ay = fma(mj3, dy, ay);
  az = fma(mj3, dz, az);
  cx = fma(-mi3, dx, cx);
  cy = fma(-mi3, dy, cy);
  cz = fma(-mi3, dz, cz);
  if (POT) {
    pp = fma(mj, y, pp);
    cp = fma(mi, y, cp);
  }
}

template <class V, int POT, int MASK>
__device__ __forceinline__ void force_block(const ForceSymArgs &A,
                                            const typename V::I (&rows)[kSymRows],
                                            const typename V::F (&mr)[kSymRows],
                                            const int (&k)[kSymRows], int64_t jb,
                                            typename V::F (&a)[kSymRows][4],
                                            typename V::F *L, int lane) {
  using F = typename V::F;
  constexpr int NV = FCols<POT>::kNV;
  // columns per transposition (float64: half, same LDS bytes); the float64 column records
  // of an 8-column batch would not fit the scalar registers, so those batch by 4
  constexpr int BLK = sizeof(F) == 4 ? FCols<POT>::kBlock : FCols<POT>::kBlock / 2;
  constexpr int UNR = sizeof(F) == 4 ? 8 : 4;
  const F eps2 = sizeof(F) == 4 ? static_cast<F>(A.eps2) : static_cast<F>(A.eps2_64);
#pragma unroll UNR
  for (int c = 0; c < BLK; ++c) {
    const int64_t j = jb + c;
    const typename V::J Jr = V::load_j(A.p32, A.p64, A.npad, j, 1.0f);
    F cx = F(0), cy = F(0), cz = F(0), cp = F(0);
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
      const bool skip = MASK && (j <= k[r] || j >= A.n || k[r] >= A.n);
      pair_acc_sym<V, POT>(rows[r], mr[r], Jr, eps2, skip, a[r][0], a[r][1], a[r][2],
                           a[r][3], cx, cy, cz, cp);
    }
    F *e = L + (c * kSymLdsStride + lane) * NV;
    e[0] = cx;
    e[1] = cy;
    e[2] = cz;
    if (POT) e[NV - 1] = cp;
  }
}

template <class V, int POT>
__global__ __launch_bounds__(kWG) void k_force_sym(ForceSymArgs A0,
                                                   const float *__restrict__ p32,
                                                   const double *__restrict__ p64,
                                                   typename V::F *__restrict__ col_part,
                                                   double *__restrict__ row_part) {
  using F = typename V::F;
  // float64: half the columns per transposition (same LDS bytes)
  constexpr int BLK = sizeof(F) == 4 ? FCols<POT>::kBlock : FCols<POT>::kBlock / 2;
  constexpr int NV = FCols<POT>::kNV;
  __shared__ F lds[kWG / 64][BLK * kSymLdsStride * NV];
  ForceSymArgs A = A0;
  A.p32 = p32;
  A.p64 = p64;
  __shared__ F xs[2][kSymWaves][NV][BLK];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int4 it = A.plan.items[blockIdx.x];  // one work item per workgroup
  F *L = lds[wv];
  F *cpart = col_part + static_cast<int64_t>(it.x) * 4 * A.npad;
  double *rp = row_part + static_cast<int64_t>(it.w) * 4 * A.plan.npad_rows;
  int buf = 0;
  SymSub sg;
  for (int sub = 0; sym_sub(A.plan, it, sub, sg); ++sub) {
    const int64_t row0 = sg.grow0 + static_cast<int64_t>(wv) * kSymWaveRows;
    typename V::I rows[kSymRows];
    F mr[kSymRows];
    int k[kSymRows];
    double tot[kSymRows][4];
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
      k[r] = static_cast<int>(row0) + r * 64 + lane;
      const int64_t kk = k[r] < A.npad ? k[r] : A.npad - 1;
      rows[r] = V::load_i(A.p32, A.p64, A.npad, kk);
      if constexpr (sizeof(F) == 4)
        mr[r] = A.p32[P32_M * A.npad + kk];
      else
        mr[r] = A.p64[P64_M * A.npad + kk];
#pragma unroll
      for (int v = 0; v < 4; ++v) tot[r][v] = 0.0;
    }
    const bool rows_pad = row0 + kSymWaveRows > A.n;
    for (int64_t jt = sg.j0; jt < it.z; jt += 64) {
      F a[kSymRows][4];
#pragma unroll
      for (int r = 0; r < kSymRows; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) a[r][v] = F(0);
      for (int64_t jb = jt; jb < jt + 64; jb += BLK) {
        if (rows_pad || jb < row0 + kSymWaveRows || jb + BLK > A.n)
          force_block<V, POT, 1>(A, rows, mr, k, jb, a, L, lane);
        else
          force_block<V, POT, 0>(A, rows, mr, k, jb, a, L, lane);
        wave_lds_sync();
        F cs[NV];
        sym_col_sums<BLK, NV>(L, lane, cs);
        sym_group_store<BLK, NV>(xs, buf, wv, lane, cs, cpart + jb, A.npad,
                                 [](F x, F y) { return x + y; }, sub > 0);
        wave_lds_sync();
      }
#pragma unroll
      for (int r = 0; r < kSymRows; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) tot[r][v] += static_cast<double>(a[r][v]);
    }
#pragma unroll
    for (int r = 0; r < kSymRows; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) rp[v * A.plan.npad_rows + k[r]] = tot[r][v];
  }
}

// Particle p (target q = inv[p]): the row partials of the items of its band that reach
// its row group, in slot order, then the column partials of the bands 0 .. its own; then
// acc, pot and the corrector (sym_sum_partials: the kernel is bound by reading the
// partials); without the potential its values are neither read nor (for the columns)
// written.  At most 4 waves per SIMD: a grid of one thread per particle has few waves
// (2 per SIMD at 2^17 particles), and under a higher occupancy target the compiler gave
// each float64 partial load the registers of its address, one load in flight at a time.
template <class F, int POT>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(1, 4))) void
k_force_sym_reduce(ForceSymArgs A) {
  constexpr int NV = POT ? 4 : 3;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (p >= A.n) return;
  const int q = A.plan.inv[p];
  if (q < 0 || q >= A.n_act) return;  // not in the list
  int band, s0, s1;
  sym_row_slots(A.plan, A.npad, p, band, s0, s1);
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  sym_sum_partials<4, NV>(static_cast<const double *>(A.plan.row_part) + p, A.plan.npad_rows,
                          s0, s1, t);
  sym_sum_partials<4, NV>(static_cast<const F *>(A.plan.col_part) + p, A.npad, 0, band + 1, t);
  const double an[3] = {t[0], t[1], t[2]};
  A.acc[q] = an[0];
  A.acc[A.n_act + q] = an[1];
  A.acc[2 * A.n_act + q] = an[2];
  if (POT) A.pot[q] = -t[3];
  if (A.correct) correct_one(A.corr, q, p, an);
}

template <class V>
hipError_t run(ForceSymArgs &A, hipStream_t st) {
  using F = typename V::F;
  const int nb = A.plan.n_items;  // one work item per workgroup
  F *cp = static_cast<F *>(A.plan.col_part);
  double *rp = static_cast<double *>(A.plan.row_part);
  if (A.pot)
    hipLaunchKernelGGL((k_force_sym<V, 1>), dim3(nb), dim3(kWG), 0, st, A, A.p32, A.p64, cp,
                       rp);
  else
    hipLaunchKernelGGL((k_force_sym<V, 0>), dim3(nb), dim3(kWG), 0, st, A, A.p32, A.p64, cp,
                       rp);
  // its error check clears the launch error state: keep what it found
  const hipError_t e = launch_sym_inverse(A.plan, A.idx, A.n_act, A.n, st);
  if (e != hipSuccess) return e;
  const dim3 grid(static_cast<unsigned>((A.n + kWG - 1) / kWG));
  if (A.pot)
    hipLaunchKernelGGL((k_force_sym_reduce<F, 1>), grid, dim3(kWG), 0, st, A);
  else
    hipLaunchKernelGGL((k_force_sym_reduce<F, 0>), grid, dim3(kWG), 0, st, A);
  return hipGetLastError();
}

}  // namespace

bool force_sym_applies(const tsbts_ctx *c, int64_t n_act) {
  return sym_enabled(c, n_act) && (c->flags & TSBTS_FLAG_NEWTON) == 0;
}

hipError_t launch_force_sym(tsbts_ctx *c, const SymPlan &plan, const int32_t *idx, int n_act,
                            double *acc, double *pot, hipStream_t st,
                            const CorrectArgs *corr, const SymSet *set) {
  ForceSymArgs A;
  A.n = set ? set->n : c->n;
  A.npad = set ? set->npad : c->npad;
  A.p32 = set ? set->p32 : c->p32;
  A.p64 = set ? set->p64 : c->p64;
  A.eps2 = static_cast<float>(c->eps * c->eps);
  A.eps2_64 = c->eps * c->eps;
  A.plan = plan;
  A.idx = idx;
  A.n_act = n_act;
  A.acc = acc;
  A.pot = pot;
  A.correct = corr ? 1 : 0;
  if (corr) A.corr = *corr;
  if (c->precision == TSBTS_FP64) return run<Fp64>(A, st);
  if (c->flags & TSBTS_FLAG_HILO_SEPARATION) return run<MixHiLo>(A, st);
  return run<MixSep64>(A, st);
}

}  // namespace tsbts
