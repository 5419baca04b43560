// Adjoint of the force when every particle is a target (not in the paper): each unordered
// pair once for both particles (symmetric all-targets scheme of sym.hpp).
//
// With e = r_j - r_k, s = |e|^2 + eps^2, y = s^(-1/2), u_k = e.g_k, u_j = e.g_j, the two
// parts of the adjoint (see backward.hip) give row k and column j, over the pair,
//   dL/dr_k += t,   dL/dr_j -= t,
//   t = y^3 (m_k g_j - m_j g_k) - y^3 [3 y^2 (m_k u_j - m_j u_k) + m_k gp_j + m_j gp_k] e,
//   dL/dm_k += -y (y^2 u_j + gp_j),   dL/dm_j += y (y^2 u_k - gp_k)
// (the position part is antisymmetric in the pair).  Mixed precision (without the Newton
// step): float32 pair arithmetic on the float64 (or hi/lo) separation, float32 sums over a
// column tile of 64 (rows) or over a work item's rows (columns), float64 across them;
// float64 mode: everything in float64.  Combined in a fixed order and added to grad_r,
// grad_m.
#include "sym.hpp"
#include "pair.hpp"

namespace tsbts {
namespace {

struct BwdSymArgs {
  int64_t n, npad;
  const float *p32;
  const double *p64;
  const double *gord;  // [4][npad] seeds in particle order (zero for padding)
  float eps2;
  double eps2_64;
  SymPlan plan;
  double *gr, *gm;
};

__global__ __launch_bounds__(kWG) void k_bwd_seeds32(int64_t len, const double *gord,
                                                     float *g32) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (e < len) g32[e] = static_cast<float>(gord[e]);
}

template <class V>
__device__ __forceinline__ void pair_bwd_sym(const typename V::I &i, typename V::F mi,
                                             const typename V::F (&gi)[4],
                                             const typename V::J &j,
                                             const typename V::F (&gj)[4],
                                             typename V::F eps2, bool skip,
                                             typename V::F (&acc)[4],
                                             typename V::F (&cacc)[4]) {
  using F = typename V::F;
  F ex, ey, ez;
  V::sep(i, j, ex, ey, ez);
  const F s = fma(ex, ex, fma(ey, ey, fma(ez, ez, eps2)));
  F y;
  if constexpr (sizeof(F) == 4)
    y = rsq_f32(s);
  else
    y = rsqrt_f64<2>(s);
  if (skip) y = F(0);
  const F y2 = y * y;
  const F y3 = y2 * y;
  const F mj = V::mass(j);
  // the masses enter only through y^3 m_k and y^3 m_j
  const F P = y3 * mi, Q = y3 * mj;
  const F uj = fma(ex, gj[0], fma(ey, gj[1], ez * gj[2]));
  const F ui = fma(ex, gi[0], fma(ey, gi[1], ez * gi[2]));
  const F a3 = fma(P, uj, -(Q * ui));        // y^3 (m_k u_j - m_j u_k)
  const F gs3 = fma(P, gj[3], Q * gi[3]);    // y^3 (m_k gp_j + m_j gp_k)
  const F c = fma(F(-3) * y2, a3, -gs3);
  const F tx = fma(P, gj[0], fma(-Q, gi[0], c * ex));
  const F ty = fma(P, gj[1], fma(-Q, gi[1], c * ey));
  const F tz = fma(P, gj[2], fma(-Q, gi[2], c * ez));
  acc[0] += tx;
  acc[1] += ty;
  acc[2] += tz;
  cacc[0] -= tx;
  cacc[1] -= ty;
  cacc[2] -= tz;
  acc[3] = fma(-y, fma(y2, uj, gj[3]), acc[3]);
  cacc[3] = fma(y, fma(y2, ui, -gi[3]), cacc[3]);
}

// columns per LDS transposition: 8 of float32, 4 of float64 (same LDS bytes)
template <class F> struct BCols { static constexpr int kBlock = sizeof(F) == 4 ? 8 : 4; };

template <class V, int MASK>
__device__ __forceinline__ void bwd_block(const BwdSymArgs &A, const typename V::F *g,
                                          const typename V::I (&rows)[kSymRows],
                                          const typename V::F (&mr)[kSymRows],
                                          const typename V::F (&gr)[kSymRows][4],
                                          const int (&k)[kSymRows], int64_t jb,
                                          typename V::F (&a)[kSymRows][4], typename V::F *L,
                                          int lane) {
  using F = typename V::F;
  const F eps2 = sizeof(F) == 4 ? static_cast<F>(A.eps2) : static_cast<F>(A.eps2_64);
#pragma unroll 2
  for (int c = 0; c < BCols<F>::kBlock; ++c) {
    const int64_t j = jb + c;
    const typename V::J Jr = V::load_j(A.p32, A.p64, A.npad, j, 1.0f);
    const F gj[4] = {g[j], g[A.npad + j], g[2 * A.npad + j], g[3 * A.npad + j]};
    F ca[4] = {F(0), F(0), F(0), F(0)};
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
      const bool skip = MASK && (j <= k[r] || j >= A.n || k[r] >= A.n);
      pair_bwd_sym<V>(rows[r], mr[r], gr[r], Jr, gj, eps2, skip, a[r], ca);
    }
    F *e = L + (c * kSymLdsStride + lane) * 4;
    e[0] = ca[0];
    e[1] = ca[1];
    e[2] = ca[2];
    e[3] = ca[3];
  }
}

template <class V>
__global__ __launch_bounds__(kWG) void k_bwd_sym(BwdSymArgs A0, const float *__restrict__ p32,
                                                 const double *__restrict__ p64,
                                                 const typename V::F *__restrict__ g32,
                                                 typename V::F *__restrict__ col_part,
                                                 double *__restrict__ row_part) {
  using F = typename V::F;
  constexpr int BLK = BCols<F>::kBlock;
  __shared__ F lds[kWG / 64][BLK * kSymLdsStride * 4];
  BwdSymArgs A = A0;
  A.p32 = p32;
  A.p64 = p64;
  __shared__ F xs[2][kSymWaves][4][BLK];
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
    F mr[kSymRows], gr[kSymRows][4];
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
      for (int v = 0; v < 4; ++v) {
        gr[r][v] = g32[v * A.npad + kk];
        tot[r][v] = 0.0;
      }
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
          bwd_block<V, 1>(A, g32, rows, mr, gr, k, jb, a, L, lane);
        else
          bwd_block<V, 0>(A, g32, rows, mr, gr, k, jb, a, L, lane);
        wave_lds_sync();
        F cs[4];
        sym_col_sums<BLK, 4>(L, lane, cs);
        sym_group_store<BLK, 4>(xs, buf, wv, lane, cs, cpart + jb, A.npad,
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

// Particle p: the row partials of the items of its band that reach its row group, in
// slot order, then the column partials of the bands 0 .. its own, added to grad_r and
// grad_m.
template <class F>
__global__ __launch_bounds__(kWG) void k_bwd_sym_reduce(BwdSymArgs A) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (p >= A.n) return;
  int band, s0, s1;
  sym_row_slots(A.plan, A.npad, p, band, s0, s1);
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  sym_sum_partials<4, 4>(static_cast<const double *>(A.plan.row_part) + p, A.plan.npad_rows,
                         s0, s1, t);
  sym_sum_partials<4, 4>(static_cast<const F *>(A.plan.col_part) + p, A.npad, 0, band + 1, t);
#pragma unroll
  for (int v = 0; v < 3; ++v) A.gr[v * A.n + p] += t[v];
  A.gm[p] += t[3];
}

template <class V>
hipError_t run(BwdSymArgs &A, hipStream_t st) {
  using F = typename V::F;
  const F *g;
  if constexpr (sizeof(F) == 4) {
    // float32 seeds for the scalar loads of the column records
    const int64_t len = 4 * A.npad;
    hipLaunchKernelGGL(k_bwd_seeds32, dim3(static_cast<unsigned>((len + kWG - 1) / kWG)),
                       dim3(kWG), 0, st, len, A.gord, A.plan.aux);
    g = A.plan.aux;
  } else {
    g = A.gord;
  }
  const int nb = A.plan.n_items;  // one work item per workgroup
  hipLaunchKernelGGL((k_bwd_sym<V>), dim3(nb), dim3(kWG), 0, st, A, A.p32, A.p64, g,
                     static_cast<F *>(A.plan.col_part),
                     static_cast<double *>(A.plan.row_part));
  hipLaunchKernelGGL(k_bwd_sym_reduce<F>, dim3(static_cast<unsigned>((A.n + kWG - 1) / kWG)),
                     dim3(kWG), 0, st, A);
  return hipGetLastError();
}

}  // namespace

bool bwd_sym_applies(const tsbts_ctx *c, int64_t n_act) {
  return sym_enabled(c, n_act) && (c->flags & TSBTS_FLAG_NEWTON) == 0;
}

// After k_bwd_order has put the seeds in particle order (gord).
hipError_t launch_bwd_sym(tsbts_ctx *c, const SymPlan &plan, double *gr, double *gm,
                          hipStream_t st) {
  BwdSymArgs A;
  A.n = c->n;
  A.npad = c->npad;
  A.p32 = c->p32;
  A.p64 = c->p64;
  A.gord = c->gord;
  A.eps2 = static_cast<float>(c->eps * c->eps);
  A.eps2_64 = c->eps * c->eps;
  A.plan = plan;
  A.gr = gr;
  A.gm = gm;
  if (c->precision == TSBTS_FP64) return run<Fp64>(A, st);
  if (c->flags & TSBTS_FLAG_HILO_SEPARATION) return run<MixHiLo>(A, st);
  return run<MixSep64>(A, st);
}

}  // namespace tsbts
