// Leapfrog corrector of the active block (Section 2, Eq. leapfrog; Algorithm 2, step 6),
// storage of every step of the era (Section 2), and small element-wise kernels.
//
// Era history: during a pass each corrected state is appended as a record
// (particle, time, r, v, a) in block-step order, together with its rank among that
// particle's records (a per-particle counter; each particle appears at most once per block
// step, so no atomics are needed).  At the end of the pass an exclusive scan of the
// per-particle counts gives each particle's first slot, and every record is scattered to
// slot offset[particle] + rank: the records end up grouped by particle and in time order
// (a stable counting sort).  Predictions of later passes walk these groups with a
// per-particle cursor that only moves forward.
#include "correct.hpp"

namespace tsbts {
namespace {

__global__ __launch_bounds__(kWG) void k_correct(CorrectArgs p) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q >= p.n_act) return;
  const double an[3] = {p.acc_new[q], p.acc_new[p.n_act + q], p.acc_new[2 * p.n_act + q]};
  correct_one(p, q, p.idx[q], an);
}

// First record of every particle: its state at its own last time.
__global__ __launch_bounds__(kWG) void k_history_begin(CorrectArgs p) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (j >= p.n) return;
  const int64_t n = p.n;
  p.pid[j] = static_cast<int32_t>(j);
  p.rank[j] = 0;
  p.cnt[j] = 1;
  p.rt[j] = p.t_last[j];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    p.rs[c * p.cap + j] = p.r[c * n + j];
    p.rs[(c + 3) * p.cap + j] = p.v[c * n + j];
    p.rs[(c + 6) * p.cap + j] = p.a[c * n + j];
  }
}

// Exclusive scan of cnt[0..n) into off[0..n] in tiles of 8192 counts, one workgroup of
// 1024 threads per tile (8 consecutive counts per thread, coalesced): a first kernel sums
// each tile, a second one scans each tile with the sum of the tiles before it as carry
// (waves scan with shuffles, wave totals meet in LDS).  Integer sums are exact, so the
// result does not depend on the order.  The second kernel also resets the interpolation
// cursors to the group starts.
constexpr int kScanWG = 1024;
constexpr int kScanPer = 8;
constexpr int64_t kScanTile = static_cast<int64_t>(kScanWG) * kScanPer;

__device__ __forceinline__ int block_sum_1024(int x, int *wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  if (lane == 0) wsum[w] = x;
  __syncthreads();
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanWG / 64; ++k) s += wsum[k];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(kScanWG) void k_scan_sums(const int32_t *cnt, int64_t n,
                                                       int32_t *tsum) {
  __shared__ int wsum[kScanWG / 64];
  const int64_t i0 = blockIdx.x * kScanTile + static_cast<int64_t>(threadIdx.x) * kScanPer;
  int local = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) local += i0 + e < n ? cnt[i0 + e] : 0;
  const int s = block_sum_1024(local, wsum);
  if (threadIdx.x == 0) tsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(kScanWG) void k_scan_tiles(const int32_t *cnt, int64_t n,
                                                        const int32_t *tsum, int32_t *off,
                                                        int32_t *cur) {
  __shared__ int wsum[kScanWG / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int b = blockIdx.x;
  int pre = 0;
  for (int k = t; k < b; k += kScanWG) pre += tsum[k];
  const int carry = block_sum_1024(pre, wsum);
  const int64_t i0 = b * kScanTile + static_cast<int64_t>(t) * kScanPer;
  int v[kScanPer];
  int local = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    v[e] = i0 + e < n ? cnt[i0 + e] : 0;
    local += v[e];
  }
  int x = local;  // inclusive scan over the wave
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kScanWG / 64; ++k) {
    before += k < w ? wsum[k] : 0;
    total += wsum[k];
  }
  int run = carry + before + x - local;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    if (i0 + e < n) {
      off[i0 + e] = run;
      cur[i0 + e] = run;
    }
    run += v[e];
  }
  if (b == gridDim.x - 1 && t == 0) off[n] = carry + total;
}

struct ScatterArgs {
  int64_t count, cap, hcap;
  const int32_t *pid, *rank, *off;
  const double *rt, *rs;
  double *ht, *hs;
};

__global__ __launch_bounds__(kWG) void k_scatter(ScatterArgs p) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (r >= p.count) return;
  const int64_t dst = static_cast<int64_t>(p.off[p.pid[r]]) + p.rank[r];
  p.ht[dst] = p.rt[r];
#pragma unroll
  for (int c = 0; c < kHistPlanes; ++c) p.hs[c * p.hcap + dst] = p.rs[c * p.cap + r];
}

__global__ __launch_bounds__(kWG) void k_set_dt(const int32_t *idx, int n_act, const double *dt_new,
                                                double *dt) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q < n_act) dt[idx[q]] = dt_new[q];
}

__global__ __launch_bounds__(kWG) void k_lf_adjoint(int64_t len, int phase, double h,
                                                    const double *rbar, double *vbar,
                                                    double *abar, double *g_out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (e >= len) return;
  const double vb = vbar[e];
  if (phase == 0) {
    g_out[e] = abar[e] + 0.5 * h * vb;
  } else {
    const double rb = rbar[e];
    abar[e] = 0.5 * h * vb + 0.5 * h * h * rb;
    vbar[e] = vb + h * rb;
  }
}

// Reverse of one block step of a fixed block schedule.  Forward (Section 2, one pass):
//   p_j = r_j + h_j v_j + h_j^2 a_j / 2 for every j, h_j = t_block - t_last_j;
//   an_i = F_i(p) for i in the active set A;
//   r_i <- p_i, v_i <- v_i + dt_i (a_i + an_i) / 2, a_i <- an_i for i in A.
// Phase 0 (active set): seed_i = abar_i + dt_i vbar_i / 2 (the adjoint of an_i);
// pbar_i = rbar_i (r_i' = p_i); abar_i = dt_i vbar_i / 2; rbar_i = 0.  pbar is zero
// elsewhere (cleared by k_fill first).  Phase 1 (every particle, after the force adjoint
// has added dL/dp into pbar): rbar += pbar, vbar += h pbar, abar += h^2 pbar / 2.
__global__ __launch_bounds__(kWG) void k_fill(int64_t len, double *x, double v) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (e < len) x[e] = v;
}

struct BlockAdjArgs {
  int64_t n;
  const int32_t *idx;
  int n_act;
  double t_block;
  const double *dt, *t_last;
  double *rbar, *vbar, *abar, *pbar, *seeds;
};

__global__ __launch_bounds__(kWG) void k_block_adj_active(BlockAdjArgs A) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q >= A.n_act) return;
  const int64_t i = A.idx[q];
  const double half = 0.5 * A.dt[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t e = c * A.n + i;
    const double vb = A.vbar[e];
    A.seeds[static_cast<int64_t>(c) * A.n_act + q] = A.abar[e] + half * vb;
    A.pbar[e] = A.rbar[e];
    A.abar[e] = half * vb;
    A.rbar[e] = 0.0;
  }
}

__global__ __launch_bounds__(kWG) void k_block_adj_predict(BlockAdjArgs A) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (j >= A.n) return;
  const double h = A.t_block - A.t_last[j];
  const double h2 = 0.5 * h * h;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t e = c * A.n + j;
    const double pb = A.pbar[e];
    A.rbar[e] += pb;
    A.vbar[e] += h * pb;
    A.abar[e] += h2 * pb;
  }
}

CorrectArgs base_args(tsbts_ctx *c) {
  CorrectArgs p;
  p.n = c->n;
  p.npad = c->npad;
  p.p64 = c->p64;
  p.v64 = c->v64;
  p.p32 = c->precision == TSBTS_MIXED ? c->p32 : nullptr;
  p.r = c->r;
  p.v = c->v;
  p.a = c->a;
  p.t_last = c->t_last;
  p.record = c->h.recording ? 1 : 0;
  p.base = c->h.count;
  p.cap = c->h.cap;
  p.pid = c->h.pid;
  p.rank = c->h.rank;
  p.cnt = c->h.cnt;
  p.rt = c->h.t;
  p.rs = c->h.s;
  p.tag = nullptr;
  p.step = 0;
  return p;
}

}  // namespace

CorrectArgs correct_args(tsbts_ctx *c, const int32_t *idx, int n_act, double t_block,
                         const double *acc_new) {
  CorrectArgs p = base_args(c);
  p.idx = idx;
  p.n_act = n_act;
  p.tb = t_block;
  p.acc_new = acc_new;
  return p;
}

hipError_t launch_correct(tsbts_ctx *c, const int32_t *idx, int n_act, double t_block,
                          const double *acc_new, hipStream_t st) {
  CorrectArgs p = correct_args(c, idx, n_act, t_block, acc_new);
  const int nb = (n_act + kWG - 1) / kWG;
  hipLaunchKernelGGL(k_correct, dim3(nb), dim3(kWG), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_history_begin(tsbts_ctx *c, hipStream_t st) {
  CorrectArgs p = base_args(c);
  const int nb = static_cast<int>((c->n + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_history_begin, dim3(nb), dim3(kWG), 0, st, p);
  return hipGetLastError();
}

static_assert(kScanTile == kScanCounts, "tile sums of launch_exclusive_scan");

hipError_t launch_exclusive_scan(const int32_t *cnt, int64_t n, int32_t *tsum, int32_t *off,
                                 int32_t *cur, hipStream_t st) {
  const int ntiles = static_cast<int>((n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_sums, dim3(ntiles), dim3(kScanWG), 0, st, cnt, n, tsum);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kScanWG), 0, st, cnt, n, tsum, off, cur);
  return hipGetLastError();
}

hipError_t launch_history_end(tsbts_ctx *c, hipStream_t st) {
  (void)launch_exclusive_scan(c->h.cnt, c->n, c->h.tsum, c->h.off, c->h.cur, st);
  ScatterArgs p;
  p.count = c->h.count;
  p.cap = c->h.cap;
  p.hcap = c->h.hcap;
  p.pid = c->h.pid;
  p.rank = c->h.rank;
  p.off = c->h.off;
  p.rt = c->h.t;
  p.rs = c->h.s;
  p.ht = c->h.ht;
  p.hs = c->h.hs;
  const int nb = static_cast<int>((c->h.count + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kWG), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_set_dt(tsbts_ctx *c, const int32_t *idx, int n_act, const double *dt_new,
                         hipStream_t st) {
  const int nb = (n_act + kWG - 1) / kWG;
  hipLaunchKernelGGL(k_set_dt, dim3(nb), dim3(kWG), 0, st, idx, n_act, dt_new, c->dt);
  return hipGetLastError();
}

hipError_t launch_leapfrog_adjoint(tsbts_ctx *c, int phase, double h, const double *rbar,
                                   double *vbar, double *abar, double *g_out,
                                   hipStream_t st) {
  const int64_t len = 3 * c->n;
  const int nb = static_cast<int>((len + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_lf_adjoint, dim3(nb), dim3(kWG), 0, st, len, phase, h, rbar, vbar,
                     abar, g_out);
  return hipGetLastError();
}

hipError_t launch_fill(double *x, int64_t len, double v, hipStream_t st) {
  if (len <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>((len + kWG - 1) / kWG)), dim3(kWG), 0,
                     st, len, x, v);
  return hipGetLastError();
}

hipError_t launch_block_adjoint(tsbts_ctx *c, int phase, const int32_t *idx, int n_act,
                                double t_block, double *rbar, double *vbar, double *abar,
                                double *pbar, double *seeds, hipStream_t st) {
  BlockAdjArgs A;
  A.n = c->n;
  A.idx = idx;
  A.n_act = n_act;
  A.t_block = t_block;
  A.dt = c->dt;
  A.t_last = c->t_last;
  A.rbar = rbar;
  A.vbar = vbar;
  A.abar = abar;
  A.pbar = pbar;
  A.seeds = seeds;
  if (phase == 0) {
    const int64_t len = 3 * c->n;
    hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>((len + kWG - 1) / kWG)), dim3(kWG),
                       0, st, len, pbar, 0.0);
    if (n_act > 0)
      hipLaunchKernelGGL(k_block_adj_active, dim3((n_act + kWG - 1) / kWG), dim3(kWG), 0, st,
                         A);
  } else {
    hipLaunchKernelGGL(k_block_adj_predict,
                       dim3(static_cast<unsigned>((c->n + kWG - 1) / kWG)), dim3(kWG), 0, st,
                       A);
  }
  return hipGetLastError();
}

}  // namespace tsbts
