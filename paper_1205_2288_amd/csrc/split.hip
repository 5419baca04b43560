// Force and time-step criterion of a large partial active set A (Algorithm 2, step 5, and
// Eq. nbdt: the active particles against all N) in two parts.  The pairs within A are
// evaluated once for both of their particles by the symmetric kernels on a compact copy
// of A; the pairs between A and the other particles I by the gather kernels, with a
// compact copy of I as the sources.  The gather kernels finish every target: the force
// adds the symmetric part's acceleration and potential after its own sums (a fixed order),
// the criterion takes the larger maximum and the smaller minimum (exact: the result equals
// the one-part gather's bit for bit); then the corrector runs as in the gather kernels.
// With half the particles active, a quarter of the target-source pairs is evaluated once
// instead of twice.
//
// Per call: marks of the particles outside A, their exclusive scan (positions in the
// copy of I, in particle order, so that the sums keep a fixed order), one copy kernel for
// both copies, the symmetric part (its work items written by a kernel), the gather part.
#include <algorithm>

#include "internal.hpp"
#include "predict.hpp"
#include "sym.hpp"

namespace tsbts {
namespace {

constexpr int64_t kSplitMinAct = 8192;    // targets, at least
constexpr int64_t kSplitAutoAct = 16384;  // automatic use from this many targets

// The split buffer for `cap` particles per copy.
struct SplitBufs {
  double *a64, *i64;  // [8][cap]: the 5 float64 planes of p64, then the 3 of v64
  float *a32, *i32;   // [12][cap]: the float32 planes
  double *sym;        // [4][cap]: symmetric part's acceleration (x, y, z) and potential;
                      // the criterion's maximum and minimum use its first two planes
  int32_t *mark;      // [cap]: 1 for a particle outside A
  int32_t *off;       // [cap + 1]: its position in the copy of I; off[n] = |I|
  int32_t *tsum;      // scan tile sums
  int32_t *iota;      // [cap]: 0, 1, 2, ... (the active list of the copy of A)
  int4 *items;        // [kSymMaxItems]: work items of the symmetric part
};

// Carve the buffer at `base` (or only count its bytes, base = null).
int64_t split_layout(int64_t cap, char *base, SplitBufs *b) {
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    char *p = base ? base + o : nullptr;
    o += (bytes + 255) / 256 * 256;
    return p;
  };
  b->a64 = reinterpret_cast<double *>(take(8 * cap * sizeof(double)));
  b->i64 = reinterpret_cast<double *>(take(8 * cap * sizeof(double)));
  b->a32 = reinterpret_cast<float *>(take(12 * cap * sizeof(float)));
  b->i32 = reinterpret_cast<float *>(take(12 * cap * sizeof(float)));
  b->sym = reinterpret_cast<double *>(take(4 * cap * sizeof(double)));
  b->mark = reinterpret_cast<int32_t *>(take(cap * sizeof(int32_t)));
  b->off = reinterpret_cast<int32_t *>(take((cap + 1) * sizeof(int32_t)));
  b->tsum = reinterpret_cast<int32_t *>(take((cap + kScanCounts - 1) / kScanCounts *
                                             sizeof(int32_t)));
  b->iota = reinterpret_cast<int32_t *>(take(cap * sizeof(int32_t)));
  b->items = reinterpret_cast<int4 *>(take(kSymMaxItems * sizeof(int4)));
  return o;
}

bool split_bufs(const tsbts_ctx *c, SplitBufs *b) {
  if (!c->split_buf || c->split_cap < c->npad) return false;
  split_layout(c->split_cap, static_cast<char *>(c->split_buf), b);
  return true;
}

__global__ __launch_bounds__(kWG) void k_split_iota(int64_t cap, int32_t *iota) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (t < cap) iota[t] = static_cast<int32_t>(t);
}

__global__ __launch_bounds__(kWG) void k_split_mark(int64_t n, int32_t *mark) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (t < n) mark[t] = 1;
}

__global__ __launch_bounds__(kWG) void k_split_unmark(const int32_t *idx, int k,
                                                      int32_t *mark) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q < k) mark[idx[q]] = 0;
}

struct CopyArgs {
  const double *p64, *v64;  // the predicted arrays
  const float *p32;
  int64_t npad;
  const int32_t *idx;
  int64_t k, ka, ki, n;
  const int32_t *mark, *off;
  Out qa, qi;  // the copies of A (ka particles) and of I (ki)
};

// Particle g's planes into position d of the copy o.
__device__ __forceinline__ void copy_record(const CopyArgs &a, const Out &o, int64_t g,
                                            int64_t d) {
  const int64_t P = a.npad, Q = o.npad;
#pragma unroll
  for (int c = 0; c < 5; ++c) o.p64[c * Q + d] = a.p64[c * P + g];
#pragma unroll
  for (int c = 0; c < 3; ++c) o.v64[c * Q + d] = a.v64[c * P + g];
  if (o.p32) {
#pragma unroll
    for (int c = 0; c < 12; ++c) o.p32[c * Q + d] = a.p32[c * P + g];
  }
}

// Thread t: position t of the copy of A (target t, or padding), particle t into the copy
// of I when it is outside A, and padding at position t of the copy of I past |I|.  A
// repeated active index makes |I| larger than n - k; the particles past the copy's ki
// positions are then dropped (the results are undefined for such lists, as for the
// symmetric kernels, but every access stays in bounds).
__global__ __launch_bounds__(kWG) void k_split_copy(CopyArgs a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (t < a.ka) {
    if (t < a.k)
      copy_record(a, a.qa, a.idx[t], t);
    else
      store_pad(a.qa, t);
  }
  if (t < a.n && a.mark[t]) {
    const int64_t d = a.off[t];
    if (d < a.ki) copy_record(a, a.qi, t, d);
  }
  if (t < a.ki && t >= a.off[a.n]) store_pad(a.qi, t);
}

// The sizes of a split call of k targets.
struct SplitShape {
  int64_t k, ka, ki;
};

SplitShape split_shape(const tsbts_ctx *c, int64_t k) {
  return SplitShape{k, round_up(k, 512), round_up(c->n - k, 512)};
}

// Marks, scan and copies for the active list idx; the copies as particle sets.
hipError_t launch_split_sets(tsbts_ctx *c, const SplitBufs &b, const SplitShape &sh,
                             const int32_t *idx, hipStream_t st, SymSet *set_a,
                             GatherSrc *src_i) {
  const int64_t n = c->n;
  hipLaunchKernelGGL(k_split_mark, dim3(static_cast<unsigned>((n + kWG - 1) / kWG)), dim3(kWG),
                     0, st, n, b.mark);
  hipLaunchKernelGGL(k_split_unmark, dim3(static_cast<unsigned>((sh.k + kWG - 1) / kWG)),
                     dim3(kWG), 0, st, idx, static_cast<int>(sh.k), b.mark);
  hipError_t e = launch_exclusive_scan(b.mark, n, b.tsum, b.off, b.off, st);
  if (e != hipSuccess) return e;
  CopyArgs a;
  a.p64 = c->p64;
  a.v64 = c->v64;
  a.p32 = c->p32;
  a.npad = c->npad;
  a.idx = idx;
  a.k = sh.k;
  a.ka = sh.ka;
  a.ki = sh.ki;
  a.n = n;
  a.mark = b.mark;
  a.off = b.off;
  const double eps2 = c->eps * c->eps;
  a.qa = Out{b.a64, b.a64 + 5 * sh.ka, c->p32 ? b.a32 : nullptr, sh.ka, eps2};
  a.qi = Out{b.i64, b.i64 + 5 * sh.ki, c->p32 ? b.i32 : nullptr, sh.ki, eps2};
  const int64_t threads = std::max<int64_t>(std::max(sh.ka, sh.ki), n);
  hipLaunchKernelGGL(k_split_copy, dim3(static_cast<unsigned>((threads + kWG - 1) / kWG)),
                     dim3(kWG), 0, st, a);
  *set_a = SymSet{sh.k, sh.ka, a.qa.p32, a.qa.p64, a.qa.v64};
  src_i->p32 = a.qi.p32;
  src_i->p64 = a.qi.p64;
  src_i->v64 = a.qi.v64;
  src_i->n = n - sh.k;
  src_i->npad = sh.ki;
  src_i->add = b.sym;
  return hipGetLastError();
}

int value_bytes(const tsbts_ctx *c) { return c->precision == TSBTS_FP64 ? 8 : 4; }

}  // namespace

bool split_applies(const tsbts_ctx *c, int64_t n_act) {
  if (c->tune_split == 0 || n_act >= c->n || n_act < kSplitMinAct) return false;
  if (c->tune_split == 2 && n_act < kSplitAutoAct) return false;
  // the symmetric force has no Newton-step form; the gather part is the scalar-load
  // kernel in its default shapes
  if ((c->flags & TSBTS_FLAG_NEWTON) || !force_scalar_j(c) || c->tune_chunk != 0) return false;
  return sym_set_bytes(round_up(n_act, 512), 4, 8, value_bytes(c)) <= kSymMaxBytes;
}

int split_prepare(tsbts_ctx *c, int64_t n_act) {
  if (!split_applies(c, n_act)) return TSBTS_OK;
  if (!c->split_buf || c->split_cap < c->npad) {
    SplitBufs b;
    const int64_t cap = c->npad;
    const int64_t bytes = split_layout(cap, nullptr, &b);
    (void)hipDeviceSynchronize();  // earlier launches may still use a smaller buffer
    if (c->split_buf) (void)hipFree(c->split_buf);
    c->split_buf = nullptr;
    c->split_cap = 0;
    if (hipMalloc(&c->split_buf, bytes) != hipSuccess) {
      (void)hipGetLastError();
      c->split_buf = nullptr;
      return TSBTS_ENOMEM;
    }
    split_layout(cap, static_cast<char *>(c->split_buf), &b);
    hipLaunchKernelGGL(k_split_iota, dim3(static_cast<unsigned>((cap + kWG - 1) / kWG)),
                       dim3(kWG), 0, 0, cap, b.iota);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      (void)hipFree(c->split_buf);
      c->split_buf = nullptr;
      return TSBTS_EHIP;
    }
    c->split_cap = cap;
  }
  const int64_t ka = round_up(n_act, 512);
  const int vb = value_bytes(c);
  return sym_reserve(c, std::max(sym_set_bytes(ka, 4, 8, vb), sym_set_bytes(ka, 2, vb, vb)));
}

hipError_t launch_force_split(tsbts_ctx *c, const int32_t *idx, int n_act, double *acc,
                              double *pot, hipStream_t st, const CorrectArgs *corr) {
  SplitBufs b;
  if (!split_bufs(c, &b)) return hipErrorNotReady;
  const SplitShape sh = split_shape(c, n_act);
  SymPlan plan;
  if (!sym_plan_set(c, sh.ka, 4, 8, value_bytes(c), b.items, st, &plan)) return hipErrorNotReady;
  SymSet set_a;
  GatherSrc src_i;
  hipError_t e = launch_split_sets(c, b, sh, idx, st, &set_a, &src_i);
  if (e != hipSuccess) return e;
  // pairs within A: acceleration [3][k], potential after it
  e = launch_force_sym(c, plan, b.iota, n_act, b.sym, pot ? b.sym + 3 * sh.k : nullptr, st,
                       nullptr, &set_a);
  if (e != hipSuccess) return e;
  // pairs with I, the symmetric part added as each target is finished (then corrected)
  return launch_force_gather(c, idx, n_act, acc, pot, c->part, c->tune_blocks, st, corr,
                             &src_i);
}

hipError_t launch_timestep_split(tsbts_ctx *c, const int32_t *idx, int n_act, double eta,
                                 double *dtc, hipStream_t st) {
  SplitBufs b;
  if (!split_bufs(c, &b)) return hipErrorNotReady;
  const SplitShape sh = split_shape(c, n_act);
  const int vb = value_bytes(c);
  SymPlan plan;
  if (!sym_plan_set(c, sh.ka, 2, vb, vb, b.items, st, &plan)) return hipErrorNotReady;
  // the copies are taken again: the corrector of the block step changes the velocities
  SymSet set_a;
  GatherSrc src_i;
  hipError_t e = launch_split_sets(c, b, sh, idx, st, &set_a, &src_i);
  if (e != hipSuccess) return e;
  // pairs within A: maximum and minimum [2][k], unfinished
  e = launch_timestep_sym(c, plan, b.iota, n_act, eta, nullptr, st, &set_a, b.sym);
  if (e != hipSuccess) return e;
  return launch_timestep_gather(c, idx, n_act, eta, dtc, st, &src_i);
}

}  // namespace tsbts
