// Symmetric evaluation of the all-targets pair sums.
//
// When every particle is a target, each unordered pair {k, j} enters two rows: k's sum
// over j and j's sum over k, with the same separation, distance and reciprocal powers.
// The symmetric kernels evaluate each pair once.  The rows are cut into row groups of
// kSymGroupRows particles (four waves, each a row tile of kSymWaveRows, kSymRows per
// lane) and the row groups into at most kSymMaxBands bands of consecutive groups.  A
// workgroup work item is a band against a contiguous chunk of columns at or right of the
// band's first particle: it takes the band's row groups in order, each against the part
// of the chunk at or right of that group's first particle.  A lane accumulates the row
// side of its particles in registers and writes one row partial per (row, item).  The
// column side of each column j is combined over the lane's rows in registers, over the 64
// lanes through a wave-private LDS transposition of a few columns at a time, over the four
// waves through LDS in wave order, and over the band's row groups in order into one
// column partial per (band, column): the first row group writes it, the later ones add
// to it.  A reduction kernel combines, for each particle, the row partials of the items
// of its band that reach its row group, in slot order, and the column partials of the
// bands at or above it, in band order.  With at most kSymMaxBands bands and at most
// kSymMaxSlots chunks per band the partials take O(N) memory.  Pairs with j <= k (the
// diagonal block and, for a group's later waves, the columns left of their rows), padding
// rows and padding columns are masked (wave-uniform choice of the masked loop, as in the
// gather kernels).
#pragma once

#include "internal.hpp"

namespace tsbts {

constexpr int kSymRows = 4;                        // rows per lane
constexpr int kSymWaveRows = 64 * kSymRows;        // rows of one wave
constexpr int kSymWaves = kWG / 64;                // waves of a work item
constexpr int kSymGroupRows = kSymWaves * kSymWaveRows;  // rows of one work item
constexpr int kSymBlock = 16;                      // columns per LDS transposition
constexpr int kSymLdsStride = 65;                  // LDS entries per column (one pad)
constexpr int kSymMinN = 32768;                    // automatic use from this many particles
constexpr int kSymTargetItems = 32768;             // waves aimed at by the column chunk
constexpr int kSymMaxBands = 128;                  // bands of row groups, at most
constexpr int kSymMaxSlots = 128;                  // column chunks of a band, at most
constexpr int64_t kSymMaxBytes = int64_t(32) << 30; // automatic use while partials fit this

struct SymPlan {
  const int4 *items;  // (band, first column, end column, slot of the band)
  int n_items;
  int n_groups;       // row groups of kSymGroupRows
  int band_groups;    // row groups per band
  int n_bands;
  int chunk;          // columns per work item (multiple of 64)
  int max_slots;      // items of band 0 (the most of any band)
  int64_t npad_rows;  // n_groups * kSymGroupRows
  void *row_part;     // [max_slots][NV][npad_rows]
  void *col_part;     // [n_bands][NV][npad]
  float *aux;         // [4][npad]: per-particle float32 values a kernel stages (seeds)
  int32_t *inv;       // [npad]: position of each particle in the active list
};

// inv[idx[q]] = q, -1 for particles not in the list (a list with repeated entries): the
// reductions run over particles in order (coalesced partial reads) and write each result
// to its place in the active list.
hipError_t launch_sym_inverse(const SymPlan &plan, const int32_t *idx, int n_act, int64_t n,
                              hipStream_t st);

// Work items of a band whose first row is `first`: its columns [first, npad) in chunks.
__host__ __device__ inline int sym_slots(int64_t npad, int64_t first, int chunk) {
  return static_cast<int>((npad - first + chunk - 1) / chunk);
}

// Row particle p of a plan: its band, and the slots [s0, s1) of the band's items that
// reach its row group (the chunks not wholly left of the group's first particle).
__host__ __device__ inline void sym_row_slots(const SymPlan &plan, int64_t npad, int64_t p,
                                              int &band, int &s0, int &s1) {
  const int64_t g = p / kSymGroupRows;
  band = static_cast<int>(g / plan.band_groups);
  const int64_t first = static_cast<int64_t>(band) * plan.band_groups * kSymGroupRows;
  s0 = static_cast<int>((g * kSymGroupRows - first) / plan.chunk);
  s1 = sym_slots(npad, first, plan.chunk);
}

// The row groups of a work item, in order: g runs over the item's band; the group takes
// columns [max(first column, its first particle), end column) and stops the item when
// that range is empty.
struct SymSub {
  int64_t grow0;  // first particle of the row group
  int64_t j0;     // first column
};
__device__ __forceinline__ bool sym_sub(const SymPlan &plan, const int4 &it, int sub,
                                        SymSub &out) {
  const int g = it.x * plan.band_groups + sub;
  if (sub >= plan.band_groups || g >= plan.n_groups) return false;
  out.grow0 = static_cast<int64_t>(g) * kSymGroupRows;
  if (out.grow0 >= it.z) return false;
  out.j0 = out.grow0 > it.y ? out.grow0 : it.y;
  return true;
}

// The four waves' column values of one transposition block (lanes < BLK of each wave hold
// those of column jb + lane) are combined through LDS in wave order by the first wave and
// stored to dst[v * stride + lane].  xs is double-buffered: one workgroup barrier per block
// keeps a wave from overwriting a buffer the first wave still reads.
// With acc, the result is combined (op) with the value already at dst: the column
// partial of an earlier row group of the same band, written by this same lane.
template <int BLK, int NV, class T, class Op>
__device__ __forceinline__ void sym_group_store(T (&xs)[2][kSymWaves][NV][BLK], int &buf,
                                                int wv, int lane, const T (&cs)[NV],
                                                T *dst, int64_t stride, Op op, bool acc) {
  if (lane < BLK) {
#pragma unroll
    for (int v = 0; v < NV; ++v) xs[buf][wv][v][lane] = cs[v];
  }
  __syncthreads();
  if (wv == 0 && lane < BLK) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T t = xs[buf][0][v][lane];
#pragma unroll
      for (int w = 1; w < kSymWaves; ++w) t = op(t, xs[buf][w][v][lane]);
      dst[v * stride + lane] = acc ? op(dst[v * stride + lane], t) : t;
    }
  }
  buf ^= 1;
}

// Make the LDS writes of this wave visible to its other lanes and keep the compiler from
// moving LDS accesses across this point (LDS operations of one wave execute in order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Column sums of one transposition block: L holds, for each of the BLK columns c, the
// NV values of every lane at (c * kSymLdsStride + lane) * NV.  Lane l adds the BLK
// entries of column l % BLK in part l / BLK, then the parts are added across lanes; lanes
// l < BLK return column l's sums (in this fixed order).
template <int BLK, int NV, class T>
__device__ __forceinline__ void sym_col_sums(const T *L, int lane, T out[NV]) {
  const int c = lane % BLK, part = lane / BLK;
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = T(0);
#pragma unroll
  for (int i = 0; i < BLK; ++i) {
    const T *e = L + (c * kSymLdsStride + part * BLK + i) * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] += e[v];
  }
#pragma unroll
  for (int off = BLK; off < 64; off <<= 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] += __shfl_xor(out[v], off, 64);
  }
}

// Add, for one particle, its partials of NV values at plane stride `stride` (value v of
// entry e at x[(NS * e + v) * stride]) for entries e in [e0, e1) into t, in entry order.
// The loads of kSymBatch entries are issued before their additions (the reductions are
// bound by reading the partials; one load in flight at a time would leave most of the
// memory system idle).
constexpr int kSymBatch = 8;
template <int NS, int NV, class T>
__device__ __forceinline__ void sym_sum_partials(const T *x, int64_t stride, int e0, int e1,
                                                 double *t) {
  const T *q = x + static_cast<int64_t>(NS) * e0 * stride;
  int e = e0;
  for (; e + kSymBatch <= e1; e += kSymBatch, q += NS * kSymBatch * stride) {
    T y[kSymBatch][NV];
#pragma unroll
    for (int b = 0; b < kSymBatch; ++b)
#pragma unroll
      for (int v = 0; v < NV; ++v) y[b][v] = q[(NS * b + v) * stride];
#pragma unroll
    for (int b = 0; b < kSymBatch; ++b)
#pragma unroll
      for (int v = 0; v < NV; ++v) t[v] += static_cast<double>(y[b][v]);
  }
  for (; e < e1; ++e, q += NS * stride)
#pragma unroll
    for (int v = 0; v < NV; ++v) t[v] += static_cast<double>(q[v * stride]);
}

// Whether the symmetric criterion serves the call (as sym_enabled).
bool criterion_sym_applies(const tsbts_ctx *c, int64_t n_act);
// Whether the symmetric kernels serve a call with n_act targets (all particles).
bool sym_enabled(const tsbts_ctx *c, int64_t n_act);
// Items and partial buffers for NV values per particle, row partials of row_bytes and
// column partials of col_bytes bytes per value: allocates (host set-up, synchronous) and
// returns a status.
int sym_prepare(tsbts_ctx *c, int nv, int row_bytes, int col_bytes);
// The plan if sym_prepare has provided for these sizes; false otherwise (no allocation).
bool sym_plan(const tsbts_ctx *c, int nv, int row_bytes, int col_bytes, SymPlan *plan);

// A particle set other than the context's predicted arrays (the compact copy of the
// active particles of a split call): n particles padded to npad (a multiple of 512),
// planes laid out as the predicted arrays with stride npad.
struct SymSet {
  int64_t n, npad;
  const float *p32;   // [12][npad] or null (float64 mode)
  const double *p64;  // [5][npad]
  const double *v64;  // [3][npad]
};
// Work items of a set of npad particles, at most this many.
constexpr int kSymMaxItems = kSymMaxBands * kSymMaxSlots;
// Partial-buffer bytes the symmetric kernels need for a set of npad particles.
int64_t sym_set_bytes(int64_t npad, int nv, int row_bytes, int col_bytes);
// Grow the context's partial buffer to at least `bytes` (host set-up, synchronous);
// returns a status.
int sym_reserve(tsbts_ctx *c, int64_t bytes);
// The plan for a set of npad particles: its work items written by a kernel on `st` into
// `items` (kSymMaxItems entries), its partials in the context's buffer; false when that
// buffer is too small (no allocation, nothing launched).
bool sym_plan_set(const tsbts_ctx *c, int64_t npad, int nv, int row_bytes, int col_bytes,
                  int4 *items, hipStream_t st, SymPlan *plan);

}  // namespace tsbts
