// Host side of the symmetric all-targets kernels: work items and partial buffers.
#include <algorithm>
#include <new>
#include <vector>

#include "sym.hpp"

namespace tsbts {
namespace {

// Layout of the work items for npad particles: row groups per band, bands, column chunk.
struct SymShape {
  int n_groups, band_groups, n_bands, chunk, max_slots;
};

SymShape sym_shape(int64_t npad) {
  SymShape s;
  s.n_groups = static_cast<int>((npad + kSymGroupRows - 1) / kSymGroupRows);
  s.band_groups = (s.n_groups + kSymMaxBands - 1) / kSymMaxBands;
  s.n_bands = (s.n_groups + s.band_groups - 1) / s.band_groups;
  // about kSymTargetItems waves' worth of items over the upper triangle (a band has about
  // npad / (2 chunk) items on average), whole column tiles of 64, and at most
  // kSymMaxSlots chunks per band
  const int64_t items = kSymTargetItems / kSymWaves;
  const int64_t by_items = (s.n_bands * npad / 2 + items - 1) / items;
  const int64_t by_slots = (npad + kSymMaxSlots - 1) / kSymMaxSlots;
  int64_t chunk = std::max<int64_t>({64, by_items, by_slots});
  chunk = (chunk + 63) / 64 * 64;
  chunk = std::min<int64_t>(chunk, (npad + 63) / 64 * 64);
  s.chunk = static_cast<int>(chunk);
  s.max_slots = sym_slots(npad, 0, s.chunk);
  return s;
}

// Partial-buffer bytes for nv values per particle: row partials of row_bytes, column
// partials of col_bytes, then the staged float32 values and the inverse permutation.
int64_t sym_buffer_bytes(const SymShape &sh, int64_t npad, int nv, int row_bytes,
                         int col_bytes) {
  const int64_t npad_rows = static_cast<int64_t>(sh.n_groups) * kSymGroupRows;
  return (static_cast<int64_t>(sh.max_slots) * npad_rows * row_bytes +
          static_cast<int64_t>(sh.n_bands) * npad * col_bytes) * nv +
         npad * static_cast<int64_t>(4 * sizeof(float) + sizeof(int32_t));
}

}  // namespace

__global__ __launch_bounds__(kWG) void k_sym_inverse(const int32_t *idx, int n_act,
                                                     int32_t *inv) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q < n_act) inv[idx[q]] = q;
}

__global__ __launch_bounds__(kWG) void k_sym_inverse_clear(int64_t n, int32_t *inv) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (p < n) inv[p] = -1;
}

hipError_t launch_sym_inverse(const SymPlan &plan, const int32_t *idx, int n_act, int64_t n,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_sym_inverse_clear, dim3(static_cast<unsigned>((n + kWG - 1) / kWG)),
                     dim3(kWG), 0, st, n, plan.inv);
  hipLaunchKernelGGL(k_sym_inverse, dim3((n_act + kWG - 1) / kWG), dim3(kWG), 0, st, idx, n_act,
                     plan.inv);
  return hipGetLastError();
}

// Partial-buffer bytes for nv values per particle (float64 rows, col_bytes columns).
int64_t sym_bytes(int64_t npad, int nv, int col_bytes) {
  return sym_buffer_bytes(sym_shape(npad), npad, nv, 8, col_bytes);
}

bool sym_enabled(const tsbts_ctx *c, int64_t n_act) {
  if (n_act != c->n) return false;
  if (c->tune_sym == 0) return false;
  if (c->tune_sym == 1) return true;
  // automatic: from kSymMinN particles while the partials (at most kSymMaxSlots row and
  // kSymMaxBands column values per particle and value: about 6 KB per particle with four
  // values, 768 MB at N = 131072) stay within kSymMaxBytes (N up to about 5.6 million)
  const int cb = c->precision == TSBTS_FP64 ? 8 : 4;
  return c->n >= kSymMinN && sym_bytes(c->npad, 4, cb) <= kSymMaxBytes;
}

bool criterion_sym_applies(const tsbts_ctx *c, int64_t n_act) {
  return sym_enabled(c, n_act);
}

int sym_prepare(tsbts_ctx *c, int nv, int row_bytes, int col_bytes) {
  const int64_t npad = c->npad;
  const SymShape sh = sym_shape(npad);
  if (c->sym_items_npad != npad || c->sym_chunk != sh.chunk) {
    std::vector<int4> items;
    try {
      for (int b = 0; b < sh.n_bands; ++b) {
        const int64_t first = static_cast<int64_t>(b) * sh.band_groups * kSymGroupRows;
        int s = 0;
        for (int64_t j0 = first; j0 < npad; j0 += sh.chunk, ++s)
          items.push_back(make_int4(b, static_cast<int>(j0),
                                    static_cast<int>(std::min<int64_t>(j0 + sh.chunk, npad)),
                                    s));
      }
    } catch (const std::bad_alloc &) {  // no exception leaves the library
      return TSBTS_ENOMEM;
    }
    (void)hipDeviceSynchronize();  // earlier launches may still read the old list
    if (c->sym_items) (void)hipFree(c->sym_items);
    c->sym_items = nullptr;
    c->sym_items_n = 0;
    c->sym_items_npad = 0;
    if (hipMalloc(reinterpret_cast<void **>(&c->sym_items), items.size() * sizeof(int4)) !=
        hipSuccess) {
      (void)hipGetLastError();
      c->sym_items = nullptr;
      return TSBTS_ENOMEM;
    }
    if (hipMemcpy(c->sym_items, items.data(), items.size() * sizeof(int4),
                  hipMemcpyHostToDevice) != hipSuccess)
      return TSBTS_EHIP;
    c->sym_items_n = static_cast<int>(items.size());
    c->sym_items_npad = npad;
    c->sym_chunk = sh.chunk;
  }
  return sym_reserve(c, sym_buffer_bytes(sh, npad, nv, row_bytes, col_bytes));
}

int sym_reserve(tsbts_ctx *c, int64_t bytes) {
  if (bytes <= c->sym_part_bytes) return TSBTS_OK;
  // earlier launches may still use the old buffer
  (void)hipDeviceSynchronize();
  if (c->sym_part) (void)hipFree(c->sym_part);
  c->sym_part = nullptr;
  c->sym_part_bytes = 0;
  if (hipMalloc(&c->sym_part, bytes) != hipSuccess) {
    (void)hipGetLastError();
    c->sym_part = nullptr;
    return TSBTS_ENOMEM;
  }
  c->sym_part_bytes = bytes;
  return TSBTS_OK;
}

int64_t sym_set_bytes(int64_t npad, int nv, int row_bytes, int col_bytes) {
  return sym_buffer_bytes(sym_shape(npad), npad, nv, row_bytes, col_bytes);
}

namespace {

// The plan's shape and buffers for npad particles (items set by the caller).
bool plan_layout(const tsbts_ctx *c, int64_t npad, int nv, int row_bytes, int col_bytes,
                 SymPlan *p) {
  const SymShape sh = sym_shape(npad);
  const int64_t npad_rows = static_cast<int64_t>(sh.n_groups) * kSymGroupRows;
  const int64_t rows = static_cast<int64_t>(sh.max_slots) * npad_rows * nv * row_bytes;
  if (!c->sym_part || sym_buffer_bytes(sh, npad, nv, row_bytes, col_bytes) > c->sym_part_bytes)
    return false;
  p->n_groups = sh.n_groups;
  p->band_groups = sh.band_groups;
  p->n_bands = sh.n_bands;
  p->chunk = sh.chunk;
  p->max_slots = sh.max_slots;
  p->npad_rows = npad_rows;
  p->row_part = c->sym_part;
  p->col_part = static_cast<char *>(c->sym_part) + rows;
  // the staged values and the inverse permutation sit at the end of the buffer
  char *end = static_cast<char *>(c->sym_part) + c->sym_part_bytes;
  p->inv = reinterpret_cast<int32_t *>(end - npad * static_cast<int64_t>(sizeof(int32_t)));
  p->aux = reinterpret_cast<float *>(end - npad * static_cast<int64_t>(sizeof(int32_t) +
                                                                      4 * sizeof(float)));
  return true;
}

// Work item t of npad particles: the same list, in the same order, as sym_prepare builds
// on the host (bands in order, each band's column chunks in order).
__global__ __launch_bounds__(kWG) void k_sym_items(int4 *items, int n_items, int64_t npad,
                                                   int band_groups, int chunk) {
  const int t = blockIdx.x * kWG + threadIdx.x;
  if (t >= n_items) return;
  int b = 0, base = 0;
  int64_t first = 0;
  for (;;) {
    first = static_cast<int64_t>(b) * band_groups * kSymGroupRows;
    const int s = sym_slots(npad, first, chunk);
    if (t < base + s) break;
    base += s;
    ++b;
  }
  const int slot = t - base;
  const int64_t j0 = first + static_cast<int64_t>(slot) * chunk;
  items[t] = make_int4(b, static_cast<int>(j0), static_cast<int>(std::min<int64_t>(j0 + chunk,
                                                                                  npad)),
                       slot);
}

}  // namespace

bool sym_plan(const tsbts_ctx *c, int nv, int row_bytes, int col_bytes, SymPlan *p) {
  const int64_t npad = c->npad;
  if (!c->sym_items || c->sym_items_npad != npad) return false;
  if (sym_shape(npad).chunk != c->sym_chunk) return false;
  if (!plan_layout(c, npad, nv, row_bytes, col_bytes, p)) return false;
  p->items = static_cast<const int4 *>(c->sym_items);
  p->n_items = c->sym_items_n;
  return true;
}

bool sym_plan_set(const tsbts_ctx *c, int64_t npad, int nv, int row_bytes, int col_bytes,
                  int4 *items, hipStream_t st, SymPlan *p) {
  if (!plan_layout(c, npad, nv, row_bytes, col_bytes, p)) return false;
  const SymShape sh = sym_shape(npad);
  int n_items = 0;
  for (int b = 0; b < sh.n_bands; ++b)
    n_items += sym_slots(npad, static_cast<int64_t>(b) * sh.band_groups * kSymGroupRows,
                         sh.chunk);
  if (n_items > kSymMaxItems) return false;
  hipLaunchKernelGGL(k_sym_items, dim3((n_items + kWG - 1) / kWG), dim3(kWG), 0, st, items,
                     n_items, npad, sh.band_groups, sh.chunk);
  p->items = items;
  p->n_items = n_items;
  return true;
}

}  // namespace tsbts
