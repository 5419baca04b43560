// Host side of the symmetric all-targets kernels: work items and partial buffers.
#include <algorithm>
#include <vector>

#include "sym.hpp"

namespace tsbts {
namespace {

int sym_chunk(int64_t npad) {
  const int64_t n_groups = (npad + kSymGroupRows - 1) / kSymGroupRows;
  // about kSymTargetItems waves' worth of items over the upper triangle, whole column tiles
  // of 64
  const int64_t waves = kSymTargetItems / kSymWaves;
  const int64_t cols = (npad * n_groups / 2 + waves - 1) / waves;
  int64_t chunk = std::max<int64_t>(64, (cols + 63) / 64 * 64);
  chunk = std::min<int64_t>(chunk, (npad + 63) / 64 * 64);
  return static_cast<int>(chunk);
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
  const int chunk = sym_chunk(npad);
  const int64_t n_groups = (npad + kSymGroupRows - 1) / kSymGroupRows;
  const int64_t npad_rows = n_groups * kSymGroupRows;
  const int64_t max_slots = sym_slots(npad, 0, chunk);
  return (max_slots * npad_rows * 8 + n_groups * npad * col_bytes) * nv +
         npad * static_cast<int64_t>(4 * sizeof(float) + sizeof(int32_t));
}

bool sym_enabled(const tsbts_ctx *c, int64_t n_act) {
  if (n_act != c->n) return false;
  if (c->tune_sym == 0) return false;
  if (c->tune_sym == 1) return true;
  // automatic: from kSymMinN particles while the partials (which grow as N^2 / 256 column
  // sums) stay within kSymMaxBytes
  const int cb = c->precision == TSBTS_FP64 ? 8 : 4;
  return c->n >= kSymMinN && sym_bytes(c->npad, 4, cb) <= kSymMaxBytes;
}

bool criterion_sym_applies(const tsbts_ctx *c, int64_t n_act) {
  return sym_enabled(c, n_act);
}

int sym_prepare(tsbts_ctx *c, int nv, int row_bytes, int col_bytes) {
  const int64_t npad = c->npad;
  const int chunk = sym_chunk(npad);
  const int n_groups = static_cast<int>((npad + kSymGroupRows - 1) / kSymGroupRows);
  if (c->sym_items_npad != npad || c->sym_chunk != chunk) {
    std::vector<int4> items;
    for (int g = 0; g < n_groups; ++g) {
      int s = 0;
      for (int64_t j0 = static_cast<int64_t>(g) * kSymGroupRows; j0 < npad; j0 += chunk, ++s)
        items.push_back(make_int4(g, static_cast<int>(j0),
                                  static_cast<int>(std::min<int64_t>(j0 + chunk, npad)), s));
    }
    if (c->sym_items) (void)hipFree(c->sym_items);
    c->sym_items = nullptr;
    c->sym_items_n = 0;
    c->sym_items_npad = 0;
    if (hipMalloc(reinterpret_cast<void **>(&c->sym_items), items.size() * sizeof(int4)) !=
        hipSuccess) {
      c->sym_items = nullptr;
      return TSBTS_ENOMEM;
    }
    if (hipMemcpy(c->sym_items, items.data(), items.size() * sizeof(int4),
                  hipMemcpyHostToDevice) != hipSuccess)
      return TSBTS_EHIP;
    c->sym_items_n = static_cast<int>(items.size());
    c->sym_items_npad = npad;
    c->sym_chunk = chunk;
  }
  const int64_t npad_rows = static_cast<int64_t>(n_groups) * kSymGroupRows;
  const int max_slots = sym_slots(npad, 0, chunk);
  const int64_t bytes = (static_cast<int64_t>(max_slots) * npad_rows * row_bytes +
                         static_cast<int64_t>(n_groups) * npad * col_bytes) * nv +
                        npad * static_cast<int64_t>(4 * sizeof(float) + sizeof(int32_t));
  if (bytes > c->sym_part_bytes) {
    (void)hipDeviceSynchronize();
    if (c->sym_part) (void)hipFree(c->sym_part);
    c->sym_part = nullptr;
    c->sym_part_bytes = 0;
    if (hipMalloc(&c->sym_part, bytes) != hipSuccess) {
      c->sym_part = nullptr;
      return TSBTS_ENOMEM;
    }
    c->sym_part_bytes = bytes;
  }
  return TSBTS_OK;
}

bool sym_plan(const tsbts_ctx *c, int nv, int row_bytes, int col_bytes, SymPlan *p) {
  const int64_t npad = c->npad;
  if (!c->sym_items || c->sym_items_npad != npad) return false;
  const int n_groups = static_cast<int>((npad + kSymGroupRows - 1) / kSymGroupRows);
  const int64_t npad_rows = static_cast<int64_t>(n_groups) * kSymGroupRows;
  const int max_slots = sym_slots(npad, 0, c->sym_chunk);
  const int64_t rows = static_cast<int64_t>(max_slots) * npad_rows * nv * row_bytes;
  const int64_t cols = static_cast<int64_t>(n_groups) * npad * nv * col_bytes;
  const int64_t bytes = rows + cols + npad * static_cast<int64_t>(4 * sizeof(float) +
                                                                 sizeof(int32_t));
  if (bytes > c->sym_part_bytes) return false;
  p->items = static_cast<const int4 *>(c->sym_items);
  p->n_items = c->sym_items_n;
  p->n_groups = n_groups;
  p->chunk = c->sym_chunk;
  p->max_slots = max_slots;
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

}  // namespace tsbts
