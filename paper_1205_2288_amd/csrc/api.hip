// C-ABI entry points of libtsbts (declared and documented in include/tsbts.h): context
// lifecycle, host-side argument validation, scratch management and error reporting.  All
// arithmetic happens in the kernels of the other files.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "correct.hpp"
#include "predict.hpp"
#include "sym.hpp"

namespace tsbts {
int64_t backward_partials_needed(const tsbts_ctx *c, int n_act);
}

using namespace tsbts;

namespace {

int fail(tsbts_ctx *c, int status, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return status;
}

int hip_fail(tsbts_ctx *c, hipError_t e, const char *what) {
  return fail(c, TSBTS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define TSBTS_CHECK_HIP(ctx, expr)                              \
  do {                                                          \
    hipError_t _e = (expr);                                     \
    if (_e != hipSuccess) return hip_fail((ctx), _e, #expr);    \
  } while (0)

template <class T>
int dev_alloc(tsbts_ctx *c, T **p, int64_t count) {
  *p = nullptr;
  if (count <= 0) return TSBTS_OK;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * static_cast<size_t>(count));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(c, TSBTS_ENOMEM, "hipMalloc of %lld bytes failed: %s",
                static_cast<long long>(sizeof(T) * count), hipGetErrorString(e));
  }
  return TSBTS_OK;
}

template <class T>
void dev_free(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

int check_ctx(const tsbts_ctx *c) { return c ? TSBTS_OK : TSBTS_EINVAL; }

__global__ __launch_bounds__(kWG) void k_zero_i32(int32_t *x, int64_t len) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (k < len) x[k] = 0;
}

// Flags an active index outside [0, n) in flag[0] and an index that occurs more than once
// in flag[1] (seen: n counters, zero on entry).
__global__ __launch_bounds__(kWG) void k_check_idx(const int32_t *idx, int32_t n_act, int64_t n,
                                                   int32_t *seen, int *flag) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (k < n_act) {
    const int32_t v = idx[k];
    if (v < 0 || v >= n)
      flag[0] = 1;
    else if (atomicAdd(&seen[v], 1) != 0)
      flag[1] = 1;
  }
}

int check_active(tsbts_ctx *c, const int32_t *idx, int32_t n_act, hipStream_t stream) {
  if (!idx) return fail(c, TSBTS_EINVAL, "active_idx is NULL");
  if (n_act < 1 || n_act > c->n)
    return fail(c, TSBTS_EINVAL, "n_active=%d outside [1, %lld]", n_act,
                static_cast<long long>(c->n));
  if (c->check_idx) {
    // every earlier use of the flags ended with a synchronisation, so they are free here
    c->idx_flag_h[0] = c->idx_flag_h[1] = 0;
    hipLaunchKernelGGL(k_zero_i32, dim3((c->n + kWG - 1) / kWG), dim3(kWG), 0, stream,
                       c->idx_seen, c->n);
    hipLaunchKernelGGL(k_check_idx, dim3((n_act + kWG - 1) / kWG), dim3(kWG), 0, stream, idx,
                       n_act, c->n, c->idx_seen, c->idx_flag_d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(c, e, "active index check");
    if (c->idx_flag_h[0])
      return fail(c, TSBTS_EINVAL, "active_idx holds an index outside [0, %lld)",
                  static_cast<long long>(c->n));
    if (c->idx_flag_h[1]) return fail(c, TSBTS_EINVAL, "active_idx repeats an index");
  }
  return TSBTS_OK;
}

int check_bound(tsbts_ctx *c) {
  if (!c->r || !c->v || !c->a || !c->m || !c->t_last || !c->dt)
    return fail(c, TSBTS_ESTATE, "no particle state bound (call tsbts_bind_state)");
  return TSBTS_OK;
}

// Work list and partials of the symmetric all-targets force, when it serves the call,
// and the buffers of a split call.
int prepare_force_sym(tsbts_ctx *c, int32_t n_act) {
  if (int s = split_prepare(c, n_act))
    return fail(c, s, "split call: buffers not allocated");
  if (!force_sym_applies(c, n_act)) return TSBTS_OK;
  if (int s = sym_prepare(c, 4, 8, c->precision == TSBTS_FP64 ? 8 : 4))
    return fail(c, s, "symmetric force: work list or partials not allocated");
  return TSBTS_OK;
}

int check_pred(tsbts_ctx *c, double t_block) {
  if (!c->have_pred) return fail(c, TSBTS_ESTATE, "no predicted particle arrays");
  if (c->pred_t != t_block)
    return fail(c, TSBTS_ESTATE, "t_block=%.17g differs from the predicted time %.17g",
                t_block, c->pred_t);
  return TSBTS_OK;
}

// Grow the split-j partial buffer to at least `need` float64 elements (synchronous).
int ensure_part(tsbts_ctx *c, int64_t need) {
  if (need <= c->part_cap) return TSBTS_OK;
  TSBTS_CHECK_HIP(c, hipDeviceSynchronize());
  const int64_t cap = std::max<int64_t>(need, c->part_cap * 2);
  dev_free(c->part);
  c->part_cap = 0;
  int st = dev_alloc(c, &c->part, cap);
  if (st) return st;
  c->part_cap = cap;
  return TSBTS_OK;
}

// Grow the era log to at least `need` records, preserving the `count` records appended
// so far.  Every new buffer is allocated before anything changes: on a failed allocation
// the log keeps its old buffers, capacity and contents.
int grow_log(tsbts_ctx *c, int64_t need, hipStream_t st) {
  History &h = c->h;
  if (need <= h.cap) return TSBTS_OK;
  const int64_t cap = std::max<int64_t>(need, h.cap + h.cap / 2 + 1024);
  double *ns = nullptr, *nt = nullptr;
  int32_t *np = nullptr, *nr = nullptr;
  int s = dev_alloc(c, &ns, cap * kHistPlanes);
  if (!s) s = dev_alloc(c, &nt, cap);
  if (!s) s = dev_alloc(c, &np, cap);
  if (!s) s = dev_alloc(c, &nr, cap);
  if (s) {
    dev_free(ns);
    dev_free(nt);
    dev_free(np);
    dev_free(nr);
    return s;
  }
  hipError_t e = hipSuccess;
  if (h.count > 0) {
    const size_t used = static_cast<size_t>(h.count);
    for (int p = 0; p < kHistPlanes && e == hipSuccess; ++p)
      e = hipMemcpyAsync(ns + p * cap, h.s + p * h.cap, used * sizeof(double),
                         hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(nt, h.t, used * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(np, h.pid, used * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(nr, h.rank, used * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
  }
  // earlier kernels may still read the old buffers, and the copies must land: wait
  // before freeing them
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    dev_free(ns);
    dev_free(nt);
    dev_free(np);
    dev_free(nr);
    return hip_fail(c, e, "era log growth");
  }
  dev_free(h.s);
  dev_free(h.t);
  dev_free(h.pid);
  dev_free(h.rank);
  h.s = ns;
  h.t = nt;
  h.pid = np;
  h.rank = nr;
  h.cap = cap;
  return TSBTS_OK;
}

}  // namespace

extern "C" {

int tsbts_version(void) { return 10000; }

const char *tsbts_strerror(int status) {
  switch (status) {
    case TSBTS_OK: return "ok";
    case TSBTS_EINVAL: return "invalid argument";
    case TSBTS_ENOMEM: return "device memory allocation failed";
    case TSBTS_EHIP: return "HIP runtime error";
    case TSBTS_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

const char *tsbts_last_error(const tsbts_ctx *ctx) { return ctx ? ctx->err : "null context"; }

int tsbts_create(tsbts_ctx **out, int64_t n, double eps, int precision, int flags) {
  if (!out) return TSBTS_EINVAL;
  *out = nullptr;
  if (n < 1 || n > (int64_t(1) << 30)) return TSBTS_EINVAL;
  if (!(eps >= 0.0) || !std::isfinite(eps)) return TSBTS_EINVAL;
  if (precision != TSBTS_FP64 && precision != TSBTS_MIXED) return TSBTS_EINVAL;
  if (flags & ~(TSBTS_FLAG_HILO_SEPARATION | TSBTS_FLAG_NEWTON)) return TSBTS_EINVAL;
  tsbts_ctx *c = new (std::nothrow) tsbts_ctx();
  if (!c) return TSBTS_ENOMEM;
  c->n = n;
  c->npad = round_up(n, kPad);
  c->eps = eps;
  c->precision = precision;
  c->flags = flags;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return TSBTS_EHIP;
  }
  // the fixed partial-sum array of tsbts_force_noalloc on this device (once per device)
  if (noalloc_setup(c->device) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return TSBTS_EHIP;
  }
  int st = TSBTS_OK;
  if (!st) st = dev_alloc(c, &c->p64, P64_PLANES * c->npad);
  if (!st) st = dev_alloc(c, &c->v64, 3 * c->npad);
  if (!st && precision == TSBTS_MIXED) st = dev_alloc(c, &c->p32, P32_PLANES * c->npad);
  if (!st) st = dev_alloc(c, &c->gord, 4 * c->npad);
  if (!st) st = dev_alloc(c, &c->h.cnt, n);
  if (!st) st = dev_alloc(c, &c->h.tsum, (n + 8191) / 8192);
  if (!st) st = dev_alloc(c, &c->h.off, n + 1);
  if (!st) st = dev_alloc(c, &c->h.cur, n);
  if (!st) st = dev_alloc(c, &c->done, 2);
  // zero before any launch on any of the caller's streams (which may not wait for the
  // null stream)
  if (!st && (hipMemset(c->done, 0, 2 * sizeof(uint32_t)) != hipSuccess ||
              hipDeviceSynchronize() != hipSuccess)) {
    (void)hipGetLastError();
    st = TSBTS_EHIP;
  }
  if (!st) {
    c->epart_cap = energy_partials_needed(c);
    st = dev_alloc(c, &c->epart, c->epart_cap);
  }
  if (!st) {
    const int64_t need = std::max({partial_elems_needed(c, static_cast<int>(n)),
                                   backward_partials_needed(c, static_cast<int>(n)),
                                   fused_partials_needed(c, static_cast<int>(n))});
    st = ensure_part(c, need);
  }
  if (st) {
    tsbts_destroy(c);
    return st;
  }
  *out = c;
  return TSBTS_OK;
}

int tsbts_destroy(tsbts_ctx *c) {
  if (!c) return TSBTS_OK;
  (void)hipDeviceSynchronize();
  destroy_scheduler(c);
  dev_free(c->p64);
  dev_free(c->v64);
  dev_free(c->p32);
  dev_free(c->part);
  dev_free(c->epart);
  dev_free(c->gord);
  if (c->sym_items) (void)hipFree(c->sym_items);
  if (c->sym_part) (void)hipFree(c->sym_part);
  if (c->split_buf) (void)hipFree(c->split_buf);
  if (c->idx_flag_h) (void)hipHostFree(c->idx_flag_h);
  dev_free(c->idx_seen);
  dev_free(c->done);
  dev_free(c->h.pid);
  dev_free(c->h.rank);
  dev_free(c->h.t);
  dev_free(c->h.s);
  dev_free(c->h.ht);
  dev_free(c->h.hs);
  dev_free(c->h.off);
  dev_free(c->h.cur);
  dev_free(c->h.cnt);
  dev_free(c->h.tsum);
  delete c;
  return TSBTS_OK;
}

int tsbts_tune(tsbts_ctx *c, int param, int value) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  switch (param) {
    case TSBTS_TUNE_BLOCKS:
      if (value < 64 || value > 65536) return fail(c, TSBTS_EINVAL, "blocks outside [64, 65536]");
      c->tune_blocks = value;
      return TSBTS_OK;
    case TSBTS_TUNE_IPL:
      if (value != 0 && value != 1 && value != 2 && value != 4)
        return fail(c, TSBTS_EINVAL, "targets per lane must be 0, 1, 2 or 4");
      c->tune_ipl = value;
      return TSBTS_OK;
    case TSBTS_TUNE_CHUNK:
      if (value != 0 && value != 64 && value != 256)
        return fail(c, TSBTS_EINVAL, "j chunk must be 0, 64 or 256");
      c->tune_chunk = value;
      return TSBTS_OK;
    case TSBTS_TUNE_SYMMETRIC:
      if (value < 0 || value > 2) return fail(c, TSBTS_EINVAL, "symmetric must be 0, 1 or 2");
      c->tune_sym = value;
      return TSBTS_OK;
    case TSBTS_TUNE_SPLIT:
      if (value < 0 || value > 2) return fail(c, TSBTS_EINVAL, "split must be 0, 1 or 2");
      c->tune_split = value;
      return TSBTS_OK;
    case TSBTS_TUNE_CHECK_INDICES:
      if (value != 0 && value != 1) return fail(c, TSBTS_EINVAL, "check must be 0 or 1");
      if (value && !c->idx_flag_h) {
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&c->idx_flag_h), 2 * sizeof(int));
        if (e == hipSuccess)
          e = hipHostGetDevicePointer(reinterpret_cast<void **>(&c->idx_flag_d), c->idx_flag_h,
                                      0);
        if (e == hipSuccess)
          e = hipMalloc(reinterpret_cast<void **>(&c->idx_seen), sizeof(int32_t) * c->n);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          if (c->idx_flag_h) (void)hipHostFree(c->idx_flag_h);
  dev_free(c->idx_seen);
          c->idx_flag_h = nullptr;
          c->idx_flag_d = nullptr;
          c->idx_seen = nullptr;
          return hip_fail(c, e, "index check buffers");
        }
      }
      c->check_idx = value;
      return TSBTS_OK;
    default:
      return fail(c, TSBTS_EINVAL, "unknown tuning parameter %d", param);
  }
}

int tsbts_bind_state(tsbts_ctx *c, double *r, double *v, double *a, const double *m,
                     double *t_last, double *dt) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (!r || !v || !a || !m || !t_last || !dt)
    return fail(c, TSBTS_EINVAL, "tsbts_bind_state: NULL array");
  c->r = r;
  c->v = v;
  c->a = a;
  c->m = m;
  c->t_last = t_last;
  c->dt = dt;
  c->have_pred = false;
  return TSBTS_OK;
}

int tsbts_predict(tsbts_ctx *c, double t_block, int use_history, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (!std::isfinite(t_block)) return fail(c, TSBTS_EINVAL, "t_block is not finite");
  if (use_history && !c->h.valid)
    return fail(c, TSBTS_ESTATE, "use_history requested without a finished history");
  hipError_t e = launch_predict(c, t_block, use_history ? 1 : 0, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_predict launch");
  c->pred_t = t_block;
  c->have_pred = true;
  return TSBTS_OK;
}

}  // extern "C"

namespace tsbts {

int predict_pending(tsbts_ctx *c, double t_block, int use_history, const PendingSteps *pend,
                    const InlineIdx *in, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (!std::isfinite(t_block)) return fail(c, TSBTS_EINVAL, "t_block is not finite");
  if (use_history && !c->h.valid)
    return fail(c, TSBTS_ESTATE, "use_history requested without a finished history");
  if (in && in->k > 0 && (in->k > kInlineIdx || !in->out))
    return fail(c, TSBTS_EINVAL, "inline active list larger than %d or without a target",
                kInlineIdx);
  hipError_t e = launch_predict(c, t_block, use_history ? 1 : 0, stream, pend, in);
  if (e != hipSuccess) return hip_fail(c, e, "predict launch");
  c->pred_t = t_block;
  c->have_pred = true;
  return TSBTS_OK;
}

}  // namespace tsbts

extern "C" {

int tsbts_load_positions(tsbts_ctx *c, const double *r, const double *m, double t_label,
                         hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (!r || !m) return fail(c, TSBTS_EINVAL, "tsbts_load_positions: NULL array");
  // the kernel also zeroes the velocity planes, so tsbts_timestep sees a defined state
  hipError_t e = launch_load_positions(c, r, m, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_load_positions launch");
  c->pred_t = t_label;
  c->have_pred = true;
  return TSBTS_OK;
}

int tsbts_force(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block, double *acc,
                double *pot, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!acc) return fail(c, TSBTS_EINVAL, "acc is NULL");
  if (int s = check_pred(c, t_block)) return s;
  if (int s = ensure_part(c, partial_elems_needed(c, n_act))) return s;
  if (int s = prepare_force_sym(c, n_act)) return s;
  hipError_t e = launch_force(c, idx, n_act, acc, pot, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_force launch");
  return TSBTS_OK;
}

int tsbts_force_noalloc(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                        double *acc, double *pot, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!acc) return fail(c, TSBTS_EINVAL, "acc is NULL");
  if (int s = check_pred(c, t_block)) return s;
  double *part = noalloc_partials(c->device);
  if (!part)
    return fail(c, TSBTS_ESTATE, "tsbts_force_noalloc: no fixed partial array on device %d",
                c->device);
  // tsbts_force's split when its partials fit the array, else fewer workgroups
  int blocks = c->tune_blocks;
  int64_t need = force_partial_elems(c, n_act, blocks);
  while (need > TSBTS_NOALLOC_PARTIALS && blocks > 64) {
    blocks = std::max(64, blocks / 2);
    need = force_partial_elems(c, n_act, blocks);
  }
  if (need > TSBTS_NOALLOC_PARTIALS)
    return fail(c, TSBTS_EINVAL,
                "tsbts_force_noalloc: the call needs %lld partial sums, more than the fixed "
                "array's %lld (n_active <= %d needs 4 * n_active per 256 particles)",
                static_cast<long long>(need), static_cast<long long>(TSBTS_NOALLOC_PARTIALS),
                small_act_limit(c));
  hipError_t e = launch_force_gather(c, idx, n_act, acc, pot, part, blocks, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_force_noalloc launch");
  return TSBTS_OK;
}

int tsbts_force_criterion(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                          double eta, double *acc, double *pot, double *dtc,
                          hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!acc || !dtc) return fail(c, TSBTS_EINVAL, "acc or dtc is NULL");
  if (!(eta > 0.0) || !std::isfinite(eta)) return fail(c, TSBTS_EINVAL, "eta must be > 0");
  if (int s = check_pred(c, t_block)) return s;
  hipError_t e;
  if (n_act <= kSmallAct) {
    // small sets: the j-parallel criterion and force kernels, criterion first, on the same
    // predicted state (same definition as the fused pass, fewer idle lanes)
    if (int s = ensure_part(c, partial_elems_needed(c, n_act))) return s;
    e = launch_timestep(c, idx, n_act, eta, dtc, stream);
    if (e == hipSuccess) e = launch_force(c, idx, n_act, acc, pot, stream);
  } else {
    if (int s = ensure_part(c, fused_partials_needed(c, n_act))) return s;
    e = launch_fused(c, idx, n_act, eta, acc, pot, dtc, stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_force_criterion launch");
  return TSBTS_OK;
}

int tsbts_force_backward(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                         const double *ga, const double *gp, double *gr, double *gm,
                         hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!ga || !gr || !gm) return fail(c, TSBTS_EINVAL, "tsbts_force_backward: NULL array");
  if (int s = check_pred(c, t_block)) return s;
  if (int s = ensure_part(c, backward_partials_needed(c, n_act))) return s;
  if (bwd_sym_applies(c, n_act)) {
    if (int s = sym_prepare(c, 4, 8, c->precision == TSBTS_FP64 ? 8 : 4))
      return fail(c, s, "symmetric adjoint: work list or partials not allocated");
  }
  hipError_t e = launch_backward(c, idx, n_act, ga, gp, gr, gm, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_force_backward launch");
  return TSBTS_OK;
}

int tsbts_correct(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                  const double *acc_new, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!acc_new) return fail(c, TSBTS_EINVAL, "acc_new is NULL");
  if (int s = check_pred(c, t_block)) return s;
  if (c->h.recording) {
    const int64_t need = c->h.count + n_act;
    if (need >= (int64_t(1) << 31))
      return fail(c, TSBTS_EINVAL, "era history exceeds 2^31 records");
    if (int s = grow_log(c, need, stream)) return s;
  }
  hipError_t e = launch_correct(c, idx, n_act, t_block, acc_new, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_correct launch");
  if (c->h.recording) c->h.count += n_act;
  return TSBTS_OK;
}

int tsbts_timestep(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double eta, double *dtc,
                   hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!dtc) return fail(c, TSBTS_EINVAL, "dtc is NULL");
  if (!(eta > 0.0) || !std::isfinite(eta)) return fail(c, TSBTS_EINVAL, "eta must be > 0");
  if (!c->have_pred) return fail(c, TSBTS_ESTATE, "no predicted particle arrays");
  if (int s = ensure_part(c, partial_elems_needed(c, n_act))) return s;
  if (criterion_sym_applies(c, n_act)) {
    const int vb = c->precision == TSBTS_FP64 ? 8 : 4;
    if (int s = sym_prepare(c, 2, vb, vb))
      return fail(c, s, "symmetric criterion: work list or partials not allocated");
  }
  if (int s = split_prepare(c, n_act)) return fail(c, s, "split call: buffers not allocated");
  hipError_t e = launch_timestep(c, idx, n_act, eta, dtc, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_timestep launch");
  return TSBTS_OK;
}

int tsbts_set_dt(tsbts_ctx *c, const int32_t *idx, int32_t n_act, const double *dt_new,
                 hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!dt_new) return fail(c, TSBTS_EINVAL, "dt_new is NULL");
  hipError_t e = launch_set_dt(c, idx, n_act, dt_new, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_set_dt launch");
  return TSBTS_OK;
}

int tsbts_history_begin(tsbts_ctx *c, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  c->h.count = 0;
  if (int s = grow_log(c, c->n, stream)) return s;
  c->h.recording = true;
  hipError_t e = launch_history_begin(c, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_history_begin launch");
  c->h.count = c->n;
  return TSBTS_OK;
}

int tsbts_history_end(tsbts_ctx *c, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (!c->h.recording) return fail(c, TSBTS_ESTATE, "no history is being recorded");
  History &h = c->h;
  if (h.count > h.hcap) {
    // the finished buffers are replaced wholesale, nothing to preserve; the new ones are
    // allocated first, so a failed allocation leaves the previous history usable
    const int64_t cap = std::max<int64_t>(h.count, h.cap);
    double *hs = nullptr, *ht = nullptr;
    int s = dev_alloc(c, &hs, cap * kHistPlanes);
    if (!s) s = dev_alloc(c, &ht, cap);
    if (s) {
      dev_free(hs);
      return s;
    }
    // earlier kernels (predictions from the previous history) may still read the old ones
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      dev_free(hs);
      dev_free(ht);
      return hip_fail(c, e, "tsbts_history_end");
    }
    dev_free(h.ht);
    dev_free(h.hs);
    h.hs = hs;
    h.ht = ht;
    h.hcap = cap;
  }
  hipError_t e = launch_history_end(c, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_history_end launch");
  h.hcount = h.count;
  h.recording = false;
  h.valid = true;
  return TSBTS_OK;
}

int tsbts_history_clear(tsbts_ctx *c) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  c->h.valid = false;
  c->h.recording = false;
  c->h.count = 0;
  return TSBTS_OK;
}

int tsbts_snapshot(tsbts_ctx *c, double T, double *r_out, double *v_out, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (!r_out || !v_out) return fail(c, TSBTS_EINVAL, "tsbts_snapshot: NULL output");
  if (!std::isfinite(T)) return fail(c, TSBTS_EINVAL, "T is not finite");
  hipError_t e = launch_snapshot(c, T, r_out, v_out, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_snapshot launch");
  return TSBTS_OK;
}

int tsbts_energy(tsbts_ctx *c, const double *r, const double *v, const double *m,
                 double *out_KW, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (!r || !v || !m || !out_KW) return fail(c, TSBTS_EINVAL, "tsbts_energy: NULL array");
  hipError_t e = launch_energy(c, r, v, m, out_KW, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_energy launch");
  return TSBTS_OK;
}

int tsbts_leapfrog_adjoint(tsbts_ctx *c, int phase, double h, const double *rbar,
                           double *vbar, double *abar, double *g_out, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (phase != 0 && phase != 1) return fail(c, TSBTS_EINVAL, "phase must be 0 or 1");
  if (!vbar || !abar) return fail(c, TSBTS_EINVAL, "tsbts_leapfrog_adjoint: NULL array");
  if (phase == 0 && !g_out) return fail(c, TSBTS_EINVAL, "g_out is NULL");
  if (phase == 1 && !rbar) return fail(c, TSBTS_EINVAL, "rbar is NULL");
  hipError_t e = launch_leapfrog_adjoint(c, phase, h, rbar, vbar, abar, g_out, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_leapfrog_adjoint launch");
  return TSBTS_OK;
}

int tsbts_block_adjoint(tsbts_ctx *c, int phase, const int32_t *idx, int32_t n_act,
                        double t_block, double *rbar, double *vbar, double *abar,
                        double *pbar, double *seeds, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (phase != 0 && phase != 1) return fail(c, TSBTS_EINVAL, "phase must be 0 or 1");
  if (!rbar || !vbar || !abar || !pbar)
    return fail(c, TSBTS_EINVAL, "tsbts_block_adjoint: NULL array");
  if (phase == 0) {
    if (int s = check_active(c, idx, n_act, stream)) return s;
    if (!seeds) return fail(c, TSBTS_EINVAL, "seeds is NULL");
  }
  hipError_t e = launch_block_adjoint(c, phase, idx, n_act, t_block, rbar, vbar, abar, pbar,
                                      seeds, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_block_adjoint launch");
  return TSBTS_OK;
}

int tsbts_history_layout(tsbts_ctx *c, int64_t *n_records, int32_t *off, double *t,
                         hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (!n_records) return fail(c, TSBTS_EINVAL, "n_records is NULL");
  if (!c->h.valid) return fail(c, TSBTS_ESTATE, "no finished history");
  *n_records = c->h.hcount;
  if (off)
    TSBTS_CHECK_HIP(c, hipMemcpyAsync(off, c->h.off, (c->n + 1) * sizeof(int32_t),
                                      hipMemcpyDeviceToDevice, stream));
  if (t && c->h.hcount > 0)
    TSBTS_CHECK_HIP(c, hipMemcpyAsync(t, c->h.ht, c->h.hcount * sizeof(double),
                                      hipMemcpyDeviceToDevice, stream));
  return TSBTS_OK;
}

int tsbts_interp_adjoint(tsbts_ctx *c, double t_block, double *pbar, double *hbar,
                         int64_t n_records, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (!pbar || !hbar) return fail(c, TSBTS_EINVAL, "tsbts_interp_adjoint: NULL array");
  if (!c->h.valid) return fail(c, TSBTS_ESTATE, "no finished history");
  if (n_records != c->h.hcount)
    return fail(c, TSBTS_EINVAL, "n_records=%lld differs from the history's %lld records",
                static_cast<long long>(n_records), static_cast<long long>(c->h.hcount));
  if (!std::isfinite(t_block)) return fail(c, TSBTS_EINVAL, "t_block is not finite");
  hipError_t e = launch_interp_adjoint(c, t_block, pbar, hbar, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_interp_adjoint launch");
  return TSBTS_OK;
}

int tsbts_record_adjoint(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                         const int32_t *off, const double *t, int64_t n_records,
                         const double *hbar, double *rbar, double *vbar, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!off || !hbar || !rbar || !vbar || (n_records > 0 && !t))
    return fail(c, TSBTS_EINVAL, "tsbts_record_adjoint: NULL array");
  if (n_records < 0) return fail(c, TSBTS_EINVAL, "n_records < 0");
  if (n_records == 0) return TSBTS_OK;
  hipError_t e = launch_record_adjoint(c, idx, n_act, t_block, off, t, n_records, hbar, rbar,
                                       vbar, stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_record_adjoint launch");
  return TSBTS_OK;
}

int tsbts_adjoint_accumulate(tsbts_ctx *c, const double *rbar, const double *vbar,
                             const double *abar, double *rbar_acc, double *vbar_acc,
                             double *abar_acc, hipStream_t stream) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (!rbar || !vbar || !abar || !rbar_acc || !vbar_acc || !abar_acc)
    return fail(c, TSBTS_EINVAL, "tsbts_adjoint_accumulate: NULL array");
  hipError_t e = launch_accumulate3(3 * c->n, rbar, vbar, abar, rbar_acc, vbar_acc, abar_acc,
                                    stream);
  if (e != hipSuccess) return hip_fail(c, e, "tsbts_adjoint_accumulate launch");
  return TSBTS_OK;
}

}  // extern "C"

namespace tsbts {

// Force on the active set followed by its corrector, in the same launches: the corrector
// of each target runs where its force is finished (end of the force kernel, or its split-j
// reduction).  Same checks and history bookkeeping as tsbts_force + tsbts_correct; used by
// the native scheduler, whose block steps need nothing between the two.
int force_correct(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                  double *acc, hipStream_t stream, const StepTags *tags) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!acc) return fail(c, TSBTS_EINVAL, "acc is NULL");
  if (int s = check_pred(c, t_block)) return s;
  if (int s = ensure_part(c, partial_elems_needed(c, n_act))) return s;
  if (c->h.recording) {
    const int64_t need = c->h.count + n_act;
    if (need >= (int64_t(1) << 31))
      return fail(c, TSBTS_EINVAL, "era history exceeds 2^31 records");
    if (int s = grow_log(c, need, stream)) return s;
  }
  if (int s = prepare_force_sym(c, n_act)) return s;
  CorrectArgs corr = correct_args(c, idx, n_act, t_block, acc);
  if (tags) {
    corr.tag = tags->tag;
    corr.step = tags->step;
  }
  hipError_t e = launch_force(c, idx, n_act, acc, nullptr, stream, &corr);
  if (e != hipSuccess) return hip_fail(c, e, "force + corrector launch");
  if (c->h.recording) c->h.count += n_act;
  return TSBTS_OK;
}

// Prediction and force with the corrector for a small active set, the sources predicted
// as the force kernel loads them (one launch less than tsbts_predict + force_correct, same
// results).  Same checks and history bookkeeping as tsbts_predict + force_correct.
int force_correct_predicted(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                            int use_history, double *acc, hipStream_t stream,
                            const StepTags *tags, const PendingSteps *pend,
                            const InlineIdx *in, double eta, double *dtc, int *crit_done) {
  if (crit_done) *crit_done = 0;
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (in && in->k > 0) {
    // the list arrives by value and is written to idx by the kernel itself
    if (in->k != n_act || in->out != idx || c->check_idx)
      return fail(c, TSBTS_EINVAL, "inline active list not usable here");
  } else if (int s = check_active(c, idx, n_act, stream)) {
    return s;
  }
  if (!acc) return fail(c, TSBTS_EINVAL, "acc is NULL");
  if (!std::isfinite(t_block)) return fail(c, TSBTS_EINVAL, "t_block is not finite");
  if (n_act > small_act_limit(c))
    return fail(c, TSBTS_EINVAL, "prediction on load serves at most %d targets",
                small_act_limit(c));
  if (use_history && !c->h.valid)
    return fail(c, TSBTS_ESTATE, "use_history requested without a finished history");
  if (int s = ensure_part(c, partial_elems_needed(c, n_act))) return s;
  if (c->h.recording) {
    const int64_t need = c->h.count + n_act;
    if (need >= (int64_t(1) << 31))
      return fail(c, TSBTS_EINVAL, "era history exceeds 2^31 records");
    if (int s = grow_log(c, need, stream)) return s;
  }
  CorrectArgs corr = correct_args(c, idx, n_act, t_block, acc);
  if (tags) {
    corr.tag = tags->tag;
    corr.step = tags->step;
  }
  const bool crit = dtc && small_criterion_fused(c, n_act);
  if (crit && (!(eta > 0.0) || !std::isfinite(eta)))
    return fail(c, TSBTS_EINVAL, "eta must be > 0");
  hipError_t e = launch_force_predicted(c, idx, n_act, t_block, use_history ? 1 : 0, acc,
                                        nullptr, stream, &corr, pend, in, eta,
                                        crit ? dtc : nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "prediction + force + corrector launch");
  if (crit_done) *crit_done = crit ? 1 : 0;
  c->pred_t = t_block;
  c->have_pred = true;
  if (c->h.recording) c->h.count += n_act;
  return TSBTS_OK;
}

// The fused force + criterion with the corrector in its reduction (the native
// scheduler's block step when the criterion is taken before the corrector).
int force_criterion_correct(tsbts_ctx *c, const int32_t *idx, int32_t n_act, double t_block,
                            double eta, double *acc, double *dtc, hipStream_t stream,
                            const StepTags *tags) {
  if (check_ctx(c)) return TSBTS_EINVAL;
  if (int s = check_bound(c)) return s;
  if (int s = check_active(c, idx, n_act, stream)) return s;
  if (!acc || !dtc) return fail(c, TSBTS_EINVAL, "acc or dtc is NULL");
  if (int s = check_pred(c, t_block)) return s;
  if (int s = ensure_part(c, std::max(fused_partials_needed(c, n_act),
                                      partial_elems_needed(c, n_act))))
    return s;
  if (c->h.recording) {
    const int64_t need = c->h.count + n_act;
    if (need >= (int64_t(1) << 31))
      return fail(c, TSBTS_EINVAL, "era history exceeds 2^31 records");
    if (int s = grow_log(c, need, stream)) return s;
  }
  CorrectArgs corr = correct_args(c, idx, n_act, t_block, acc);
  if (tags) {
    corr.tag = tags->tag;
    corr.step = tags->step;
  }
  hipError_t e;
  if (n_act <= kSmallAct) {
    // small sets: the criterion on the predicted state first, then the force with the
    // corrector (the corrector rewrites the velocities the criterion reads)
    e = launch_timestep(c, idx, n_act, eta, dtc, stream);
    if (e == hipSuccess) e = launch_force(c, idx, n_act, acc, nullptr, stream, &corr);
  } else {
    e = launch_fused(c, idx, n_act, eta, acc, nullptr, dtc, stream, &corr);
  }
  if (e != hipSuccess) return hip_fail(c, e, "force + criterion + corrector launch");
  if (c->h.recording) c->h.count += n_act;
  return TSBTS_OK;
}

}  // namespace tsbts
