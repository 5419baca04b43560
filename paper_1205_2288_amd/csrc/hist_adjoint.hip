// Adjoints of the passes of an era (not in the paper: gradients through the method).
//
// From the second pass on, the predictor takes every non-active particle from the
// previous pass's stored states (Section 2's time-symmetric interpolation): the record
// itself at a stored time, else the cubic Hermite interpolant of the two bracketing
// records, else (no bracket) the Taylor polynomial of its own state.  The interpolated
// position is linear in the stored positions and velocities, so its adjoint scatters the
// position adjoint into the adjoints of those records with the same four weights.  The
// records of a pass are states the corrector wrote, so in the reverse sweep of that pass
// their adjoints are added to the state adjoint at the block step that wrote them; the
// first record of each particle is its era-start state.
//
// One thread per particle (interpolation adjoint) or per active particle (record
// injection): each thread touches only its own particle's records, so there are no
// atomics and the results do not depend on the launch.
#include "hermite.hpp"

namespace tsbts {
namespace {

struct InterpAdjArgs {
  int64_t n;
  double tb;
  const double *t_last, *dt;
  const double *ht;
  const int32_t *off;
  int64_t nrec;
  double *pbar;  // [3][n]
  double *hbar;  // [6][nrec]
};

__global__ __launch_bounds__(kWG) void k_interp_adjoint(InterpAdjArgs A) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (j >= A.n) return;
  if (A.t_last[j] + A.dt[j] == A.tb) return;  // active: its own Taylor prediction
  const int lo = A.off[j], hi = A.off[j + 1];
  if (hi <= lo) return;
  const int k = bracket_search(A.ht, lo, hi, A.tb);
  const bool exact = (A.ht[k] == A.tb);
  if (!exact && k + 1 >= hi) return;  // no bracket: Taylor-predicted
  const int64_t n = A.n, R = A.nrec;
  double p[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) p[c] = A.pbar[c * n + j];
  if (exact) {
#pragma unroll
    for (int c = 0; c < 3; ++c) A.hbar[c * R + k] += p[c];
  } else {
    const Herm H(A.ht[k], A.ht[k + 1], A.tb);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      A.hbar[c * R + k] += H.h00 * p[c];
      A.hbar[(c + 3) * R + k] += H.h10h * p[c];
      A.hbar[c * R + k + 1] += H.h01 * p[c];
      A.hbar[(c + 3) * R + k + 1] += H.h11h * p[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) A.pbar[c * n + j] = 0.0;
}

struct RecordAdjArgs {
  int64_t n;
  const int32_t *idx;
  int n_act;
  double tb;
  const int32_t *off;
  const double *ht;
  int64_t nrec;
  const double *hbar;
  double *rbar, *vbar;
};

__global__ __launch_bounds__(kWG) void k_record_adjoint(RecordAdjArgs A) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q >= A.n_act) return;
  const int64_t i = A.idx[q];
  const int lo = A.off[i], hi = A.off[i + 1];
  if (hi <= lo) return;
  const int k = bracket_search(A.ht, lo, hi, A.tb);
  if (A.ht[k] != A.tb) return;
  const int64_t n = A.n, R = A.nrec;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    A.rbar[c * n + i] += A.hbar[c * R + k];
    A.vbar[c * n + i] += A.hbar[(c + 3) * R + k];
  }
}

__global__ __launch_bounds__(kWG) void k_accumulate3(int64_t len, const double *x0,
                                                     const double *x1, const double *x2,
                                                     double *y0, double *y1, double *y2) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (e >= len) return;
  y0[e] += x0[e];
  y1[e] += x1[e];
  y2[e] += x2[e];
}

}  // namespace

hipError_t launch_interp_adjoint(tsbts_ctx *c, double t_block, double *pbar, double *hbar,
                                 hipStream_t st) {
  InterpAdjArgs A;
  A.n = c->n;
  A.tb = t_block;
  A.t_last = c->t_last;
  A.dt = c->dt;
  A.ht = c->h.ht;
  A.off = c->h.off;
  A.nrec = c->h.hcount;
  A.pbar = pbar;
  A.hbar = hbar;
  hipLaunchKernelGGL(k_interp_adjoint, dim3(static_cast<unsigned>((c->n + kWG - 1) / kWG)),
                     dim3(kWG), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_record_adjoint(tsbts_ctx *c, const int32_t *idx, int n_act, double t_block,
                                 const int32_t *off, const double *ht, int64_t n_records,
                                 const double *hbar, double *rbar, double *vbar,
                                 hipStream_t st) {
  RecordAdjArgs A;
  A.n = c->n;
  A.idx = idx;
  A.n_act = n_act;
  A.tb = t_block;
  A.off = off;
  A.ht = ht;
  A.nrec = n_records;
  A.hbar = hbar;
  A.rbar = rbar;
  A.vbar = vbar;
  hipLaunchKernelGGL(k_record_adjoint, dim3((n_act + kWG - 1) / kWG), dim3(kWG), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_accumulate3(int64_t len, const double *x0, const double *x1,
                              const double *x2, double *y0, double *y1, double *y2,
                              hipStream_t st) {
  if (len <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_accumulate3, dim3(static_cast<unsigned>((len + kWG - 1) / kWG)),
                     dim3(kWG), 0, st, len, x0, x1, x2, y0, y1, y2);
  return hipGetLastError();
}

}  // namespace tsbts
