/*
 * tsbts.h - C ABI of the MI355X (gfx950) hot path of the dynamic-era time-symmetric block
 * time-step (TSBTS) N-body method of Kaplan & Saygin, arXiv 1205.2288.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Pointers are DEVICE pointers (HIP global memory on the current device) unless the
 *   comment says "host".  Vectors of particles are float64 structure-of-arrays: an array
 *   documented as [3][n] holds all x, then all y, then all z.
 * - Every call that takes a stream enqueues its work asynchronously on that stream (0 is
 *   the legacy default stream) and returns without synchronising, except where stated.
 *   Results are valid once the stream has been synchronised.
 * - The return value is a status: TSBTS_OK (0) or a negative code below.  Argument checks
 *   are done on the host before anything is enqueued; on error nothing is enqueued and
 *   tsbts_last_error() describes the problem.  No C++ exception crosses this interface.
 * - One context serves one stream at a time; calls on one context must not overlap.
 * - Caller-owned arrays stay owned by the caller.  The context owns only its scratch
 *   (predicted particle arrays, partial sums, stored era history) and frees it in
 *   tsbts_destroy().
 * - Units: G = 1 (Section 3 of the paper).  Softening is of Plummer type with length eps:
 *   a pair at separation d interacts through (|d|^2 + eps^2)^(-1/2).
 */
#ifndef TSBTS_H
#define TSBTS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TSBTS_OK 0
#define TSBTS_EINVAL (-1) /* invalid argument (null pointer, size or index out of range) */
#define TSBTS_ENOMEM (-2) /* device allocation failed (or the scheduler's host memory) */
#define TSBTS_EHIP (-3)   /* a HIP runtime call failed; tsbts_last_error() has its text */
#define TSBTS_ESTATE (-4) /* call out of order (e.g. force at a time that was not predicted) */

/* force precision, chosen at creation */
#define TSBTS_FP64 0  /* all pair arithmetic in float64 */
#define TSBTS_MIXED 1 /* float64 positions, float32 pair arithmetic, float64 tile sums */

/* creation flags (MIXED precision only; the default is the fastest variant on gfx950:
 * separations formed in float64 and rounded once to float32, and the hardware float32
 * reciprocal square root used as is) */
#define TSBTS_FLAG_HILO_SEPARATION 1 /* form separations from float32 hi/lo position pairs:
                                        (x_hi_j - x_hi_i) + (x_lo_j - x_lo_i) */
#define TSBTS_FLAG_NEWTON 2          /* refine the float32 1/sqrt by one Newton step */

typedef struct tsbts_ctx tsbts_ctx;

/* Library version (major*10000 + minor*100 + patch). */
int tsbts_version(void);

/* Human-readable text of a status code (static string). */
const char *tsbts_strerror(int status);

/* Text of the last error reported on ctx (host string owned by ctx; "" if none). */
const char *tsbts_last_error(const tsbts_ctx *ctx);

/* Create a context for n particles (n >= 1) with softening length eps >= 0 on the current
 * HIP device.  precision is TSBTS_FP64 or TSBTS_MIXED; flags is a bitwise OR of
 * TSBTS_FLAG_* values.  Allocates the context's scratch (synchronous).  *out receives the
 * context, or NULL on error. */
int tsbts_create(tsbts_ctx **out, int64_t n, double eps, int precision, int flags);

/* Free the context and everything it owns (synchronises the device first).  NULL is a
 * no-op. */
int tsbts_destroy(tsbts_ctx *ctx);

/* tuning parameters of tsbts_tune */
#define TSBTS_TUNE_BLOCKS 1
#define TSBTS_TUNE_IPL 2
#define TSBTS_TUNE_CHUNK 3
#define TSBTS_TUNE_SYMMETRIC 4
#define TSBTS_TUNE_CHECK_INDICES 5
#define TSBTS_TUNE_SPLIT 6

/* Launch-shape tuning of the pair kernels (force, criterion, adjoint); host-side only.
 *   TSBTS_TUNE_BLOCKS: workgroups a split-j launch aims for (64 .. 65536; default 8192)
 *   TSBTS_TUNE_IPL:    kernel form of the force and criterion (0 = automatic: the force,
 *                      and the criterion from 8192 targets, read the j-particles through
 *                      wave-uniform scalar loads; 1, 2 or 4 = the LDS-staged kernels with
 *                      that many target particles per lane)
 *   TSBTS_TUNE_CHUNK:  j-particles per split unit of the scalar-load kernels (0 =
 *                      automatic: 64 when 256-particle units would give fewer than 512
 *                      workgroups, else 256; or 64, 256)
 *   TSBTS_TUNE_SYMMETRIC: when every particle is a target (n_active = n), evaluate each
 *                      unordered pair once for both of its particles (0 = never, 1 =
 *                      always, 2 = automatic: from 32768 particles while the partial
 *                      sums, which grow linearly (about 6 KB per particle), fit 32 GiB:
 *                      N up to about 5.6 million; default 2).  The criterion (maxima and
 *                      minima) is then bit-identical; sums are combined in another fixed
 *                      order.  The first such call on a context allocates its work list
 *                      and partial buffers.
 *   TSBTS_TUNE_SPLIT:  when a proper subset of at least 8192 particles is active
 *                      (tsbts_force, tsbts_timestep and the native scheduler's block
 *                      steps, without TSBTS_FLAG_NEWTON and with the automatic kernel
 *                      form and chunk), evaluate the pairs among the targets once for both
 *                      (the symmetric kernels on a compact copy of the targets) and their
 *                      pairs with the other particles by the gather kernels (a compact
 *                      copy of those as the sources); the criterion is then bit-identical,
 *                      force sums are combined in another fixed order (0 = never, 1 = from
 *                      8192 targets, 2 = automatic: from 16384 targets, force calls only
 *                      without the potential; default 2).  The
 *                      first such call on a context allocates the copies (about 270 bytes
 *                      per particle) and the symmetric partial buffers for its size.
 *   TSBTS_TUNE_CHECK_INDICES: 1 = every call that takes active_idx first checks on the
 *                      device that each index lies in [0, n) and occurs once, synchronises
 *                      the stream and returns TSBTS_EINVAL, with nothing else launched, if
 *                      not (a debugging aid: two extra launches and one synchronisation
 *                      per call; enabling it allocates n counters); 0 = indices trusted
 *                      (default; an index outside [0, n) is then undefined behaviour, and
 *                      a repeated index leaves undefined output rows when every particle
 *                      is a target and the symmetric kernels serve the call, or when a
 *                      split call does).
 * Results do not depend on these except through the order of float64 tile sums.
 * Invalid values return TSBTS_EINVAL and leave the setting unchanged. */
int tsbts_tune(tsbts_ctx *ctx, int param, int value);

/* Attach the caller's particle state, used by predict / correct / timestep / snapshot /
 * history calls (Algorithm 2's per-particle data: positions, velocities, accelerations,
 * time of the last step and current block step).
 *   r, v, a   [3][n] float64   positions, velocities, accelerations (read and written)
 *   m         [n]    float64   masses (read)
 *   t_last    [n]    float64   time of each particle's last step (read and written)
 *   dt        [n]    float64   current block step of each particle (read)
 * Times and steps must be dyadic (multiples of a power of two), so that the activity test
 * t_last + dt == t_block is exact.  The pointers must stay valid while bound. */
int tsbts_bind_state(tsbts_ctx *ctx, double *r, double *v, double *a, const double *m,
                     double *t_last, double *dt);

/* Predict every particle to t_block (Section 2 predictor; Algorithm 2, step 4) into the
 * context's particle arrays used by tsbts_force / tsbts_timestep / tsbts_force_backward:
 *   - a particle with t_last + dt == t_block (active) is Taylor-predicted from its own
 *     state: r + v h + a h^2/2, v + a h with h = t_block - t_last;
 *   - otherwise, when use_history != 0 and the stored records of the previous pass (see
 *     tsbts_history_end) bracket t_block, it is interpolated between the two bracketing
 *     records by cubic Hermite interpolation (positions from (r, v), velocities from
 *     (v, a) at both ends) - the time-symmetric interpolation of the second and later
 *     passes;
 *   - otherwise it is Taylor-predicted.
 * Requires bound state.  use_history requires a completed history (else TSBTS_ESTATE).
 * The interpolation keeps a per-particle cursor into the history that follows t_block in
 * either direction (forward within a pass, backward in a reverse sweep). */
int tsbts_predict(tsbts_ctx *ctx, double t_block, int use_history, hipStream_t stream);

/* Load explicit positions r [3][n] and masses m [n] (float64) into the context's particle
 * arrays, labelled with time t_label, in place of a prediction (used to evaluate forces
 * of arbitrary configurations, e.g. inside a differentiated leapfrog).  Velocities used by
 * tsbts_timestep are set to zero. */
int tsbts_load_positions(tsbts_ctx *ctx, const double *r, const double *m, double t_label,
                         hipStream_t stream);

/* Softened acceleration and potential of the active particles against all n particles
 * (Algorithm 2, step 5; Plummer softening of Section 3), from the arrays of the last
 * tsbts_predict / tsbts_load_positions, whose time must equal t_block (else
 * TSBTS_ESTATE):
 *   acc_i =  sum_{j != i} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^(3/2)
 *   pot_i = -sum_{j != i} m_j / (|r_j - r_i|^2 + eps^2)^(1/2)
 *   active_idx [n_active] int32   particle indices in [0, n), any order, each at most
 *                                 once (both checked with TSBTS_TUNE_CHECK_INDICES)
 *   acc        [3][n_active]      float64 output, row k for particle active_idx[k]
 *   pot        [n_active]         float64 output, or NULL to skip
 * 1 <= n_active <= n.  The sum over j is split over workgroups when the active set is small
 * (the paper's work partitioning, Section 5) and combined in a fixed order, so results are
 * bit-reproducible. */
int tsbts_force(tsbts_ctx *ctx, const int32_t *active_idx, int32_t n_active, double t_block,
                double *acc, double *pot, hipStream_t stream);

/* Float64 values in the fixed device array of tsbts_force_noalloc (64 MiB per GPU). */
#define TSBTS_NOALLOC_PARTIALS (1 << 23)

/* For callers that cannot allocate device memory (work under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tsbts_force with the split-j partial
 * sums in a fixed device array of TSBTS_NOALLOC_PARTIALS float64 values instead of the
 * context's buffer.  The call allocates and frees nothing (no hipMalloc, hipFree or
 * allocating library routine); the array is part of the library's code object, held by
 * every GPU the library runs on until the process ends, and its address is looked up
 * once per device by the first tsbts_create there.
 * Arguments, checks and outputs are those of tsbts_force.  Differences:
 *   - the all-targets symmetric kernels are never used (their partials take about 6 KB
 *     per particle); the gather kernels serve every call;
 *   - the split of the j-sum is tsbts_force's when its partials fit the array, otherwise
 *     it aims for fewer workgroups (halving until they fit); results are then equal to
 *     tsbts_force's within rounding (another fixed order of float64 tile sums), and bit
 *     for bit whenever tsbts_force also takes the gather kernels with the same split;
 *   - a call that cannot fit at all (n_active <= 32, or <= 16 in TSBTS_FP64, needs
 *     4 * n_active partials per 256 particles: beyond 2^24 particles) returns
 *     TSBTS_EINVAL with nothing enqueued.
 * Every call on one GPU shares that GPU's array and leaves its partials there (each value
 * a call reads is written earlier in the same call, so nothing needs clearing): calls
 * that overlap on one GPU (other streams, contexts or host threads) race and give
 * undefined results; serialise them. */
int tsbts_force_noalloc(tsbts_ctx *ctx, const int32_t *active_idx, int32_t n_active,
                        double t_block, double *acc, double *pot, hipStream_t stream);

/* Vector-Jacobian product of tsbts_force at the same arrays and time (the adjoint used for
 * gradients; not in the paper).  Given grad_acc = dL/dacc [3][n_active] and optionally
 * grad_pot = dL/dpot [n_active] (NULL = zero), ADDS dL/dr into grad_r [3][n] and dL/dm into
 * grad_m [n] (both float64, caller-initialised):
 *   d = r_k - r_c, s = |d|^2 + eps^2, T(d) = s^(-3/2) I - 3 s^(-5/2) d d^T;
 *   for every particle k and active target c != k:
 *     dL/dr_k += m_k (T(d) g_c + gp_c s^(-3/2) d),  dL/dm_k += g_c.d s^(-3/2) - gp_c s^(-1/2)
 *   for every active k (over all j != k, d = r_k - r_j):
 *     dL/dr_k += -sum_j m_j T(d) g_k + gp_k sum_j m_j s^(-3/2) d
 * 1 <= n_active <= n. */
int tsbts_force_backward(tsbts_ctx *ctx, const int32_t *active_idx, int32_t n_active,
                         double t_block, const double *grad_acc, const double *grad_pot,
                         double *grad_r, double *grad_m, hipStream_t stream);

/* Leapfrog corrector of the active particles (Section 2, Eq. leapfrog) at t_block, after
 * tsbts_predict(t_block) and tsbts_force:
 *   r <- r + v h + a h^2/2 (= the predicted position),  v <- v + (a + acc_new) h / 2,
 *   a <- acc_new,  t_last <- t_block,  with h = t_block - t_last.
 * acc_new [3][n_active] float64.  The corrected velocities also replace the predicted ones
 * used by tsbts_timestep.  While a history is being recorded (tsbts_history_begin) the new
 * states are appended to it (Section 2: every step of the era is stored); the stored log
 * grows geometrically, and a growth synchronises the stream. */
int tsbts_correct(tsbts_ctx *ctx, const int32_t *active_idx, int32_t n_active,
                  double t_block, const double *acc_new, hipStream_t stream);

/* Time-step criterion Eq. (nbdt) for the active particles, against all others at the last
 * predicted time (corrected velocities for the active ones):
 *   dtc_i = eta * min_{j != i} min(|r_ij| / |v_ij|, (|r_ij|^2 + eps^2)^(3/4) / sqrt(m_j))
 * i.e. the collision time and the free-fall time sqrt(|r_ij| / |a_ij|) with
 * |a_ij| = m_j |r_ij| / (|r_ij|^2 + eps^2)^(3/2).  dtc [n_active] float64 output. */
int tsbts_timestep(tsbts_ctx *ctx, const int32_t *active_idx, int32_t n_active, double eta,
                   double *dtc, hipStream_t stream);

/* Force, potential and time-step criterion of the active set in one pass over the pairs:
 * a variant of Algorithm 2's order in which the criterion is taken before the corrector,
 * with the predicted velocities of the active particles (the paper takes it after the
 * corrector, with their corrected velocities; positions are the same either way).
 * acc, pot as tsbts_force (pot may be NULL); dtc [n_active] as tsbts_timestep.  Needs a
 * prediction at t_block; errors as tsbts_force and tsbts_timestep. */
int tsbts_force_criterion(tsbts_ctx *ctx, const int32_t *active_idx, int32_t n_active,
                          double t_block, double eta, double *acc, double *pot, double *dtc,
                          hipStream_t stream);

/* Scatter new block steps: dt[active_idx[k]] = dt_new[k] (dt_new device [n_active]). */
int tsbts_set_dt(tsbts_ctx *ctx, const int32_t *active_idx, int32_t n_active,
                 const double *dt_new, hipStream_t stream);

/* Start recording a pass of an era (Section 2: positions, velocities and accelerations of
 * every step are stored during each era).  The first record of every particle is its
 * current bound state at its own t_last. */
int tsbts_history_begin(tsbts_ctx *ctx, hipStream_t stream);

/* Finish the recording: group the records by particle (in time order) so that they become
 * the interpolation source of tsbts_predict(..., use_history=1) and tsbts_snapshot, and
 * reset the per-particle interpolation cursors.  The previous source is replaced. */
int tsbts_history_end(tsbts_ctx *ctx, hipStream_t stream);

/* Forget the interpolation source (e.g. at the start of a new era's first pass). */
int tsbts_history_clear(tsbts_ctx *ctx);

/* Positions and velocities of all particles at time T (era-end synchronisation, Section 2):
 * a particle whose t_last equals T gives its state; otherwise, if the finished history
 * brackets T, cubic Hermite interpolation of its records; otherwise its Taylor prediction.
 * r_out, v_out [3][n] float64.  Does not modify the bound state. */
int tsbts_snapshot(tsbts_ctx *ctx, double T, double *r_out, double *v_out, hipStream_t stream);

/* Total energy terms (Section 3 energy-error diagnostic), all in float64:
 *   out_KW[0] = K =  1/2 sum_i m_i |v_i|^2
 *   out_KW[1] = W = -sum_{i<j} m_i m_j / (|r_i - r_j|^2 + eps^2)^(1/2)
 * r, v [3][n], m [n] float64; out_KW device [2].  Fixed-order reduction (bit-reproducible). */
int tsbts_energy(tsbts_ctx *ctx, const double *r, const double *v, const double *m,
                 double *out_KW, hipStream_t stream);

/* Reverse sweep of one shared-step leapfrog step (adjoint of the corrector of Section 2),
 * element-wise over [3][n] float64 arrays, for step h:
 *   phase 0:  g_out = abar + (h/2) vbar                      (the adjoint of a_{k+1})
 *   phase 1:  abar  = (h/2) vbar + (h^2/2) rbar ;  vbar += h rbar   (adjoints of step k)
 * rbar is read in phase 1; g_out is written in phase 0 only. */
int tsbts_leapfrog_adjoint(tsbts_ctx *ctx, int phase, double h, const double *rbar,
                           double *vbar, double *abar, double *g_out, hipStream_t stream);

/* Reverse sweep of one block step of a fixed block schedule (Section 2's individual
 * power-of-two steps in one pass: every particle predicted by the Taylor polynomial to
 * t_block with h_j = t_block - t_last_j, the force on the active set, the leapfrog corrector
 * r_i <- p_i, v_i <- v_i + dt_i (a_i + an_i)/2, a_i <- an_i on the active set).
 * rbar, vbar, abar [3][n] float64 device: on entry the adjoint of the state after the block
 * step, on exit (after phase 1) the adjoint of the state before it.  pbar [3][n] float64
 * device: the adjoint of the predicted positions.  seeds [3][n_act] float64 device.
 * The bound dt and t_last must hold the steps and the pre-step times of that block step.
 *   phase 0 (idx [n_act] = the active set, sorted or not): pbar = 0 except
 *           pbar_i = rbar_i;  seeds[:, q] = abar_i + (dt_i/2) vbar_i;
 *           abar_i = (dt_i/2) vbar_i;  rbar_i = 0   (i = idx[q]).
 *   then    tsbts_force_backward(idx, t_block, seeds, NULL, pbar, mbar) with the positions
 *           predicted to t_block from the pre-step state (adds dL/dp into pbar).
 *   phase 1 (every particle):  rbar += pbar;  vbar += h_j pbar;  abar += (h_j^2/2) pbar.
 * idx and seeds are ignored in phase 1.  Not in the paper: gradients through the method. */
int tsbts_block_adjoint(tsbts_ctx *ctx, int phase, const int32_t *idx, int32_t n_act,
                        double t_block, double *rbar, double *vbar, double *abar,
                        double *pbar, double *seeds, hipStream_t stream);

/* Adjoints through the passes of an era (not in the paper: gradients through the method).
 * From the second pass on, tsbts_predict(t_block, use_history=1) takes each non-active
 * particle from the finished history of the previous pass (Section 2's time-symmetric
 * interpolation).  A reverse sweep over such a pass needs the transposes of that map and
 * of the recording of a pass's states; the four calls below provide them.  The records
 * of a finished history are numbered as tsbts_history_layout reports them: particle j's
 * records are off[j] .. off[j+1]-1, in time order, the first one its state when the
 * recording began.  A record adjoint array hbar [6][n_records] float64 (device) holds the
 * adjoints of the stored positions (rows 0-2) and velocities (rows 3-5). */

/* Size and numbering of the finished history: *n_records (host) = number of records;
 * off [n+1] int32 and t [n_records] float64 (device, either may be NULL = not copied) get
 * the per-particle offsets and the record times.  Asynchronous copies on `stream`.
 * TSBTS_ESTATE without a finished history. */
int tsbts_history_layout(tsbts_ctx *ctx, int64_t *n_records, int32_t *off, double *t,
                         hipStream_t stream);

/* Adjoint of the interpolation in tsbts_predict(t_block, use_history=1) for the bound
 * state and the current finished history (the same one the prediction used).  For every
 * particle j that the prediction took from the history:
 *   - a record k at exactly t_block:  hbar[0..2][k] += pbar_j;
 *   - else the bracketing records k, k+1 (times t0 < t_block < t1, h = t1 - t0):
 *       hbar[0..2][k]   += H00 pbar_j,   hbar[3..5][k]   += h H10 pbar_j,
 *       hbar[0..2][k+1] += H01 pbar_j,   hbar[3..5][k+1] += h H11 pbar_j
 *     (the cubic Hermite weights of tsbts_predict);
 * and sets pbar_j = 0.  Active and Taylor-predicted particles keep their pbar.
 * pbar [3][n] float64 device (adjoint of the predicted positions, e.g. after
 * tsbts_force_backward); hbar [6][n_records] float64 device, accumulated; n_records must
 * be the history's record count (else TSBTS_EINVAL). */
int tsbts_interp_adjoint(tsbts_ctx *ctx, double t_block, double *pbar, double *hbar,
                         int64_t n_records, hipStream_t stream);

/* Adds the adjoints of the records that the particles active_idx [n_active] received at
 * t_block into the state adjoint: rbar_i += hbar[0..2][k], vbar_i += hbar[3..5][k] for
 * the record k of particle i with time t_block (particles without one are skipped).
 * off [n+1], t [n_records] (device) describe a history as tsbts_history_layout copied
 * them; hbar [6][n_records] is that history's record adjoint; rbar, vbar [3][n] float64
 * device.  In a reverse sweep it is called before the block step that wrote the records
 * is undone, and with every particle at the era start for the first records.  No
 * duplicates in active_idx. */
int tsbts_record_adjoint(tsbts_ctx *ctx, const int32_t *active_idx, int32_t n_active,
                         double t_block, const int32_t *off, const double *t,
                         int64_t n_records, const double *hbar, double *rbar, double *vbar,
                         hipStream_t stream);

/* rbar_acc += rbar, vbar_acc += vbar, abar_acc += abar, all [3][n] float64 device: every
 * pass restarts from the era-start state, whose adjoint is the sum over the passes. */
int tsbts_adjoint_accumulate(tsbts_ctx *ctx, const double *rbar, const double *vbar,
                             const double *abar, double *rbar_acc, double *vbar_acc,
                             double *abar_acc, hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Native host scheduler (Algorithm 2 with Eq. blockcondition, Algorithm 1 and Algorithm 3).
 * Block times are integers in ticks of 2^-20 and every step is a power of two of ticks.
 * The scheduler keeps host copies of each particle's time, step and last criterion value
 * and drives the entry points above; each block step synchronises the stream once (to
 * read the criterion of the active set).  Readings of the paper it follows:
 *   - admissible step = largest power of two <= mean of the criterion at the start and at
 *     the end of the step, within [dt_min, dt_max] (Eq. blockcondition);
 *   - first pass of an era: drop to the admissible step, or double at a multiple of twice
 *     the step when that is admissible (the standard block-step scheme);
 *   - later passes (Algorithm 1, as its prose describes it): even time: double, else keep,
 *     else halve once; odd time: keep, else halve once; the end-of-step criterion comes
 *     from the previous pass's values of the particle, linear in time between them, the
 *     start value beyond the last one;
 *   - every pass restarts from the era-start state; passes after the first interpolate
 *     the non-active particles from the previous pass (tsbts_predict with history);
 *   - fixed era: a multiple of dt_max; dynamic era (Algorithm 3): size = last minus first
 *     next block time, clamped to [dt_max/8, dt_max] and rounded up to a power of two,
 *     dt_max when that is below the largest step in use (Section 4), the era ending at
 *     the next multiple of it; particles whose next time is past the era end are not
 *     advanced in that era;
 *   - from the second pass on, the step of each particle at the era start is chosen
 *     again by Algorithm 1 with the previous pass's end values.
 * --------------------------------------------------------------------------------------- */

/* Admissible step (ticks) for criterion values begin and end at the start and end of a
 * step (Eq. blockcondition), within [dt_min, dt_max] (ticks, powers of two).  Host only. */
int tsbts_sched_admissible(double begin, double end, int64_t dt_min, int64_t dt_max,
                           int64_t *out);

/* New step (ticks) of a particle with step dt at block time t_block (ticks, a multiple of
 * dt) given its criterion value `begin` at t_block and the end values end_dt and end_2dt
 * for the candidate steps dt and 2 dt: the first-pass rule when first_pass != 0, else
 * Algorithm 1.  Host only; returns TSBTS_EINVAL for inconsistent arguments. */
int tsbts_sched_rule(int first_pass, int64_t dt, int64_t t_block, double begin, double end_dt,
                     double end_2dt, int64_t dt_min, int64_t dt_max, int64_t *out);

/* End (ticks) of the era that starts at t0 (ticks) for particles at times t_ticks [n] with
 * steps dt_ticks [n] (host arrays, ticks): t0 + era for a fixed era (era > 0, a multiple
 * of dt_max), else Algorithm 3 as read above - size = last minus first next block time
 * t_i + dt_i, clamped to [dt_max/8, dt_max] and rounded up to a power of two, dt_max when
 * that is below the largest step, the era ending at the next multiple of the size after
 * t0.  Every particle must be in an era-start state (steps powers of two up to dt_max, t
 * aligned to the step, t <= t0 < t + dt), else TSBTS_EINVAL.  Host only. */
int tsbts_sched_era_end(int64_t t0, const int64_t *t_ticks, const int64_t *dt_ticks, int64_t n,
                        int64_t dt_max, int64_t era, int64_t *out);

/* Start a scheduled integration of the bound state at time 0 (Algorithm 2, step 1):
 * sets t_last = 0, computes the accelerations of all particles (into the bound a), their
 * criterion values and block steps (into the bound dt).  eta: accuracy parameter of
 * Eq. nbdt; passes >= 1 (1 = no symmetrization); dt_min, dt_max: step bounds (powers of
 * two, multiples of 2^-20); era > 0: fixed era size (a multiple of dt_max), era <= 0:
 * dynamic era.  Allocates the scheduler's staging (pinned host and device buffers);
 * synchronises the stream. */
int tsbts_sched_init(tsbts_ctx *ctx, double eta, int passes, double dt_min, double dt_max,
                     double era, hipStream_t stream);

/* options of tsbts_sched_option */
#define TSBTS_SCHED_CRITERION_BEFORE_CORRECTOR 1
#define TSBTS_SCHED_PREDICT_ON_LOAD 2
#define TSBTS_SCHED_RULE_THREADS 3

/* Scheduler option (host only; applies from the next block step):
 *   TSBTS_SCHED_CRITERION_BEFORE_CORRECTOR: 0 = the paper's order, criterion after the
 *     corrector (default); 1 = criterion with the predicted velocities, in the same pass
 *     over the pairs as the force (tsbts_force_criterion).
 *   TSBTS_SCHED_PREDICT_ON_LOAD: 1 = for active sets of at most 32 particles (16 in
 *     float64) the predictor's work is done by the force kernel as it loads its sources,
 *     and on few particles (groups of 8 targets times 256-particle tiles at most 8: N up
 *     to 512 with 32 targets, 1024 with 16, 2048 with 8) that kernel's last workgroup
 *     also takes the criterion of the corrected targets: one or two launches per such
 *     block step instead of three or four, the same results bit for bit (default);
 *     0 = separate predictor and criterion launches.  Not combined with the option
 *     above.
 *   TSBTS_SCHED_RULE_THREADS: host threads (1 .. 16; default 4) that share the step rule
 *     (Algorithm 1 with the block condition) of block steps with at least 8192 active
 *     particles; each particle's rule reads and writes its own state only, so the
 *     results are the same for every value (1: the calling thread alone).  The threads
 *     are started at the first such block step and kept until the scheduler is freed.
 * Returns TSBTS_ESTATE before tsbts_sched_init, TSBTS_EINVAL for an unknown option or
 * value. */
int tsbts_sched_option(tsbts_ctx *ctx, int option, int value);

/* Integrate one era with all its passes (Algorithm 2); *era_end (host, may be NULL)
 * receives its end time.  Every pass restarts from the era-start state; from the second
 * pass on, the step of each particle at the era start is chosen again by Algorithm 1
 * (from the step that brought it there) with the previous pass's criterion values, and
 * later steps likewise.  The bound state then holds the final pass's state; particles are
 * synchronised at era ends that are multiples of dt_max. */
int tsbts_sched_era(tsbts_ctx *ctx, double *era_end, hipStream_t stream);

/* Host copies of the scheduler state (each pointer may be NULL): t_ticks, dt_ticks [n]
 * int64, dtc [n] float64 (last criterion values), stats [4] int64 (block steps, force
 * calls, interactions, eras), *time (current era end). */
int tsbts_sched_state(const tsbts_ctx *ctx, int64_t *t_ticks, int64_t *dt_ticks, double *dtc,
                      int64_t *stats, double *time);

/* Wall-clock breakdown of the scheduler's block steps since tsbts_sched_init (host
 * only): for four classes of active-set size k (k <= 32, k <= 256, k <= 1024, larger),
 * seconds[4 * cls + ph] holds the time spent in phase ph: 0 = building the active set and
 * issuing the step's launches (host), 1 = waiting for the step's criterion values (the
 * GPU's work after the last launch returned), 2 = the step rule and bookkeeping of
 * Algorithm 1 on the host, 3 = the whole step from the end of the previous one; counts
 * [2 * cls] the block steps and [2 * cls + 1] their summed active-set sizes.  Either
 * pointer may be NULL; TSBTS_EINVAL without a scheduler. */
int tsbts_sched_timing(const tsbts_ctx *ctx, double *seconds, int64_t *counts);

/* Host copy of each particle's previous step (the step that brought it to its current
 * time; 0 before its first step), dtp_ticks [n] int64: with tsbts_sched_state and the
 * bound r, v, a it makes an era-end checkpoint.  TSBTS_EINVAL without a scheduler. */
int tsbts_sched_prev_steps(const tsbts_ctx *ctx, int64_t *dtp_ticks);

/* Resume from an era-end checkpoint (Section 2: every era end is a point where the
 * integration can stop and start again).  The caller first writes the checkpoint's r, v
 * and a into the bound arrays; this call sets the scheduler's times t_ticks, steps
 * dt_ticks, previous steps dtp_ticks, criterion values dtc ([n] host arrays, copied),
 * statistics stats ([4] host, may be NULL: kept) and current time `time` (a multiple of
 * 2^-20), and writes the bound t_last and dt from them.  The scheduler must have been
 * started with the same eta, passes, step bounds and era (tsbts_sched_init).  Returns
 * TSBTS_EINVAL, changing nothing, unless every particle is in an era-end state: steps
 * powers of two within the bounds, t aligned to the step, t <= time < t + dt, dtp zero or
 * a power of two that divides t and is not above it, dtc finite and positive.
 * Synchronises the stream. */
int tsbts_sched_restore(tsbts_ctx *ctx, const int64_t *t_ticks, const int64_t *dt_ticks,
                        const int64_t *dtp_ticks, const double *dtc, const int64_t *stats,
                        double time, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TSBTS_H */
