/*
 * Plain FP64 CPU oracle for the TSBTS hot path (Kaplan & Saygin, arXiv 1205.2288).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the HIP path.
 *
 * Every routine is the plain definition written out as a double loop over particles in
 * ascending index order, IEEE double rounding, compiled with -O2 -ffp-contract=off (no
 * fused multiply-add), optionally with OpenMP over the outer index.  Arrays are float64
 * structure-of-arrays: x[n], y[n], z[n] (and likewise for velocities).
 *
 * Units (Section 3): G = 1.  Plummer softening (Section 3): a pair at separation d
 * interacts through (|d|^2 + eps^2)^(-1/2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* Acceleration and potential on the listed target particles (Section 2; Algorithm 2,
 * "calculate forces on the active particles"):
 *   a_i   =  sum_{j != i} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^(3/2)
 *   phi_i = -sum_{j != i} m_j / (|r_j - r_i|^2 + eps^2)^(1/2)
 * The self pair is excluded by index.  Outputs are indexed by position in idx. */
void oracle_force(int64_t n, const double *x, const double *y, const double *z,
                  const double *m, double eps, const int32_t *idx, int64_t nact,
                  double *ax, double *ay, double *az, double *pot)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nact; ++k) {
        const int64_t i = idx[k];
        double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[j] - x[i];
            const double dy = y[j] - y[i];
            const double dz = z[j] - z[i];
            const double s = dx * dx + dy * dy + dz * dz + eps2;
            const double rinv = 1.0 / sqrt(s);
            const double rinv3 = rinv * rinv * rinv;
            sx += m[j] * dx * rinv3;
            sy += m[j] * dy * rinv3;
            sz += m[j] * dz * rinv3;
            sp -= m[j] * rinv;
        }
        ax[k] = sx;
        ay[k] = sy;
        az[k] = sz;
        if (pot) pot[k] = sp;
    }
}

/* Total energy E = K + W (Section 3 energy-error diagnostic), with the same softening
 * as the force:
 *   K =  1/2 sum_i m_i |v_i|^2
 *   W = -sum_{i<j} m_i m_j / (|r_i - r_j|^2 + eps^2)^(1/2)
 * Each row i sums j > i in ascending order; rows are added in ascending i. */
void oracle_energy(int64_t n, const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz,
                   const double *m, double eps, double *kin, double *pot)
{
    const double eps2 = eps * eps;
    double k = 0.0;
    for (int64_t i = 0; i < n; ++i)
        k += 0.5 * m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    /* rows in parallel, each row's j-sum in ascending order; rows then added in
     * ascending i, so the result does not depend on the thread count */
    double *row = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = i + 1; j < n; ++j) {
            const double dx = x[j] - x[i];
            const double dy = y[j] - y[i];
            const double dz = z[j] - z[i];
            s += m[i] * m[j] / sqrt(dx * dx + dy * dy + dz * dz + eps2);
        }
        row[i] = s;
    }
    double w = 0.0;
    for (int64_t i = 0; i < n; ++i) w -= row[i];
    free(row);
    *kin = k;
    *pot = w;
}

/* Time-step criterion, Eq. (nbdt) of Section 2:
 *   dt_i = eta * min_{j != i} min( |r_ij| / |v_ij| , sqrt(|r_ij| / |a_ij|) )
 * with the pairwise acceleration taken as the softened pull of j on i,
 *   |a_ij| = m_j |r_ij| / (|r_ij|^2 + eps^2)^(3/2),
 * so that |r_ij| / |a_ij| = (|r_ij|^2 + eps^2)^(3/2) / m_j (this form also defines the
 * limit |r_ij| -> 0).  A zero relative speed makes the collision term infinite. */
void oracle_timestep(int64_t n, const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz,
                     const double *m, double eps, double eta,
                     const int32_t *idx, int64_t nact, double *dt)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nact; ++k) {
        const int64_t i = idx[k];
        double best = INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[j] - x[i];
            const double dy = y[j] - y[i];
            const double dz = z[j] - z[i];
            const double dvx = vx[j] - vx[i];
            const double dvy = vy[j] - vy[i];
            const double dvz = vz[j] - vz[i];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double v = sqrt(dvx * dvx + dvy * dvy + dvz * dvz);
            const double s = r * r + eps2;
            const double tcol = (v > 0.0) ? r / v : INFINITY;
            const double tff = (m[j] > 0.0) ? sqrt(s * sqrt(s) / m[j]) : INFINITY;
            if (tcol < best) best = tcol;
            if (tff < best) best = tff;
        }
        dt[k] = eta * best;
    }
}

/* Vector-Jacobian product of oracle_force (not in the paper; the adjoint of the force
 * step).  Given g_c = dL/da_c and gp_c = dL/dphi_c for every listed target c, add to
 * grad_r[k] = dL/dr_k and grad_m[k] = dL/dm_k for every particle k:
 *
 *   with d = r_k - r_c, s = |d|^2 + eps^2 and T(d) = s^(-3/2) I - 3 s^(-5/2) d d^T,
 *   source term (k is the source of the pull on target c, k != c):
 *     dL/dr_k += m_k [ T(d) g_c + gp_c s^(-3/2) d ]
 *     dL/dm_k += g_c . d s^(-3/2) - gp_c s^(-1/2)
 *   target term (k = c is a target, summed over all sources j != k, d = r_k - r_j):
 *     dL/dr_k += -sum_j m_j T(d) g_k + gp_k sum_j m_j s^(-3/2) d
 *
 * The loops below evaluate these sums literally, one pair at a time. */

/* source term of row k: sum over the listed targets c != k (adds to out[0..3]) */
static void bwd_source_row(int64_t k, const double *x, const double *y, const double *z,
                           const double *m, double eps2, const int32_t *idx, int64_t nact,
                           const double *gax, const double *gay, const double *gaz,
                           const double *gp, double out[4])
{
    double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
    for (int64_t q = 0; q < nact; ++q) {
        const int64_t c = idx[q];
        if (c == k) continue;
        const double dx = x[k] - x[c];
        const double dy = y[k] - y[c];
        const double dz = z[k] - z[c];
        const double s = dx * dx + dy * dy + dz * dz + eps2;
        const double rinv = 1.0 / sqrt(s);
        const double r3 = rinv * rinv * rinv;
        const double r5 = r3 * rinv * rinv;
        const double dg = dx * gax[q] + dy * gay[q] + dz * gaz[q];
        const double g2 = gp ? gp[q] : 0.0;
        sx += r3 * gax[q] - 3.0 * r5 * dg * dx + g2 * r3 * dx;
        sy += r3 * gay[q] - 3.0 * r5 * dg * dy + g2 * r3 * dy;
        sz += r3 * gaz[q] - 3.0 * r5 * dg * dz + g2 * r3 * dz;
        sm += dg * r3 - g2 * rinv;
    }
    out[0] += m[k] * sx;
    out[1] += m[k] * sy;
    out[2] += m[k] * sz;
    out[3] += sm;
}

/* target term of the listed target q (particle k = idx[q]): sum over all sources j != k */
static void bwd_target_row(int64_t q, int64_t n, const double *x, const double *y,
                           const double *z, const double *m, double eps2, const int32_t *idx,
                           const double *gax, const double *gay, const double *gaz,
                           const double *gp, double out[3])
{
    const int64_t k = idx[q];
    const double g2 = gp ? gp[q] : 0.0;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == k) continue;
        const double dx = x[k] - x[j];
        const double dy = y[k] - y[j];
        const double dz = z[k] - z[j];
        const double s = dx * dx + dy * dy + dz * dz + eps2;
        const double rinv = 1.0 / sqrt(s);
        const double r3 = rinv * rinv * rinv;
        const double r5 = r3 * rinv * rinv;
        const double dg = dx * gax[q] + dy * gay[q] + dz * gaz[q];
        sx += -m[j] * (r3 * gax[q] - 3.0 * r5 * dg * dx) + g2 * m[j] * r3 * dx;
        sy += -m[j] * (r3 * gay[q] - 3.0 * r5 * dg * dy) + g2 * m[j] * r3 * dy;
        sz += -m[j] * (r3 * gaz[q] - 3.0 * r5 * dg * dz) + g2 * m[j] * r3 * dz;
    }
    out[0] += sx;
    out[1] += sy;
    out[2] += sz;
}

void oracle_force_backward(int64_t n, const double *x, const double *y, const double *z,
                           const double *m, double eps, const int32_t *idx, int64_t nact,
                           const double *gax, const double *gay, const double *gaz,
                           const double *gp, double *grx, double *gry, double *grz,
                           double *gm)
{
    const double eps2 = eps * eps;
    /* source terms: every particle k against every target c */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        double o[4] = {0.0, 0.0, 0.0, 0.0};
        bwd_source_row(k, x, y, z, m, eps2, idx, nact, gax, gay, gaz, gp, o);
        grx[k] += o[0];
        gry[k] += o[1];
        grz[k] += o[2];
        gm[k] += o[3];
    }
    /* target terms: every listed target k against every source j */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nact; ++q) {
        const int64_t k = idx[q];
        double o[3] = {0.0, 0.0, 0.0};
        bwd_target_row(q, n, x, y, z, m, eps2, idx, gax, gay, gaz, gp, o);
        grx[k] += o[0];
        gry[k] += o[1];
        grz[k] += o[2];
    }
}

/* The same gradient for the listed rows only: out_r[3][nrows], out_m[nrows] (written, not
 * accumulated) for particles rows[0..nrows), each the source term of its row plus, when
 * the row is a listed target, its target term. */
void oracle_force_backward_rows(int64_t n, const double *x, const double *y, const double *z,
                                const double *m, double eps, const int32_t *idx, int64_t nact,
                                const double *gax, const double *gay, const double *gaz,
                                const double *gp, const int32_t *rows, int64_t nrows,
                                double *out_r, double *out_m)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t k = rows[t];
        double o[4] = {0.0, 0.0, 0.0, 0.0};
        bwd_source_row(k, x, y, z, m, eps2, idx, nact, gax, gay, gaz, gp, o);
        double src[3] = {o[0], o[1], o[2]};
        for (int64_t q = 0; q < nact; ++q) {
            if (idx[q] != k) continue;
            double tg[3] = {0.0, 0.0, 0.0};
            bwd_target_row(q, n, x, y, z, m, eps2, idx, gax, gay, gaz, gp, tg);
            src[0] += tg[0];
            src[1] += tg[1];
            src[2] += tg[2];
        }
        out_r[t] = src[0];
        out_r[nrows + t] = src[1];
        out_r[2 * nrows + t] = src[2];
        out_m[t] = o[3];
    }
}

/* Rounding scale of the vector-Jacobian product above: the same sums with every product
 * replaced by its magnitude and every sum of products by the sum of their magnitudes,
 *   source (k != c):  S_r[k] += |m_k| [ s^(-3/2) |g_c| + 3 s^(-5/2) e_c |d| + |gp_c| s^(-3/2) |d| ]
 *                     S_m[k] += e_c s^(-3/2) + |gp_c| s^(-1/2)
 *   target (k = c, over all j != k):
 *                     S_r[k] += sum_j |m_j| [ s^(-3/2) |g_k| + 3 s^(-5/2) e_k |d| ]
 *                               + |gp_k| sum_j |m_j| s^(-3/2) |d|
 * with |.| taken per component and e_c = |d_x g_cx| + |d_y g_cy| + |d_z g_cz|.  By the
 * triangle inequality |dL/dr_k| <= S_r[k] and |dL/dm_k| <= S_m[k] component by component,
 * with equality when a single term of one sign enters; an implementation that evaluates
 * each term with relative error u and sums them has an error of at most about u S.
 * Written (not accumulated) into sr_x, sr_y, sr_z, sm [n], or for the listed rows only
 * when rows is not NULL ([nrows] outputs indexed by position in rows). */
static void scale_source_row(int64_t k, const double *x, const double *y, const double *z,
                             const double *m, double eps2, const int32_t *idx, int64_t nact,
                             const double *gax, const double *gay, const double *gaz,
                             const double *gp, double out[4])
{
    double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
    for (int64_t q = 0; q < nact; ++q) {
        const int64_t c = idx[q];
        if (c == k) continue;
        const double dx = x[k] - x[c];
        const double dy = y[k] - y[c];
        const double dz = z[k] - z[c];
        const double s = dx * dx + dy * dy + dz * dz + eps2;
        const double rinv = 1.0 / sqrt(s);
        const double r3 = rinv * rinv * rinv;
        const double r5 = r3 * rinv * rinv;
        const double e = fabs(dx * gax[q]) + fabs(dy * gay[q]) + fabs(dz * gaz[q]);
        const double g2 = gp ? fabs(gp[q]) : 0.0;
        sx += r3 * fabs(gax[q]) + 3.0 * r5 * e * fabs(dx) + g2 * r3 * fabs(dx);
        sy += r3 * fabs(gay[q]) + 3.0 * r5 * e * fabs(dy) + g2 * r3 * fabs(dy);
        sz += r3 * fabs(gaz[q]) + 3.0 * r5 * e * fabs(dz) + g2 * r3 * fabs(dz);
        sm += e * r3 + g2 * rinv;
    }
    out[0] = fabs(m[k]) * sx;
    out[1] = fabs(m[k]) * sy;
    out[2] = fabs(m[k]) * sz;
    out[3] = sm;
}

static void scale_target_row(int64_t q, int64_t n, const double *x, const double *y,
                             const double *z, const double *m, double eps2,
                             const int32_t *idx, const double *gax, const double *gay,
                             const double *gaz, const double *gp, double out[3])
{
    const int64_t k = idx[q];
    const double g2 = gp ? fabs(gp[q]) : 0.0;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == k) continue;
        const double dx = x[k] - x[j];
        const double dy = y[k] - y[j];
        const double dz = z[k] - z[j];
        const double s = dx * dx + dy * dy + dz * dz + eps2;
        const double rinv = 1.0 / sqrt(s);
        const double r3 = rinv * rinv * rinv;
        const double r5 = r3 * rinv * rinv;
        const double e = fabs(dx * gax[q]) + fabs(dy * gay[q]) + fabs(dz * gaz[q]);
        const double mj = fabs(m[j]);
        sx += mj * (r3 * fabs(gax[q]) + 3.0 * r5 * e * fabs(dx)) + g2 * mj * r3 * fabs(dx);
        sy += mj * (r3 * fabs(gay[q]) + 3.0 * r5 * e * fabs(dy)) + g2 * mj * r3 * fabs(dy);
        sz += mj * (r3 * fabs(gaz[q]) + 3.0 * r5 * e * fabs(dz)) + g2 * mj * r3 * fabs(dz);
    }
    out[0] = sx;
    out[1] = sy;
    out[2] = sz;
}

void oracle_force_backward_scale(int64_t n, const double *x, const double *y,
                                 const double *z, const double *m, double eps,
                                 const int32_t *idx, int64_t nact, const double *gax,
                                 const double *gay, const double *gaz, const double *gp,
                                 const int32_t *rows, int64_t nrows, double *sr_x,
                                 double *sr_y, double *sr_z, double *sm)
{
    const double eps2 = eps * eps;
    const int64_t nout = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nout; ++t) {
        const int64_t k = rows ? rows[t] : t;
        double o[4];
        scale_source_row(k, x, y, z, m, eps2, idx, nact, gax, gay, gaz, gp, o);
        for (int64_t q = 0; q < nact; ++q) {
            if (idx[q] != k) continue;
            double tg[3];
            scale_target_row(q, n, x, y, z, m, eps2, idx, gax, gay, gaz, gp, tg);
            o[0] += tg[0];
            o[1] += tg[1];
            o[2] += tg[2];
        }
        sr_x[t] = o[0];
        sr_y[t] = o[1];
        sr_z[t] = o[2];
        sm[t] = o[3];
    }
}

/* Number of threads the OpenMP runtime will use (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
