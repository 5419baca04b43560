/*
 * Host memory-safety check of the oracle (test infrastructure): every routine of
 * oracle/oracle.c on random small systems held in exact-size heap arrays, so that the
 * AddressSanitizer build catches any read or write past an array, and UBSan any undefined
 * arithmetic.  Sizes include one particle, one target, every particle a target, and
 * row lists.  A few invariants are checked on the way (Newton's third law for full sets,
 * the rounding scale bounding the adjoint); the exit status is 0 when all hold.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_force(int64_t n, const double *x, const double *y, const double *z,
                  const double *m, double eps, const int32_t *idx, int64_t nact,
                  double *ax, double *ay, double *az, double *pot);
void oracle_energy(int64_t n, const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz,
                   const double *m, double eps, double *kin, double *pot);
void oracle_timestep(int64_t n, const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz,
                     const double *m, double eps, double eta,
                     const int32_t *idx, int64_t nact, double *dt);
void oracle_force_backward(int64_t n, const double *x, const double *y, const double *z,
                           const double *m, double eps, const int32_t *idx, int64_t nact,
                           const double *gax, const double *gay, const double *gaz,
                           const double *gp, double *grx, double *gry, double *grz,
                           double *gm);
void oracle_force_backward_rows(int64_t n, const double *x, const double *y, const double *z,
                                const double *m, double eps, const int32_t *idx, int64_t nact,
                                const double *gax, const double *gay, const double *gaz,
                                const double *gp, const int32_t *rows, int64_t nrows,
                                double *out_r, double *out_m);
void oracle_force_backward_scale(int64_t n, const double *x, const double *y,
                                 const double *z, const double *m, double eps,
                                 const int32_t *idx, int64_t nact, const double *gax,
                                 const double *gay, const double *gaz, const double *gp,
                                 const int32_t *rows, int64_t nrows, double *sr_x,
                                 double *sr_y, double *sr_z, double *sm);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double uniform(void) {  /* xorshift64*, in [0, 1) */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static double *vec(int64_t n, double lo, double hi) {
    double *a = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) a[i] = lo + (hi - lo) * uniform();
    return a;
}

/* nact distinct indices out of n, in random order */
static int32_t *subset(int64_t n, int64_t nact) {
    int32_t *all = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) all[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        const int64_t j = (int64_t)(uniform() * (double)(i + 1));
        const int32_t t = all[i];
        all[i] = all[j];
        all[j] = t;
    }
    int32_t *out = (int32_t *)malloc(sizeof(int32_t) * (size_t)nact);
    for (int64_t i = 0; i < nact; ++i) out[i] = all[i];
    free(all);
    return out;
}

static int check_case(int64_t n, int64_t nact, double eps, int with_gp) {
    int bad = 0;
    double *x = vec(n, -1, 1), *y = vec(n, -1, 1), *z = vec(n, -1, 1);
    double *vx = vec(n, -1, 1), *vy = vec(n, -1, 1), *vz = vec(n, -1, 1);
    double *m = vec(n, 0.1, 1.0);
    int32_t *idx = subset(n, nact);
    double *ax = vec(nact, 0, 0), *ay = vec(nact, 0, 0), *az = vec(nact, 0, 0);
    double *pot = vec(nact, 0, 0), *dt = vec(nact, 0, 0);
    oracle_force(n, x, y, z, m, eps, idx, nact, ax, ay, az, pot);
    oracle_force(n, x, y, z, m, eps, idx, nact, ax, ay, az, NULL);
    if (nact == n && n > 1) {  /* Newton's third law */
        double sx = 0, sa = 0;
        for (int64_t k = 0; k < nact; ++k) {
            sx += m[idx[k]] * ax[k];
            sa += fabs(m[idx[k]] * ax[k]);
        }
        if (fabs(sx) > 1e-12 * sa) bad |= 1;
    }
    double kin = 0, w = 0;
    oracle_energy(n, x, y, z, vx, vy, vz, m, eps, &kin, &w);
    if (!(kin > 0) || !(w <= 0)) bad |= 2;
    oracle_timestep(n, x, y, z, vx, vy, vz, m, eps, 0.1, idx, nact, dt);
    double *gax = vec(nact, -1, 1), *gay = vec(nact, -1, 1), *gaz = vec(nact, -1, 1);
    double *gp = with_gp ? vec(nact, -1, 1) : NULL;
    double *grx = vec(n, 0, 0), *gry = vec(n, 0, 0), *grz = vec(n, 0, 0), *gm = vec(n, 0, 0);
    oracle_force_backward(n, x, y, z, m, eps, idx, nact, gax, gay, gaz, gp, grx, gry, grz, gm);
    double *sx = vec(n, 0, 0), *sy = vec(n, 0, 0), *sz = vec(n, 0, 0), *sm = vec(n, 0, 0);
    oracle_force_backward_scale(n, x, y, z, m, eps, idx, nact, gax, gay, gaz, gp, NULL, 0,
                                sx, sy, sz, sm);
    for (int64_t k = 0; k < n; ++k)
        if (fabs(grx[k]) > sx[k] * (1 + 1e-12) || fabs(gry[k]) > sy[k] * (1 + 1e-12) ||
            fabs(grz[k]) > sz[k] * (1 + 1e-12) || fabs(gm[k]) > sm[k] * (1 + 1e-12))
            bad |= 4;
    const int64_t nrows = n > 3 ? 3 : n;
    int32_t *rows = subset(n, nrows);
    double *out_r = vec(3 * nrows, 0, 0), *out_m = vec(nrows, 0, 0);
    oracle_force_backward_rows(n, x, y, z, m, eps, idx, nact, gax, gay, gaz, gp, rows, nrows,
                               out_r, out_m);
    double *rsx = vec(nrows, 0, 0), *rsy = vec(nrows, 0, 0), *rsz = vec(nrows, 0, 0);
    double *rsm = vec(nrows, 0, 0);
    oracle_force_backward_scale(n, x, y, z, m, eps, idx, nact, gax, gay, gaz, gp, rows, nrows,
                                rsx, rsy, rsz, rsm);
    for (int64_t t = 0; t < nrows; ++t)
        if (out_r[t] != grx[rows[t]] || out_m[t] != gm[rows[t]] || rsx[t] != sx[rows[t]])
            bad |= 8;
    double *all[] = {x, y, z, vx, vy, vz, m, ax, ay, az, pot, dt, gax, gay, gaz, gp, grx, gry,
                     grz, gm, sx, sy, sz, sm, out_r, out_m, rsx, rsy, rsz, rsm};
    for (size_t i = 0; i < sizeof(all) / sizeof(all[0]); ++i) free(all[i]);
    free(idx);
    free(rows);
    if (bad) printf("case n=%lld nact=%lld eps=%g gp=%d failed (%d)\n", (long long)n,
                    (long long)nact, eps, with_gp, bad);
    return bad;
}

int main(void) {
    int bad = 0;
    const int64_t sizes[][2] = {{1, 1}, {2, 1}, {2, 2}, {3, 3}, {17, 5}, {40, 40}, {64, 1},
                                {100, 37}};
    for (size_t c = 0; c < sizeof(sizes) / sizeof(sizes[0]); ++c)
        for (int g = 0; g < 2; ++g)
            bad |= check_case(sizes[c][0], sizes[c][1], g ? 0.05 : 0.01, g);
    if (bad) return 1;
    printf("oracle host check ok\n");
    return 0;
}
