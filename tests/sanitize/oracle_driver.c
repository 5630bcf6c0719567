/*
 * The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every
 * exported routine on small systems, including the edge cases (one and two
 * particles, one-species systems, the planar system, outputs shorter than the
 * schedule).  The oracle source is included whole (it has no header).  Exit
 * status 0 and no sanitizer report: every check passed.
 */
#include "../../oracle/ka_oracle.c"

#include <stdio.h>

static int g_failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
            ++g_failures;                                                        \
        }                                                                        \
    } while (0)

static ora_model ka(void)
{
    ora_model m = {{1.0, 1.5, 0.5}, {1.0, 0.8, 0.88}, 2.5};
    return m;
}

/* jittered simple-cubic (or square) lattice of n sites in a box of edge L */
static void lattice(int dim, int n, double L, unsigned seed, double *x, double *y, double *z)
{
    int m = 1;
    while ((dim == 2 ? m * m : m * m * m) < n) ++m;
    const double a = L / m;
    for (int i = 0; i < n; ++i) {
        seed = seed * 1664525u + 1013904223u;
        const double j = ((seed >> 8) / 16777216.0 - 0.5) * 0.1 * a;
        x[i] = (0.5 + i % m) * a + j;
        y[i] = (0.5 + (i / m) % m) * a - j;
        z[i] = dim == 2 ? 0.0 : (0.5 + i / (m * m)) * a + 0.5 * j;
    }
}

static double *alloc(int n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

static void system_checks(int dim, int n, int na, double rho)
{
    const ora_model m = ka();
    const double L = dim == 2 ? sqrt(n / rho) : cbrt(n / rho);
    double *x = alloc(n), *y = alloc(n), *z = alloc(n), *vx = alloc(n), *vy = alloc(n), *vz = alloc(n);
    double *ax = alloc(n), *ay = alloc(n), *az = alloc(n), *bx = alloc(n), *by = alloc(n), *bz = alloc(n);
    double *x0 = alloc(n), *y0 = alloc(n), *z0 = alloc(n);
    int32_t *img = (int32_t *)calloc((size_t)(3 * n + 1), sizeof(int32_t));
    int32_t *ids = (int32_t *)calloc((size_t)(n + 1), sizeof(int32_t));
    for (int i = 0; i < n; ++i) ids[i] = i;
    lattice(dim, n, L, 17u + (unsigned)n, x, y, z);
    memcpy(x0, x, sizeof(double) * (size_t)n);
    memcpy(y0, y, sizeof(double) * (size_t)n);
    memcpy(z0, z, sizeof(double) * (size_t)n);
    double pe1, w1, pe2, w2;
    ora_forces_brute(&m, n, na, L, x, y, z, ax, ay, az, &pe1, &w1);
    if (L > 2.0 * 2.5) {
        ora_forces_cell(&m, n, na, L, x, y, z, bx, by, bz, &pe2, &w2);
        for (int i = 0; i < n; ++i) CHECK(fabs(ax[i] - bx[i]) <= 1e-9 * (1.0 + fabs(ax[i])));
        CHECK(fabs(pe1 - pe2) <= 1e-9 * (1.0 + fabs(pe1)));
    }
    if (n >= 2) CHECK(ora_min_distance(n, L, x, y, z) > 0.0);
    ora_mb_velocities_d(dim, n, 1.0, 99u, 0u, 0u, ids, vx, vy, vz);
    CHECK(ora_kinetic(n, vx, vy, vz) >= 0.0);
    const int steps = 20;
    double *e = alloc(5 * steps);
    for (int cell = 0; cell <= (L > 2.0 * 2.5 ? 1 : 0); ++cell) {
        ora_run(&m, cell, dim, n, na, L, 0.002, steps, 0, x, y, z, vx, vy, vz, ax, ay, az, img, 5, 1.0, 7u, 0u,
                ids, e);
        for (int s = 0; s < 3 * steps; ++s) CHECK(isfinite(e[s]));
    }
    double nh[2] = {0.0, 0.0};
    ora_run_nh(&m, 0, dim, n, na, L, 0.002, steps, 1.0, 10.0, 0, x, y, z, vx, vy, vz, ax, ay, az, img, nh, e);
    for (int s = 0; s < 5 * steps; ++s) CHECK(isfinite(e[s]));
    const int nbins = 40;
    uint64_t hist[3 * 40], vh[2 * 40];
    memset(hist, 0, sizeof hist);
    memset(vh, 0, sizeof vh);
    ora_rdf_hist(n, na, L, x, y, z, 0.5 * L / nbins, nbins, hist);
    double msd[2];
    ora_msd(n, na, L, x, y, z, img, x0, y0, z0, msd);
    CHECK(msd[0] >= 0.0 && msd[1] >= 0.0);
    ora_van_hove_self(n, na, L, x, y, z, img, x0, y0, z0, 0.05, nbins, vh);
    free(x), free(y), free(z), free(vx), free(vy), free(vz), free(ax), free(ay), free(az);
    free(bx), free(by), free(bz), free(x0), free(y0), free(z0), free(img), free(ids), free(e);
}

int main(void)
{
    const ora_model m = ka();
    double v;
    for (int p = 0; p < 3; ++p) {
        CHECK(ora_pair_force(&m, p, 100.0, &v) == 0.0 && v == 0.0);
        CHECK(ora_pair_force(&m, p, 1.0, &v) != 0.0);
    }
    const uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0};
    uint32_t out[4];
    ora_philox4x32_10(ctr, key, out);
    double g[3];
    ora_gauss3(12345u, 1u, 2u, 3u, g);
    CHECK(isfinite(g[0]) && isfinite(g[1]) && isfinite(g[2]));
    int32_t sched[64];
    const int cnt = ora_log_schedule(1000, 1.0, 60, sched, 64);
    CHECK(cnt == 50);
    int32_t few[4];
    CHECK(ora_log_schedule(100000, 1.0, 200, few, 4) > 4);
    for (int dim = 3; dim >= 2; --dim) {
        system_checks(dim, 1, 1, 1.2);
        system_checks(dim, 2, 1, 1.2);
        system_checks(dim, 250, 200, 1.2);
        system_checks(dim, 300, 0, 1.2);
        system_checks(dim, 300, 300, 1.2);
    }
    system_checks(3, 1000, 800, 1.2);
    printf("oracle driver: %d failed checks\n", g_failures);
    return g_failures ? 1 : 0;
}
