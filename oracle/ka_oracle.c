/*
 * ka_oracle.c -- plain FP64 CPU oracle for the Kob-Andersen binary
 * Lennard-Jones molecular-dynamics method of "Introduction to molecular
 * dynamics simulations" (Vollmayr-Lee, arXiv:2001.07089).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only tests/, __graft_entry__.smoke() and
 * the cpu_baseline leg of bench.py may load it.  It shares no source, header,
 * table or constant generator with the GPU library.
 *
 * Every function is the plain definition of what the paper computes, written
 * for readability, in binary64, compiled without floating-point contraction
 * (-ffp-contract=off).  The only acceleration is the cell list of
 * ora_forces_cell, which enumerates exactly the same pair set as the O(N^2)
 * loop and is itself tested against it.
 *
 * Conventions (shared with the callers of this file, not with the GPU code):
 *   - one system of n particles in a cubic periodic box of side L;
 *   - particles 0..na-1 are type A, na..n-1 are type B (the paper stores the
 *     A block first, Sec. III.A);
 *   - pair index p = ti + tj: 0 = AA, 1 = AB, 2 = BB;
 *   - masses are 1 (Sec. II.B), so accelerations equal forces.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Model table: epsilon and sigma per pair type, cutoff factor (Sec. II.B,
 * Eq. (VKALJ) and the truncation of Eq. (VshiftedKALJ)). */
typedef struct {
    double eps[3];
    double sigma[3];
    double rc_factor;
} ora_model;

/* Pair constants derived from the model table. */
typedef struct {
    double eps, sig6, sig12, rc2, vshift;
} ora_pair;

static void pair_constants(const ora_model *m, int p, ora_pair *out)
{
    double s = m->sigma[p];
    double s2 = s * s;
    double s6 = s2 * s2 * s2;
    double rc = m->rc_factor * s;
    out->eps = m->eps[p];
    out->sig6 = s6;
    out->sig12 = s6 * s6;
    out->rc2 = rc * rc;
    /* V_ab(r_c) of Eq. (VKALJ), subtracted inside the cutoff by
     * Eq. (VshiftedKALJ). */
    double ir2 = 1.0 / out->rc2;
    double ir6 = ir2 * ir2 * ir2;
    out->vshift = 4.0 * out->eps * (out->sig12 * ir6 * ir6 - out->sig6 * ir6);
}

static int type_of(int i, int na) { return i < na ? 0 : 1; }

/* Minimum-image convention in the branch form of Sec. III.D: one correction
 * by +-L when the separation exceeds half the box. */
static double min_image(double d, double L)
{
    double half = 0.5 * L;
    if (d > half)
        d -= L;
    else if (d < -half)
        d += L;
    return d;
}

/* Evaluate one pair at squared distance r2 (already inside the cutoff).
 * Returns the scalar f such that F_i = f * (r_i - r_j), Eq. (KAFix):
 *   f = 48 eps (sigma^12 / r^14 - 0.5 sigma^6 / r^8).
 * *v receives the shifted potential of Eq. (VshiftedKALJ). */
static double pair_eval(const ora_pair *c, double r2, double *v)
{
    double ir2 = 1.0 / r2;
    double ir4 = ir2 * ir2;
    double ir6 = ir4 * ir2;
    double ir8 = ir4 * ir4;
    double ir14 = ir8 * ir6;
    *v = 4.0 * c->eps * (c->sig12 * ir6 * ir6 - c->sig6 * ir6) - c->vshift;
    return 48.0 * c->eps * (c->sig12 * ir14 - 0.5 * c->sig6 * ir8);
}

/* Exported closed form of a single pair at squared distance r2 with pair
 * index p: returns f (F_i = f r_ij) and the shifted potential; both are zero
 * at or beyond the cutoff (strict "<", Sec. II.B). */
double ora_pair_force(const ora_model *m, int p, double r2, double *v_out)
{
    ora_pair c;
    pair_constants(m, p, &c);
    if (!(r2 < c.rc2)) {
        if (v_out) *v_out = 0.0;
        return 0.0;
    }
    double v;
    double f = pair_eval(&c, r2, &v);
    if (v_out) *v_out = v;
    return f;
}

/* Forces, potential energy and virial by the O(N^2) half loop over i < j
 * with Newton's third law (Sec. III.D).  pe and w may be NULL.
 * Virial W = sum_{i<j} r_ij . F_ij = sum f r^2 (not in the paper; used for
 * the pressure P = rho T + W / (3V)). */
void ora_forces_brute(const ora_model *m, int n, int na, double L,
                      const double *x, const double *y, const double *z,
                      double *fx, double *fy, double *fz,
                      double *pe, double *w)
{
    ora_pair c[3];
    for (int p = 0; p < 3; ++p) pair_constants(m, p, &c[p]);
    for (int i = 0; i < n; ++i) fx[i] = fy[i] = fz[i] = 0.0;
    double epot = 0.0, vir = 0.0;
    for (int i = 0; i < n - 1; ++i) {
        int ti = type_of(i, na);
        for (int j = i + 1; j < n; ++j) {
            int p = ti + type_of(j, na);
            double dx = min_image(x[i] - x[j], L);
            double dy = min_image(y[i] - y[j], L);
            double dz = min_image(z[i] - z[j], L);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < c[p].rc2) {
                double v;
                double f = pair_eval(&c[p], r2, &v);
                fx[i] += f * dx; fx[j] -= f * dx;
                fy[i] += f * dy; fy[j] -= f * dy;
                fz[i] += f * dz; fz[j] -= f * dz;
                epot += v;
                vir += f * r2;
            }
        }
    }
    if (pe) *pe = epot;
    if (w) *w = vir;
}

/* Cell index of a coordinate already in [0, L). */
static int cell_coord(double u, double L, int nc)
{
    int k = (int)(u / L * nc);
    if (k < 0) k = 0;
    if (k >= nc) k = nc - 1;
    return k;
}

/* Same forces, potential and virial as ora_forces_brute, enumerated with a
 * cell list of cell side >= the largest cutoff so that every interacting pair
 * lies in neighbouring cells (the neighbour-list idea the paper mentions at
 * the end of Sec. III.E).  Each particle sums over all its partners (the
 * definition of F_i in Eq. (KAFix)); pe and w take half of every pair term.
 * Requires positions in [0, L).  Falls back to the O(N^2) loop when fewer
 * than 3 cells fit along the box edge.  Parallel over particles with OpenMP;
 * the per-particle sums run in a fixed order, so the result is
 * deterministic. */
void ora_forces_cell(const ora_model *m, int n, int na, double L,
                     const double *x, const double *y, const double *z,
                     double *fx, double *fy, double *fz,
                     double *pe, double *w)
{
    ora_pair c[3];
    double rcmax = 0.0;
    for (int p = 0; p < 3; ++p) {
        pair_constants(m, p, &c[p]);
        double rc = m->rc_factor * m->sigma[p];
        if (rc > rcmax) rcmax = rc;
    }
    int nc = (int)floor(L / rcmax);
    if (nc < 3) {
        ora_forces_brute(m, n, na, L, x, y, z, fx, fy, fz, pe, w);
        return;
    }
    int ncell = nc * nc * nc;
    int *head = (int *)malloc(sizeof(int) * (size_t)ncell);
    int *next = (int *)malloc(sizeof(int) * (size_t)n);
    int *cell = (int *)malloc(sizeof(int) * (size_t)n);
    double *epi = (double *)malloc(sizeof(double) * (size_t)n);
    double *wpi = (double *)malloc(sizeof(double) * (size_t)n);
    for (int k = 0; k < ncell; ++k) head[k] = -1;
    /* Build the linked lists from the last particle down so that each list
     * runs in increasing particle index. */
    for (int i = n - 1; i >= 0; --i) {
        int cx = cell_coord(x[i], L, nc);
        int cy = cell_coord(y[i], L, nc);
        int cz = cell_coord(z[i], L, nc);
        int k = (cz * nc + cy) * nc + cx;
        cell[i] = k;
        next[i] = head[k];
        head[k] = i;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int ti = type_of(i, na);
        int k = cell[i];
        int cx = k % nc, cy = (k / nc) % nc, cz = k / (nc * nc);
        double axi = 0.0, ayi = 0.0, azi = 0.0, ei = 0.0, wi = 0.0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int qx = (cx + ox + nc) % nc;
                    int qy = (cy + oy + nc) % nc;
                    int qz = (cz + oz + nc) % nc;
                    for (int j = head[(qz * nc + qy) * nc + qx]; j >= 0; j = next[j]) {
                        if (j == i) continue;
                        int p = ti + type_of(j, na);
                        double dx = min_image(x[i] - x[j], L);
                        double dy = min_image(y[i] - y[j], L);
                        double dz = min_image(z[i] - z[j], L);
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 < c[p].rc2) {
                            double v;
                            double f = pair_eval(&c[p], r2, &v);
                            axi += f * dx;
                            ayi += f * dy;
                            azi += f * dz;
                            ei += 0.5 * v;
                            wi += 0.5 * f * r2;
                        }
                    }
                }
        fx[i] = axi; fy[i] = ayi; fz[i] = azi;
        epi[i] = ei; wpi[i] = wi;
    }
    double epot = 0.0, vir = 0.0;
    for (int i = 0; i < n; ++i) { epot += epi[i]; vir += wpi[i]; }
    if (pe) *pe = epot;
    if (w) *w = vir;
    free(head); free(next); free(cell); free(epi); free(wpi);
}

/* Smallest minimum-image pair distance (brute force); used to check
 * initial configurations. */
double ora_min_distance(int n, double L, const double *x, const double *y,
                        const double *z)
{
    double best = INFINITY;
    for (int i = 0; i < n - 1; ++i)
        for (int j = i + 1; j < n; ++j) {
            double dx = min_image(x[i] - x[j], L);
            double dy = min_image(y[i] - y[j], L);
            double dz = min_image(z[i] - z[j], L);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < best) best = r2;
        }
    return sqrt(best);
}

/* Periodic wrap into [0, L): u <- u - L floor(u/L), with a guard against the
 * rounding cases where the result lands on L or just below 0.  The number of
 * box lengths removed is added to the image counter so that u + img*L is the
 * unwrapped coordinate (Sec. VI.B.1).  Image counters are stored as three
 * blocks of n: img[i], img[n + i], img[2n + i] for x, y, z. */
static double wrap(double u, double L, int32_t *img)
{
    double k = floor(u / L);
    u = u - k * L;
    if (u >= L) { u -= L; k += 1.0; }
    if (u < 0.0) { u += L; k -= 1.0; }
    *img += (int32_t)k;
    return u;
}

/* Kinetic energy sum_i v_i^2 / 2 with m = 1 (Eq. (EsysNpart)). */
double ora_kinetic(int n, const double *vx, const double *vy, const double *vz)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
    return 0.5 * s;
}

/* Force routine selector: 0 = O(N^2) half loop, 1 = cell list. */
static void forces(const ora_model *m, int use_cell, int n, int na, double L,
                   const double *x, const double *y, const double *z,
                   double *ax, double *ay, double *az, double *pe, double *w)
{
    if (use_cell)
        ora_forces_cell(m, n, na, L, x, y, z, ax, ay, az, pe, w);
    else
        ora_forces_brute(m, n, na, L, x, y, z, ax, ay, az, pe, w);
}

/* ---------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): a 4-word counter is transformed by ten rounds of
 * two 32x32->64 multiplications and xors with a 2-word key; the key is
 * bumped by the Weyl constants between rounds.
 * ------------------------------------------------------------------- */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Uniform deviate in (0,1) from two 32-bit words: 26 high bits of each form
 * a 52-bit integer k, and u = (2k + 1) / 2^53 is exact in binary64 and never
 * 0 or 1. */
static double uniform_open(uint32_t a, uint32_t b)
{
    uint64_t k = ((uint64_t)(a >> 6) << 26) | (uint64_t)(b >> 6);
    return (double)(2 * k + 1) * 0x1p-53;
}

/* Three standard normal deviates for particle `id` of replica `rep` at draw
 * `tag`, by the Box-Muller transform of Philox uniforms.
 * Counter = {id, tag, rep, block}, key = the two halves of the seed. */
void ora_gauss3(uint64_t seed, uint32_t rep, uint32_t tag, uint32_t id, double g[3])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {id, tag, rep, 0u};
    uint32_t o[4];
    const double twopi = 6.283185307179586476925286766559;
    ora_philox4x32_10(ctr, key, o);
    double u1 = uniform_open(o[0], o[1]);
    double u2 = uniform_open(o[2], o[3]);
    double rad = sqrt(-2.0 * log(u1));
    g[0] = rad * cos(twopi * u2);
    g[1] = rad * sin(twopi * u2);
    ctr[3] = 1u;
    ora_philox4x32_10(ctr, key, o);
    u1 = uniform_open(o[0], o[1]);
    u2 = uniform_open(o[2], o[3]);
    rad = sqrt(-2.0 * log(u1));
    g[2] = rad * cos(twopi * u2);
}

/* Maxwell-Boltzmann velocities at temperature T, following the four steps
 * of the flow chart in Sec. II.E.1: (1) Gaussian components with standard
 * deviation sqrt(kT/m), Eqs. (vxocitydistribution),(sigmavx); (2) mass
 * scaling (m = 1, nothing to do); (3) subtract the centre-of-mass velocity;
 * (4) rescale so that sum v^2 = d N T exactly (Eq. (equip3N), with 3
 * replaced by d for the planar system of the appendix, which keeps vz = 0).
 * A single particle has no velocity left after step (3); step (4) then has
 * nothing to rescale and the particle stays at rest (the flow chart does not
 * treat n = 1; this is the reading taken).
 * ids[i] is the counter word identifying particle i (its index in the
 * caller's order); NULL means ids[i] = i.  dim is 3 or 2. */
void ora_mb_velocities_d(int dim, int n, double T, uint64_t seed, uint32_t rep, uint32_t tag,
                         const int32_t *ids, double *vx, double *vy, double *vz)
{
    double sig = sqrt(T);
    for (int i = 0; i < n; ++i) {
        double g[3];
        ora_gauss3(seed, rep, tag, ids ? (uint32_t)ids[i] : (uint32_t)i, g);
        vx[i] = sig * g[0];
        vy[i] = sig * g[1];
        vz[i] = dim == 2 ? 0.0 : sig * g[2];
    }
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int i = 0; i < n; ++i) { sx += vx[i]; sy += vy[i]; sz += vz[i]; }
    sx /= (double)n; sy /= (double)n; sz /= (double)n;
    for (int i = 0; i < n; ++i) { vx[i] -= sx; vy[i] -= sy; vz[i] -= sz; }
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
    double scale = s2 > 0.0 ? sqrt((double)dim * T * (double)n / s2) : 0.0;
    for (int i = 0; i < n; ++i) { vx[i] *= scale; vy[i] *= scale; vz[i] *= scale; }
}

void ora_mb_velocities(int n, double T, uint64_t seed, uint32_t rep, uint32_t tag,
                       const int32_t *ids, double *vx, double *vy, double *vz)
{
    ora_mb_velocities_d(3, n, T, seed, rep, tag, ids, vx, vy, vz);
}

/* Velocity-Verlet NVE steps in the order of the time loop of Sec. III.E:
 *   r += v dt + a dt^2 / 2 (Eq. (velVerletPos)); wrap into the box;
 *   v += a dt / 2; a = F(r); v += a dt / 2 (Eq. (velVerletVel)).
 * On entry a must hold the forces of the entry positions.
 * Optional stochastic bath (Sec. III.G): after step s (s counted from
 * step0 + 1), when nb > 0 and s % nb == 0, all velocities are redrawn by
 * ora_mb_velocities_d (dimension dim) with draw tag s.  A planar system
 * (dim 2, z = vz = 0 on entry) stays planar: its forces have no z part.
 * energy_out (may be NULL) receives, per step, {KE, PE, W} after the step. */
void ora_run(const ora_model *m, int use_cell, int dim, int n, int na, double L, double dt,
             int nsteps, int64_t step0,
             double *x, double *y, double *z, double *vx, double *vy, double *vz,
             double *ax, double *ay, double *az, int32_t *img,
             int nb, double T, uint64_t seed, uint32_t rep, const int32_t *ids,
             double *energy_out)
{
    double dt2 = dt * dt;
    for (int s = 1; s <= nsteps; ++s) {
        for (int i = 0; i < n; ++i) {
            x[i] += vx[i] * dt + 0.5 * ax[i] * dt2;
            y[i] += vy[i] * dt + 0.5 * ay[i] * dt2;
            z[i] += vz[i] * dt + 0.5 * az[i] * dt2;
            x[i] = wrap(x[i], L, &img[i]);
            y[i] = wrap(y[i], L, &img[n + i]);
            z[i] = wrap(z[i], L, &img[2 * n + i]);
            vx[i] += 0.5 * ax[i] * dt;
            vy[i] += 0.5 * ay[i] * dt;
            vz[i] += 0.5 * az[i] * dt;
        }
        double pe, w;
        forces(m, use_cell, n, na, L, x, y, z, ax, ay, az, &pe, &w);
        for (int i = 0; i < n; ++i) {
            vx[i] += 0.5 * ax[i] * dt;
            vy[i] += 0.5 * ay[i] * dt;
            vz[i] += 0.5 * az[i] * dt;
        }
        int64_t step = step0 + s;
        if (nb > 0 && step % nb == 0)
            ora_mb_velocities_d(dim, n, T, seed, rep, (uint32_t)step, ids, vx, vy, vz);
        if (energy_out) {
            energy_out[3 * (s - 1) + 0] = ora_kinetic(n, vx, vy, vz);
            energy_out[3 * (s - 1) + 1] = pe;
            energy_out[3 * (s - 1) + 2] = w;
        }
    }
}

/* Nose-Hoover steps with the Fox-Andersen velocity-Verlet scheme of
 * Appendix B (m = 1, X = d N with d = dim, k_B = 1).  Per step, with K = sum v(t)^2 and
 * G = (K - X T) / Q:
 *   r(t+dt)  = r + v dt + (a - xi v) dt^2 / 2         Eq. (Noseupdate_ri),
 *              read with the velocity where the text prints the position;
 *   ln s    += xi dt + G dt^2 / 2                     Eq. (Noseupdate_lns);
 *   xi_a     = xi + G dt                              Eq. (Noseupdate_xiapprox);
 *   a'       = F(r(t+dt));
 *   v(t+dt)  = v + (dt/2) {a + a' - (xi + xi_a) v} [1 - (dt/2) xi_a]
 *              Eq. (ridotKVLRoman), with the bracket multiplying the braces
 *              only (the reading that agrees with Eq. (ridotsolved) to
 *              second order);
 *   xi(t+dt) = xi + (dt/2) [G + G'] with G' from v(t+dt)
 *              (Eq. (FoxAndersen_ydottplush) applied to y = ln s).
 * If exact_solve != 0 the velocity uses the closed-form solution
 * Eq. (ridotsolved) instead (used by tests to compare the two forms).
 * nh_state = {xi, ln_s} is updated in place.
 * energy_out (may be NULL) receives per step {KE, PE, W, xi, ln_s}. */
void ora_run_nh(const ora_model *m, int use_cell, int dim, int n, int na, double L, double dt,
                int nsteps, double T, double Q, int exact_solve,
                double *x, double *y, double *z, double *vx, double *vy, double *vz,
                double *ax, double *ay, double *az, int32_t *img,
                double *nh_state, double *energy_out)
{
    double xi = nh_state[0], lns = nh_state[1];
    double X = (double)dim * (double)n;  /* degrees of freedom, X = dN */
    double dt2 = dt * dt;
    double *bx = (double *)malloc(sizeof(double) * (size_t)n);
    double *by = (double *)malloc(sizeof(double) * (size_t)n);
    double *bz = (double *)malloc(sizeof(double) * (size_t)n);
    for (int s = 1; s <= nsteps; ++s) {
        double K = 2.0 * ora_kinetic(n, vx, vy, vz);
        double G = (K - X * T) / Q;
        for (int i = 0; i < n; ++i) {
            x[i] += vx[i] * dt + 0.5 * (ax[i] - xi * vx[i]) * dt2;
            y[i] += vy[i] * dt + 0.5 * (ay[i] - xi * vy[i]) * dt2;
            z[i] += vz[i] * dt + 0.5 * (az[i] - xi * vz[i]) * dt2;
            x[i] = wrap(x[i], L, &img[i]);
            y[i] = wrap(y[i], L, &img[n + i]);
            z[i] = wrap(z[i], L, &img[2 * n + i]);
        }
        lns += xi * dt + 0.5 * G * dt2;
        double xia = xi + G * dt;
        double pe, w;
        forces(m, use_cell, n, na, L, x, y, z, bx, by, bz, &pe, &w);
        double h = 0.5 * dt;
        for (int i = 0; i < n; ++i) {
            if (exact_solve) {
                double den = 1.0 + h * xia;
                vx[i] = (vx[i] + h * (ax[i] - xi * vx[i] + bx[i])) / den;
                vy[i] = (vy[i] + h * (ay[i] - xi * vy[i] + by[i])) / den;
                vz[i] = (vz[i] + h * (az[i] - xi * vz[i] + bz[i])) / den;
            } else {
                double fac = 1.0 - h * xia;
                vx[i] = vx[i] + h * ((ax[i] + bx[i]) - (xi + xia) * vx[i]) * fac;
                vy[i] = vy[i] + h * ((ay[i] + by[i]) - (xi + xia) * vy[i]) * fac;
                vz[i] = vz[i] + h * ((az[i] + bz[i]) - (xi + xia) * vz[i]) * fac;
            }
            ax[i] = bx[i]; ay[i] = by[i]; az[i] = bz[i];
        }
        double K1 = 2.0 * ora_kinetic(n, vx, vy, vz);
        double G1 = (K1 - X * T) / Q;
        xi = xi + h * (G + G1);
        if (energy_out) {
            energy_out[5 * (s - 1) + 0] = 0.5 * K1;
            energy_out[5 * (s - 1) + 1] = pe;
            energy_out[5 * (s - 1) + 2] = w;
            energy_out[5 * (s - 1) + 3] = xi;
            energy_out[5 * (s - 1) + 4] = lns;
        }
    }
    nh_state[0] = xi;
    nh_state[1] = lns;
    free(bx); free(by); free(bz);
}

/* Radial-distribution histogram of one configuration (Sec. VI.A.1): every
 * unique pair j > i, minimum-image distance r = sqrt(r^2), bin = int(r/dr)
 * (a true division, as the paper writes it), counted when bin < nbins; AA and
 * BB bins get 2 per pair, AB bins get 1.  hist is [3][nbins] in pair-index
 * order AA, AB, BB and is accumulated into (not cleared). */
void ora_rdf_hist(int n, int na, double L, const double *x, const double *y,
                  const double *z, double dr, int nbins, uint64_t *hist)
{
    for (int i = 0; i < n - 1; ++i) {
        int ti = type_of(i, na);
        for (int j = i + 1; j < n; ++j) {
            int p = ti + type_of(j, na);
            double dx = min_image(x[i] - x[j], L);
            double dy = min_image(y[i] - y[j], L);
            double dz = min_image(z[i] - z[j], L);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            int bin = (int)(r / dr);
            if (bin < nbins) hist[(size_t)p * nbins + bin] += (p == 1) ? 1u : 2u;
        }
    }
}

/* Mean-square displacement per species (Eq. (msdwithi), or Eq. (msdtw) for
 * an origin taken at t_w): unwrapped positions x + img L (Sec. VI.B.1)
 * against stored unwrapped origin positions.  out = {msd_A, msd_B}. */
void ora_msd(int n, int na, double L, const double *x, const double *y,
             const double *z, const int32_t *img, const double *x0,
             const double *y0, const double *z0, double out[2])
{
    double sa = 0.0, sb = 0.0;
    for (int i = 0; i < n; ++i) {
        double ux = x[i] + (double)img[i] * L;
        double uy = y[i] + (double)img[n + i] * L;
        double uz = z[i] + (double)img[2 * n + i] * L;
        double dx = ux - x0[i], dy = uy - y0[i], dz = uz - z0[i];
        double d2 = dx * dx + dy * dy + dz * dz;
        if (i < na) sa += d2; else sb += d2;
    }
    out[0] = na > 0 ? sa / (double)na : 0.0;
    out[1] = n - na > 0 ? sb / (double)(n - na) : 0.0;
}

/* Self part of the van Hove correlation function, the time generalisation
 * of g(r) named at the end of Sec. VI.A (definition of Hansen and McDonald,
 * as used by Kob and Andersen): per species, the histogram over particles of
 * the distance r = |r_u(t) - r_u(t_w)| between the unwrapped position and the
 * unwrapped origin, bin = int(r / dr), counted when bin < nbins.  Normalised
 * to G_s(r, t) by the caller (divide by N_a and the shell volume).
 * out: [2][nbins] counts, accumulated. */
void ora_van_hove_self(int n, int na, double L, const double *x, const double *y,
                       const double *z, const int32_t *img, const double *x0,
                       const double *y0, const double *z0, double dr, int nbins,
                       uint64_t *out)
{
    for (int i = 0; i < n; ++i) {
        double ux = x[i] + (double)img[i] * L;
        double uy = y[i] + (double)img[n + i] * L;
        double uz = z[i] + (double)img[2 * n + i] * L;
        double dx = ux - x0[i], dy = uy - y0[i], dz = uz - z0[i];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        int bin = (int)(r / dr);
        if (bin < nbins) out[(size_t)(i < na ? 0 : 1) * nbins + bin] += 1u;
    }
}

/* Logarithmically spaced measurement steps (Sec. VI.B.1,
 * Eqs. (logtimessteps),(A)): A = (nMD / t0)^(1/kmax); the next measurement
 * step is the nearest integer to t0 A^k (ties to even), advancing k while the
 * rounded value does not move past the current step.  Writes at most maxout
 * steps to out and returns how many there are. */
int ora_log_schedule(int nmd, double t0, int kmax, int32_t *out, int maxout)
{
    double A = pow((double)nmd / t0, 1.0 / (double)kmax);
    double t = t0;
    long next = (long)nearbyint(t0);
    int cnt = 0;
    for (long step = 1; step <= nmd; ++step) {
        if (next == step) {
            while (next == step) {
                t = A * t;
                next = (long)nearbyint(t);
            }
            if (cnt < maxout) out[cnt] = (int32_t)step;
            ++cnt;
        }
    }
    return cnt;
}

/* Threads the OpenMP loops of this file will use. */
int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the threads of the OpenMP loops (for timing the oracle on 1 core and
 * on all cores); n < 1 restores the number of processors. */
void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n >= 1 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}
