/*
 * FP64 CPU oracle for the Lennard-Jones / Kob-Andersen MD hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the HIP library.
 *
 * It is the plain definition of what the method computes, written for
 * obviousness, not speed:
 *   - pair potential: 12-6 Lennard-Jones (Sec. 3, performance section),
 *     truncated at rc_ab with the energy shifted by V(rc_ab) so that it is
 *     continuous; the force is not shifted (our reading of the plain cutoff);
 *   - KA mixture: per-species-pair eps/sigma (Sec. 5), rc_ab = 2.5 sigma_ab;
 *   - minimum image in a cubic periodic box, d -= L * nearbyint(d / L);
 *   - forces by brute force over every j != i, O(N^2), no neighbour lists;
 *   - velocity Verlet (Sec. 2.2):
 *       v += dt/(2m) F;  r += dt v;  wrap r into [0, L);  F = F(r);
 *       v += dt/(2m) F;
 *   - neighbour-list membership (Sec. 2.2: every particle within the cutoff
 *     plus a skin): j in L_i  iff  j != i and |d_ij| < rc_{s_i s_j} + skin;
 *   - optional C2 smoothing (Sec. 4, numerical long-time stability): the
 *     truncated-and-shifted potential times g(x) = x^4 / (1 + x^4) with
 *     x = (r - rc_ab) / (h sigma_ab); h = 0 means no smoothing.  The purely
 *     repulsive WCA potential of the same section is LJ cut at
 *     rc = 2^(1/6) sigma with the energy shifted by +eps, which the shifted
 *     truncation gives for that cutoff.
 *
 * Everything is double precision; OpenMP parallelises over i only (each i is
 * an independent sum in a fixed j order).
 *
 * A second, independent route to the same definition closes the file: the
 * cell-list forces and the velocity Verlet over skin-padded Verlet lists of
 * Sec. 2.2, in FP64 (orc_forces_cells, orc_vv_lists).  It is what makes the
 * oracle usable at N = 1e6 (trajectories, CPU timing); the tests pin it
 * against the brute-force functions above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n_species;
    double eps[2][2];
    double sig[2][2];
    double rc[2][2];
    double shift[2][2]; /* V_LJ(rc_ab), subtracted from the energy */
} orc_table;

static double lj_v(double r2, double eps, double sig)
{
    double s2 = sig * sig / r2;
    double s6 = s2 * s2 * s2;
    return 4.0 * eps * (s6 * s6 - s6);
}

/* Radial force factor: F_vec = ff * d_vec with ff = -(dV/dr)/r. */
static double lj_ff(double r2, double eps, double sig)
{
    double s2 = sig * sig / r2;
    double s6 = s2 * s2 * s2;
    return 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
}

static void make_table(orc_table *t, int n_species, const double *eps,
                       const double *sig, const double *rc)
{
    t->n_species = n_species;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            t->eps[a][b] = eps[2 * a + b];
            t->sig[a][b] = sig[2 * a + b];
            t->rc[a][b] = rc[2 * a + b];
            t->shift[a][b] = lj_v(rc[2 * a + b] * rc[2 * a + b], eps[2 * a + b],
                                  sig[2 * a + b]);
        }
}

static void min_image(const double *ri, const double *rj, double L, double d[3])
{
    for (int c = 0; c < 3; ++c) {
        double x = ri[c] - rj[c];
        d[c] = x - L * nearbyint(x / L);
    }
}

/*
 * Pair energy (shifted; smoothed when h > 0) and force factor ff with
 * F_vec = ff * d_vec; both zero at and beyond the cutoff.  Smoothing:
 *   V_s(r) = V_ts(r) g(x),  x = (r - rc) / (h sig),  g(x) = x^4 / (1 + x^4)
 *   -dV_s/dr = (-dV_ts/dr) g(x) - V_ts(r) g'(x) / (h sig),
 *   g'(x) = 4 x^3 / (1 + x^4)^2.
 */
void orc_pair(double r2, double eps, double sig, double rc, double h,
              double *v_shifted, double *ff)
{
    if (!(r2 < rc * rc)) {
        *v_shifted = 0.0;
        *ff = 0.0;
        return;
    }
    double v = lj_v(r2, eps, sig) - lj_v(rc * rc, eps, sig);
    double f = lj_ff(r2, eps, sig); /* (-dV/dr) / r */
    if (h > 0.0) {
        double r = sqrt(r2);
        double x = (r - rc) / (h * sig);
        double x2 = x * x, x4 = x2 * x2;
        double g = x4 / (1.0 + x4);
        double dg = 4.0 * x2 * x / ((1.0 + x4) * (1.0 + x4));
        f = f * g - v * dg / (h * sig) / r;
        v = v * g;
    }
    *v_shifted = v;
    *ff = f;
}

/*
 * Forces, per-particle energy and per-particle virial for the particles in
 * `sel` (all particles when sel == NULL, m == n):
 *   F_i   = sum_{j != i} ff(r_ij) d_ij
 *   e_i   = 1/2 sum_{j != i} V_ts(r_ij)     (sum_i e_i = E_pot)
 *   w_i   = 1/2 sum_{j != i} ff(r_ij) r_ij^2 (sum_i w_i = W = sum_{i<j} d.F)
 */
void orc_forces(int n, double L, const int *species, const double *pos,
                int n_species, const double *eps, const double *sig,
                const double *rc, double h, const int *sel, int m, double *f,
                double *e_i, double *w_i)
{
    orc_table t;
    make_table(&t, n_species, eps, sig, rc);
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < m; ++k) {
        int i = sel ? sel[k] : k;
        double fx = 0, fy = 0, fz = 0, e = 0, w = 0;
        int si = n_species > 1 ? species[i] : 0;
        for (int j = 0; j < n; ++j) {
            if (j == i)
                continue;
            int sj = n_species > 1 ? species[j] : 0;
            double d[3];
            min_image(pos + 3 * i, pos + 3 * j, L, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double v, ff;
            orc_pair(r2, t.eps[si][sj], t.sig[si][sj], t.rc[si][sj], h, &v, &ff);
            fx += ff * d[0];
            fy += ff * d[1];
            fz += ff * d[2];
            e += 0.5 * v;
            w += 0.5 * ff * r2;
        }
        if (f) {
            f[3 * k + 0] = fx;
            f[3 * k + 1] = fy;
            f[3 * k + 2] = fz;
        }
        if (e_i)
            e_i[k] = e;
        if (w_i)
            w_i[k] = w;
    }
}

/*
 * Neighbour-list membership for the particles in `sel`: every j != i with
 * |d_ij| < rlist_{s_i s_j}, in ascending j.  counts[k] holds the full count
 * even when it exceeds cap (only the first cap ids are stored).
 */
void orc_neighbours(int n, double L, const int *species, const double *pos,
                    int n_species, const double *rlist, const int *sel, int m,
                    int cap, int *counts, int *ids)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < m; ++k) {
        int i = sel ? sel[k] : k;
        int si = n_species > 1 ? species[i] : 0;
        int c = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i)
                continue;
            int sj = n_species > 1 ? species[j] : 0;
            double d[3];
            min_image(pos + 3 * i, pos + 3 * j, L, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double rl = rlist[2 * si + sj];
            if (r2 < rl * rl) {
                if (c < cap)
                    ids[(int64_t)k * cap + c] = j;
                ++c;
            }
        }
        counts[k] = c;
    }
}

/*
 * Velocity Verlet for `steps` steps (equal masses m), forces by brute force.
 * pos/vel are updated in place; pos is wrapped into [0, L) every step and the
 * number of box lengths crossed is accumulated in `image` (may be NULL).
 * Returns the forces at the final positions in f (may be NULL).
 */
void orc_vv(int n, double L, const int *species, double *pos, double *vel,
            int *image, int n_species, const double *eps, const double *sig,
            const double *rc, double h, double mass, double dt, int steps,
            double *f_out)
{
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    orc_forces(n, L, species, pos, n_species, eps, sig, rc, h, NULL, n, f, NULL,
               NULL);
    double hk = 0.5 * dt / mass; /* half-kick factor */
    for (int s = 0; s < steps; ++s) {
        for (int i = 0; i < 3 * n; ++i) {
            vel[i] += hk * f[i];
            pos[i] += dt * vel[i];
            double k = floor(pos[i] / L);
            pos[i] -= k * L;
            if (pos[i] >= L) { /* rounding edge: r == L maps to 0 */
                pos[i] -= L;
                k += 1.0;
            }
            if (pos[i] < 0.0) {
                pos[i] += L;
                k -= 1.0;
            }
            if (image)
                image[i] += (int)k;
        }
        orc_forces(n, L, species, pos, n_species, eps, sig, rc, h, NULL, n, f,
                   NULL, NULL);
        for (int i = 0; i < 3 * n; ++i)
            vel[i] += hk * f[i];
    }
    if (f_out)
        memcpy(f_out, f, sizeof(double) * 3 * (size_t)n);
    free(f);
}


/* ======================================================================
 * Cell-list variant (an independent, faster route to the same definition).
 *
 * Sec. 2.2 bins the particles into cells no smaller than the interaction
 * range, so that every partner of a particle lies in its own cell or one of
 * the 26 adjacent cells, and keeps Verlet lists of all partners within the
 * cutoff plus a skin, rebuilt once some particle has moved more than half
 * the skin since the last build.  The functions below do exactly that on the
 * CPU in FP64.  They reach the same forces as orc_forces up to the order of
 * the floating-point sums (they visit the partners in another order), and
 * the tests pin them against orc_forces and orc_vv.
 * ====================================================================== */

/* Fold x into [0, L): the image counter is floor(x / L); the rounding edge
 * fl(x - L floor(x/L)) == L is mapped to 0. */
static double fold_into_box(double x, double L)
{
    double w = x - L * floor(x / L);
    if (w >= L)
        w -= L;
    if (w < 0.0)
        w += L;
    return w;
}

/* Cell grid: nc cells per edge of width L/nc >= reach, and for every cell
 * the particles in it (counting sort by cell, ascending particle index).
 * nc < 3 means one cell (all pairs). */
typedef struct {
    int nc;
    int *start; /* nc^3 + 1 */
    int *list;  /* n */
} orc_cells;

static void cells_build(orc_cells *g, int n, double L, const double *pos, double reach)
{
    int nc = (int)floor(L / reach);
    if (nc < 3)
        nc = 1;
    int ncell = nc * nc * nc;
    int *cell = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    g->nc = nc;
    g->start = (int *)calloc((size_t)ncell + 1, sizeof(int));
    g->list = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        int c[3];
        for (int d = 0; d < 3; ++d) {
            int k = (int)(fold_into_box(pos[3 * i + d], L) / L * nc);
            c[d] = k < 0 ? 0 : (k >= nc ? nc - 1 : k);
        }
        cell[i] = c[0] + nc * (c[1] + nc * c[2]);
        g->start[cell[i] + 1]++;
    }
    for (int c = 0; c < ncell; ++c)
        g->start[c + 1] += g->start[c];
    int *fill = (int *)malloc(sizeof(int) * (size_t)ncell);
    memcpy(fill, g->start, sizeof(int) * (size_t)ncell);
    for (int i = 0; i < n; ++i)
        g->list[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
}

static void cells_free(orc_cells *g)
{
    free(g->start);
    free(g->list);
}

/* The (up to) 27 distinct cells around the cell of particle i. */
static int cells_around(const orc_cells *g, double L, const double *ri, int out[27])
{
    int nc = g->nc;
    if (nc == 1) {
        out[0] = 0;
        return 1;
    }
    int c[3];
    for (int d = 0; d < 3; ++d) {
        int k = (int)(fold_into_box(ri[d], L) / L * nc);
        c[d] = k < 0 ? 0 : (k >= nc ? nc - 1 : k);
    }
    int m = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int x = (c[0] + dx + nc) % nc, y = (c[1] + dy + nc) % nc, z = (c[2] + dz + nc) % nc;
                out[m++] = x + nc * (y + nc * z);
            }
    return m;
}

static double max_cutoff(const orc_table *t)
{
    double m = 0.0;
    for (int a = 0; a < t->n_species; ++a)
        for (int b = 0; b < t->n_species; ++b)
            if (t->rc[a][b] > m)
                m = t->rc[a][b];
    return m;
}

/* Forces, e_i and w_i (as in orc_forces) for all n particles, each
 * particle's partners found in its own and the adjacent cells. */
void orc_forces_cells(int n, double L, const int *species, const double *pos, int n_species,
                      const double *eps, const double *sig, const double *rc, double h, double *f,
                      double *e_i, double *w_i)
{
    orc_table t;
    make_table(&t, n_species, eps, sig, rc);
    orc_cells g;
    cells_build(&g, n, L, pos, max_cutoff(&t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int nb[27];
        int m = cells_around(&g, L, pos + 3 * i, nb);
        int si = n_species > 1 ? species[i] : 0;
        double fx = 0, fy = 0, fz = 0, e = 0, w = 0;
        for (int q = 0; q < m; ++q)
            for (int k = g.start[nb[q]]; k < g.start[nb[q] + 1]; ++k) {
                int j = g.list[k];
                if (j == i)
                    continue;
                int sj = n_species > 1 ? species[j] : 0;
                double d[3];
                min_image(pos + 3 * i, pos + 3 * j, L, d);
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                double v, ff;
                orc_pair(r2, t.eps[si][sj], t.sig[si][sj], t.rc[si][sj], h, &v, &ff);
                fx += ff * d[0];
                fy += ff * d[1];
                fz += ff * d[2];
                e += 0.5 * v;
                w += 0.5 * ff * r2;
            }
        if (f) {
            f[3 * i + 0] = fx;
            f[3 * i + 1] = fy;
            f[3 * i + 2] = fz;
        }
        if (e_i)
            e_i[i] = e;
        if (w_i)
            w_i[i] = w;
    }
    cells_free(&g);
}

/* Verlet lists: for every i, all j != i with |d_ij| < max cutoff + skin
 * (a superset of every pair's list radius: the force test below still uses
 * each pair's own cutoff), found through cells of edge >= that radius. */
typedef struct {
    int *start; /* n + 1 */
    int *nbr;
} orc_vlist;

static void vlist_build(orc_vlist *vl, int n, double L, const double *pos, double rl)
{
    orc_cells g;
    cells_build(&g, n, L, pos, rl);
    int *cnt = (int *)calloc((size_t)n + 1, sizeof(int));
    /* two passes (count, then fill) so the list needs no capacity */
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int i = 0; i < n; ++i) {
            int nb[27];
            int m = cells_around(&g, L, pos + 3 * i, nb);
            int c = 0;
            int *out = pass ? vl->nbr + vl->start[i] : NULL;
            for (int q = 0; q < m; ++q)
                for (int k = g.start[nb[q]]; k < g.start[nb[q] + 1]; ++k) {
                    int j = g.list[k];
                    if (j == i)
                        continue;
                    double d[3];
                    min_image(pos + 3 * i, pos + 3 * j, L, d);
                    if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rl * rl) {
                        if (out)
                            out[c] = j;
                        ++c;
                    }
                }
            if (!pass)
                cnt[i] = c;
        }
        if (!pass) {
            vl->start = (int *)malloc(sizeof(int) * ((size_t)n + 1));
            vl->start[0] = 0;
            for (int i = 0; i < n; ++i)
                vl->start[i + 1] = vl->start[i] + cnt[i];
            vl->nbr = (int *)malloc(sizeof(int) * (size_t)(vl->start[n] > 0 ? vl->start[n] : 1));
        }
    }
    free(cnt);
    cells_free(&g);
}

static void vlist_free(orc_vlist *vl)
{
    free(vl->start);
    free(vl->nbr);
}

static void vlist_forces(const orc_vlist *vl, int n, double L, const int *species, const double *pos,
                         const orc_table *t, double h, double *f)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int si = t->n_species > 1 ? species[i] : 0;
        double fx = 0, fy = 0, fz = 0;
        for (int k = vl->start[i]; k < vl->start[i + 1]; ++k) {
            int j = vl->nbr[k];
            int sj = t->n_species > 1 ? species[j] : 0;
            double d[3];
            min_image(pos + 3 * i, pos + 3 * j, L, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double v, ff;
            orc_pair(r2, t->eps[si][sj], t->sig[si][sj], t->rc[si][sj], h, &v, &ff);
            fx += ff * d[0];
            fy += ff * d[1];
            fz += ff * d[2];
        }
        f[3 * i + 0] = fx;
        f[3 * i + 1] = fy;
        f[3 * i + 2] = fz;
    }
}

/*
 * Velocity Verlet as orc_vv, with forces over Verlet lists of radius
 * max cutoff + skin (skin > 0) built through cells, rebuilt before a force
 * evaluation whenever some particle has moved more than skin/2 (minimum
 * image) since the last build.  Returns the number of list builds.
 */
int orc_vv_lists(int n, double L, const int *species, double *pos, double *vel, int *image,
                 int n_species, const double *eps, const double *sig, const double *rc, double h,
                 double mass, double dt, double skin, int steps, double *f_out)
{
    orc_table t;
    make_table(&t, n_species, eps, sig, rc);
    double rl = max_cutoff(&t) + skin;
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *ref = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    orc_vlist vl;
    vlist_build(&vl, n, L, pos, rl);
    memcpy(ref, pos, sizeof(double) * 3 * (size_t)n);
    int builds = 1;
    vlist_forces(&vl, n, L, species, pos, &t, h, f);
    double hk = 0.5 * dt / mass;
    for (int s = 0; s < steps; ++s) {
        for (int i = 0; i < 3 * n; ++i) {
            vel[i] += hk * f[i];
            pos[i] += dt * vel[i];
            double k = floor(pos[i] / L);
            pos[i] -= k * L;
            if (pos[i] >= L) {
                pos[i] -= L;
                k += 1.0;
            }
            if (pos[i] < 0.0) {
                pos[i] += L;
                k -= 1.0;
            }
            if (image)
                image[i] += (int)k;
        }
        double dmax2 = 0.0;
        for (int i = 0; i < n; ++i) {
            double d[3];
            min_image(pos + 3 * i, ref + 3 * i, L, d);
            double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (d2 > dmax2)
                dmax2 = d2;
        }
        if (dmax2 > 0.25 * skin * skin) {
            vlist_free(&vl);
            vlist_build(&vl, n, L, pos, rl);
            memcpy(ref, pos, sizeof(double) * 3 * (size_t)n);
            ++builds;
        }
        vlist_forces(&vl, n, L, species, pos, &t, h, f);
        for (int i = 0; i < 3 * n; ++i)
            vel[i] += hk * f[i];
    }
    if (f_out)
        memcpy(f_out, f, sizeof(double) * 3 * (size_t)n);
    vlist_free(&vl);
    free(ref);
    free(f);
    return builds;
}
