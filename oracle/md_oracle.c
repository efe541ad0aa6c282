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
 *     continuous; the force is not shifted (reading of "cut off at rc");
 *   - KA mixture: per-species-pair eps/sigma (Sec. 5), rc_ab = 2.5 sigma_ab;
 *   - minimum image in a cubic periodic box, d -= L * nearbyint(d / L);
 *   - forces by brute force over every j != i, O(N^2), no neighbour lists;
 *   - velocity Verlet (Sec. 2.2, "The MD integration step"):
 *       v += dt/(2m) F;  r += dt v;  wrap r into [0, L);  F = F(r);
 *       v += dt/(2m) F;
 *   - neighbour-list membership (Sec. 2.2: every particle within the cutoff
 *     plus a skin): j in L_i  iff  j != i and |d_ij| < rc_{s_i s_j} + skin.
 *
 * Everything is double precision; OpenMP parallelises over i only (each i is
 * an independent sum in a fixed j order).
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

/* Pair energy (shifted) and force factor; zero at and beyond the cutoff. */
void orc_pair(double r2, double eps, double sig, double rc, double *v_shifted,
              double *ff)
{
    if (r2 < rc * rc) {
        *v_shifted = lj_v(r2, eps, sig) - lj_v(rc * rc, eps, sig);
        *ff = lj_ff(r2, eps, sig);
    } else {
        *v_shifted = 0.0;
        *ff = 0.0;
    }
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
                const double *rc, const int *sel, int m, double *f,
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
            orc_pair(r2, t.eps[si][sj], t.sig[si][sj], t.rc[si][sj], &v, &ff);
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
            const double *rc, double mass, double dt, int steps, double *f_out)
{
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    orc_forces(n, L, species, pos, n_species, eps, sig, rc, NULL, n, f, NULL,
               NULL);
    double h = 0.5 * dt / mass;
    for (int s = 0; s < steps; ++s) {
        for (int i = 0; i < 3 * n; ++i) {
            vel[i] += h * f[i];
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
        orc_forces(n, L, species, pos, n_species, eps, sig, rc, NULL, n, f,
                   NULL, NULL);
        for (int i = 0; i < 3 * n; ++i)
            vel[i] += h * f[i];
    }
    if (f_out)
        memcpy(f_out, f, sizeof(double) * 3 * (size_t)n);
    free(f);
}
