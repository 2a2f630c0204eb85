/*
 * Random sequential addition (RSA) of spheres into a box: the seeded initial
 * configurations used by tests and benchmarks.  This file only places
 * non-overlapping spheres (plus, optionally, spheres that touch one earlier
 * sphere with a small prescribed overlap); it contains no contact law, no
 * time integration and nothing else of the simulated method.
 *
 * Random numbers come from splitmix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), seeded by the caller.
 *
 * Built by gen/__init__.py with gcc into gen/librsa.so.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sm_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
/* uniform double in [0,1) from the top 53 bits */
static double sm_unif(uint64_t *s) { return (double)(sm_next(s) >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
    double lo[3], L[3], cell;
    int nc[3];
    uint32_t periodic;
    int *head, *next;
    const double *x, *r;
} grid_t;

static int cell_of(const grid_t *g, const double *p, int ax) {
    int c = (int)floor((p[ax] - g->lo[ax]) / g->cell);
    if (c < 0) c = 0;
    if (c >= g->nc[ax]) c = g->nc[ax] - 1;
    return c;
}

/* Returns 1 if a sphere of radius rr at p overlaps any placed sphere other
 * than `skip`; periodic axes use the minimum image. */
static int overlaps(const grid_t *g, const double *p, double rr, int skip) {
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = cell_of(g, p, a);
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                int o[3] = {ox, oy, oz}, q[3];
                int ok = 1;
                for (int a = 0; a < 3; ++a) {
                    q[a] = c[a] + o[a];
                    if (q[a] < 0 || q[a] >= g->nc[a]) {
                        if (g->periodic & (1u << a)) q[a] = (q[a] + g->nc[a]) % g->nc[a];
                        else ok = 0;
                    }
                }
                if (!ok) continue;
                /* with fewer than 3 cells on a periodic axis the wrapped
                 * offsets repeat; skip the repeats */
                int dup = 0;
                for (int a = 0; a < 3; ++a)
                    if ((g->periodic & (1u << a)) && g->nc[a] < 3 && o[a] != 0) {
                        if (g->nc[a] == 1) dup = 1;
                        if (g->nc[a] == 2 && o[a] == 1) dup = 1;
                    }
                if (dup) continue;
                int cid = (q[2] * g->nc[1] + q[1]) * g->nc[0] + q[0];
                for (int k = g->head[cid]; k >= 0; k = g->next[k]) {
                    if (k == skip) continue;
                    double d2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double d = g->x[3 * k + a] - p[a];
                        if (g->periodic & (1u << a)) {
                            if (d > 0.5 * g->L[a]) d -= g->L[a];
                            else if (d < -0.5 * g->L[a]) d += g->L[a];
                        }
                        d2 += d * d;
                    }
                    double s = g->r[k] + rr;
                    if (d2 < s * s) return 1;
                }
            }
    return 0;
}

/*
 * Place n spheres of radii r[0..n) (in that order) into [lo, hi).
 *   periodic      bit a set: axis a is periodic (no wall clearance needed)
 *   p_touch       probability that a new sphere is placed touching a random
 *                 earlier sphere q, at overlap dn = f * min(r, r_q) with
 *                 f ~ U[0, touch_max)
 *   max_attempts  per sphere
 * Output x (3n, xyz interleaved).  Returns the number placed (n on success).
 */
int rsa_place(int n, const double *r, const double *lo, const double *hi, uint32_t periodic,
              double p_touch, double touch_max, uint64_t seed, int max_attempts, double *x) {
    grid_t g;
    double rmax = 0.0;
    for (int i = 0; i < n; ++i) if (r[i] > rmax) rmax = r[i];
    g.cell = 2.0 * rmax;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = lo[a];
        g.L[a] = hi[a] - lo[a];
        g.nc[a] = (int)floor(g.L[a] / g.cell);
        if (g.nc[a] < 1) g.nc[a] = 1;
    }
    g.cell = fmax(g.cell, 0.0);
    /* cells must be at least 2 rmax wide along every axis */
    double cw = 1e300;
    for (int a = 0; a < 3; ++a) cw = fmin(cw, g.L[a] / g.nc[a]);
    g.cell = cw;
    for (int a = 0; a < 3; ++a) {
        g.nc[a] = (int)floor(g.L[a] / g.cell);
        if (g.nc[a] < 1) g.nc[a] = 1;
    }
    g.periodic = periodic;
    long ncell = (long)g.nc[0] * g.nc[1] * g.nc[2];
    g.head = (int *)malloc(sizeof(int) * ncell);
    g.next = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (long c = 0; c < ncell; ++c) g.head[c] = -1;
    g.x = x;
    g.r = r;
    uint64_t st = seed;
    int placed = 0;
    for (int i = 0; i < n; ++i) {
        double rr = r[i];
        int ok = 0;
        for (int att = 0; att < max_attempts && !ok; ++att) {
            double p[3];
            int skip = -1;
            if (placed > 0 && p_touch > 0.0 && sm_unif(&st) < p_touch) {
                int q = (int)(sm_unif(&st) * placed);
                if (q >= placed) q = placed - 1;
                double z = 2.0 * sm_unif(&st) - 1.0, ph = 6.283185307179586 * sm_unif(&st);
                double sxy = sqrt(fmax(0.0, 1.0 - z * z));
                double u[3] = {sxy * cos(ph), sxy * sin(ph), z};
                double f = touch_max * sm_unif(&st);
                double dn = f * fmin(rr, r[q]);
                double dist = r[q] + rr - dn;
                for (int a = 0; a < 3; ++a) p[a] = x[3 * q + a] + u[a] * dist;
                skip = q;
            } else {
                for (int a = 0; a < 3; ++a) {
                    if (periodic & (1u << a)) p[a] = lo[a] + sm_unif(&st) * g.L[a];
                    else p[a] = lo[a] + rr + sm_unif(&st) * (g.L[a] - 2.0 * rr);
                }
            }
            int inside = 1;
            for (int a = 0; a < 3; ++a) {
                if (periodic & (1u << a)) {
                    while (p[a] >= hi[a]) p[a] -= g.L[a];
                    while (p[a] < lo[a]) p[a] += g.L[a];
                } else if (p[a] - rr < lo[a] || p[a] + rr > hi[a]) {
                    inside = 0;
                }
            }
            if (!inside) continue;
            if (overlaps(&g, p, rr, skip)) continue;
            for (int a = 0; a < 3; ++a) x[3 * i + a] = p[a];
            int cid = (cell_of(&g, p, 2) * g.nc[1] + cell_of(&g, p, 1)) * g.nc[0] + cell_of(&g, p, 0);
            g.next[i] = g.head[cid];
            g.head[cid] = i;
            ok = 1;
        }
        if (!ok) break;
        ++placed;
    }
    free(g.head);
    free(g.next);
    return placed;
}
