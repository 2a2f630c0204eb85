/*
 * dem_oracle.c -- plain, slow, FP64 reference of one DEM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the simulator links, loads or calls
 * this file; it exists so that tests, the smoke check and the benchmark's CPU
 * baseline can compare the GPU library against an independent reading of the
 * paper (Nakahara & Washizawa, "Accelerating DEM simulations on GPUs by
 * reducing the impact of warp divergences", arXiv:1503.03553).  It shares no
 * source with the GPU path.
 *
 * What one step computes (section 2 of the paper, "Particle simulations based
 * on DEM"):
 *   1. contact set: every ordered pair (i, j), i != j, with
 *      |x_j - x_i|^2 < (r_i + r_j)^2, and every box face closer than r_i;
 *   2. per contact, in ascending partner id with faces last: normal overlap
 *      dn, Eq. (2) tangential relative velocity, Eq. (3) tangential
 *      displacement, Hertz/Mindlin stiffnesses, damping, Eq. (1) force,
 *      Eq. (4) sliding cap with the displacement recomputed from the capped
 *      force, and the torque T = r (n x F);
 *   3. per-particle sums plus gravity m g (kernel list: "ForceGravity");
 *   4. semi-implicit Euler update of velocity, position, angular velocity
 *      (kernel list: "Integrate"; the paper does not name the scheme);
 *   5. the new pair history replaces the old one: pairs no longer touching
 *      are forgotten (kernel list: "InitializeContactIDs").
 *
 * Readings of points the paper leaves open (all documented in the design
 * notes of the repository):
 *   - n points from particle i to its partner; v = v_i - v_j; F acts on i;
 *   - k_n uses (2 - sigma^2)/E as printed (kn_form 0) or the textbook
 *     (1 - sigma^2)/E (kn_form 1);
 *   - alpha(eps) = -sqrt(5) ln(eps) / sqrt(ln(eps)^2 + pi^2), the damping
 *     prefactor for which a head-on collision under this force law restitutes
 *     exactly eps;
 *   - pair restitution and friction are the means of the two materials';
 *     a box face takes the particle's own material, infinite radius and mass;
 *   - extra walls (kernel list: "CollideRectangle", "CollideLine") are
 *     static closed rectangles or segments acting like a box face; the
 *     contact point is the wall's point closest to the centre, the normal
 *     points from the centre to it, the overlap is r_i minus that distance;
 *     a centre exactly on a rectangle takes the normal u x v, a centre
 *     exactly on a segment makes no contact;
 *   - solid spheres: m = rho 4/3 pi r^3, I = 2/5 m r^2;
 *   - Lees-Edwards shear along x with gradient along y when shear_rate != 0.
 *
 * Built with gcc -O2 -ffp-contract=off -fno-fast-math (optionally -fopenmp).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXMAT 8
#define ORC_FACE_ID 0xFFFFFFF0u /* partner id of box face f is ORC_FACE_ID + f */
#define ORC_MAX_WALLS 10        /* extra wall k has partner id ORC_FACE_ID + 6 + k */

/* An extra wall: kind 0 the rectangle p + s u + t v (u and v orthogonal),
 * kind 1 the segment p + s u; s, t in [0, 1]. */
typedef struct {
    int32_t kind;
    int32_t pad;
    double p[3], u[3], v[3];
} orc_wall;

typedef struct {
    double lo[3], hi[3];
    uint32_t walls;    /* bit 2a: low face of axis a, bit 2a+1: high face */
    uint32_t periodic; /* bit a: axis a periodic */
    double gravity[3];
    double shear_rate; /* Lees-Edwards: d(v_x)/dy, needs periodic x and y */
    double time;       /* simulation time at the start of the step */
    double dt;
    int32_t kn_form;
    int32_t n_mats;
    double E[ORC_MAXMAT], poisson[ORC_MAXMAT], G[ORC_MAXMAT];
    double density[ORC_MAXMAT], restitution[ORC_MAXMAT], mu[ORC_MAXMAT];
    int32_t n_extra;
    int32_t pad;
    orc_wall extra[ORC_MAX_WALLS];
} orc_params;

/* ------------------------------------------------------------ constants */
static const double ORC_PI = 3.14159265358979323846;

/* Damping prefactor alpha(eps) of the damping coefficient
 * eta = alpha sqrt(m* k_n sqrt(dn)) (section 2, definition of eta). */
double orc_alpha(double eps) {
    if (eps >= 1.0) return 0.0;
    double l = log(eps);
    return -sqrt(5.0) * l / sqrt(l * l + ORC_PI * ORC_PI);
}

double orc_mass(double rho, double r) { return rho * (4.0 / 3.0) * ORC_PI * r * r * r; }
double orc_inertia(double m, double r) { return 0.4 * m * r * r; }

/* Normal stiffness k_n (section 2).  rj <= 0 means a box face (r* = ri). */
double orc_kn(const orc_params *P, int mi, int mj, double ri, double rj) {
    double rs = rj > 0.0 ? ri * rj / (ri + rj) : ri;
    double ci, cj;
    if (P->kn_form == 1) {
        ci = 1.0 - P->poisson[mi] * P->poisson[mi];
        cj = 1.0 - P->poisson[mj] * P->poisson[mj];
    } else {
        ci = 2.0 - P->poisson[mi] * P->poisson[mi];
        cj = 2.0 - P->poisson[mj] * P->poisson[mj];
    }
    return 4.0 / 3.0 * sqrt(rs) / (ci / P->E[mi] + cj / P->E[mj]);
}

/* Tangential stiffness k_t at overlap dn (section 2). */
double orc_kt(const orc_params *P, int mi, int mj, double ri, double rj, double dn) {
    double rs = rj > 0.0 ? ri * rj / (ri + rj) : ri;
    double gi = (2.0 - P->poisson[mi]) / P->G[mi];
    double gj = (2.0 - P->poisson[mj]) / P->G[mj];
    return 8.0 * sqrt(rs * dn) / (gi + gj);
}

/* Beta function via log-gamma. */
static double orc_beta(double a, double b) { return exp(lgamma(a) + lgamma(b) - lgamma(a + b)); }

/* Duration of an undamped head-on Hertz contact: integrating
 * m* s'' = -k_n s^(3/2) from s = 0, s' = v0 until s returns to 0 gives
 * t_c = (4/5) B(2/5, 1/2) (5/4)^(2/5) (m_star / k_n)^(2/5) v0^(-1/5). */
double orc_contact_time(double mstar, double kn, double v0) {
    double c = 0.8 * orc_beta(0.4, 0.5) * pow(1.25, 0.4);
    return c * pow(mstar / kn, 0.4) * pow(v0, -0.2);
}

/* Time-step rule: t_c / 50 for two spheres of the smallest radius (and that
 * sphere's material) approaching at 0.1 m/s. */
double orc_dt_rule(const orc_params *P, long n, const double *r, const uint16_t *mat) {
    long k = 0;
    for (long i = 1; i < n; ++i) if (r[i] < r[k]) k = i;
    int m = mat ? mat[k] : 0;
    double mi = orc_mass(P->density[m], r[k]);
    double ms = mi * mi / (mi + mi);
    double kn = orc_kn(P, m, m, r[k], r[k]);
    return orc_contact_time(ms, kn, 0.1) / 50.0;
}

/* ------------------------------------------------------ the contact law */
typedef struct {
    double F[3], T[3], dt[3];
    double dn;
    int capped;
    /* diagnostics (not used by the step): of the sliding test, |F_t| before
     * the cap, mu |F_n|, and the sum of the magnitudes of the terms that
     * enter both (k_t |dt|, eta (|v| + |r1 w1 + r2 w2|), mu (k_n dn^1.5 +
     * eta |v|)), the scale of the rounding of a lower-precision evaluation;
     * of Eq. (1), the sum of the magnitudes of its four terms before the cap
     * (k_n dn^1.5 + eta |v_n| + k_t |dt| + eta |v_t|), the scale of the
     * rounding of a lower-precision evaluation of the force; and k_t */
    double ft_pre, mufn, scale, fterm, kt;
} orc_pair_out;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Extra wall W and a centre c: w = q - c for the wall's point q closest to
 * c (the parameters s, t of the rectangle or segment clamped to [0, 1]);
 * returns |w|^2.  No fused multiply-add anywhere, so the contact decision
 * |w|^2 < r^2 is reproducible bit for bit. */
static double orc_wall_gap(const orc_wall *W, const double *c, double *wv) {
    double d[3], q[3];
    for (int a = 0; a < 3; ++a) d[a] = c[a] - W->p[a];
    double s = dot3(d, W->u) / dot3(W->u, W->u);
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    for (int a = 0; a < 3; ++a) q[a] = W->p[a] + s * W->u[a];
    if (W->kind == 0) {
        double t = dot3(d, W->v) / dot3(W->v, W->v);
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        for (int a = 0; a < 3; ++a) q[a] = q[a] + t * W->v[a];
    }
    for (int a = 0; a < 3; ++a) wv[a] = q[a] - c[a];
    double d2 = wv[0] * wv[0] + wv[1] * wv[1];
    return d2 + wv[2] * wv[2];
}

/* Whether a sphere of radius ri centred at c touches extra wall W. */
static int orc_wall_touch(const orc_wall *W, const double *c, double ri) {
    double wv[3];
    double d2 = orc_wall_gap(W, c, wv);
    return d2 < ri * ri && (W->kind == 0 || d2 > 0.0);
}

/* Unit normal from the centre c towards extra wall W and the overlap. */
static void orc_wall_normal(const orc_wall *W, const double *c, double ri, double *n, double *dn) {
    double wv[3];
    double d = sqrt(orc_wall_gap(W, c, wv));
    if (d > 0.0) {
        for (int a = 0; a < 3; ++a) n[a] = wv[a] / d;
    } else {
        cross3(W->u, W->v, n);
        double l = sqrt(dot3(n, n));
        for (int a = 0; a < 3; ++a) n[a] = n[a] / l;
    }
    *dn = ri - d;
}

/*
 * Force, torque and new tangential displacement of one contact acting on
 * particle i (Eq. 1 - 4 and the torque line of section 2).
 *   n     unit normal from i towards its partner
 *   dn    normal overlap
 *   v     relative velocity v_i - v_j (centre velocities)
 *   rw    r_i w_i + r_j w_j  (a face contributes nothing)
 *   rs    r* ; ms  m*
 *   face  1 for a box face (then mj = mi)
 */
void orc_contact_law(const orc_params *P, int mi, int mj, double ri, double rs, double ms,
                     const double *n, double dn, const double *v, const double *rw,
                     const double *dt_old, orc_pair_out *o) {
    /* Eq. (2): v_t = v - (v.n) n + (r1 w1 + r2 w2) x n */
    double vns = dot3(v, n), vn[3], vt[3], rwxn[3];
    cross3(rw, n, rwxn);
    for (int a = 0; a < 3; ++a) {
        vn[a] = vns * n[a];
        vt[a] = v[a] - vn[a] + rwxn[a];
    }
    /* Eq. (3): project the old displacement onto the tangent plane, integrate v_t */
    double dtn = dot3(dt_old, n), dtv[3];
    for (int a = 0; a < 3; ++a) dtv[a] = dt_old[a] - dtn * n[a] + vt[a] * P->dt;

    /* stiffnesses and damping */
    double ci, cj;
    if (P->kn_form == 1) {
        ci = 1.0 - P->poisson[mi] * P->poisson[mi];
        cj = 1.0 - P->poisson[mj] * P->poisson[mj];
    } else {
        ci = 2.0 - P->poisson[mi] * P->poisson[mi];
        cj = 2.0 - P->poisson[mj] * P->poisson[mj];
    }
    double kn = 4.0 / 3.0 * sqrt(rs) / (ci / P->E[mi] + cj / P->E[mj]);
    double kt = 8.0 * sqrt(rs * dn) /
                ((2.0 - P->poisson[mi]) / P->G[mi] + (2.0 - P->poisson[mj]) / P->G[mj]);
    double eps = 0.5 * (P->restitution[mi] + P->restitution[mj]);
    double eta = orc_alpha(eps) * sqrt(ms * kn * sqrt(dn));
    double mu = 0.5 * (P->mu[mi] + P->mu[mj]);

    /* Eq. (1) split into its normal and tangential parts */
    double Fn[3], Ft[3];
    double el = kn * pow(dn, 1.5);
    for (int a = 0; a < 3; ++a) {
        Fn[a] = -el * n[a] - eta * vn[a];
        Ft[a] = -kt * dtv[a] - eta * vt[a];
    }
    double fn = sqrt(dot3(Fn, Fn)), ft = sqrt(dot3(Ft, Ft));
    o->ft_pre = ft;
    o->mufn = mu * fn;
    o->scale = kt * sqrt(dot3(dtv, dtv)) + eta * (sqrt(dot3(v, v)) + sqrt(dot3(rw, rw))) +
               mu * (el + eta * sqrt(dot3(v, v)));
    o->fterm = el + eta * sqrt(dot3(vn, vn)) + kt * sqrt(dot3(dtv, dtv)) + eta * sqrt(dot3(vt, vt));
    o->kt = kt;
    o->capped = 0;
    /* Eq. (4): sliding friction, then the displacement that reproduces it */
    if (ft > mu * fn) {
        double s = mu * fn / ft;
        for (int a = 0; a < 3; ++a) {
            Ft[a] = s * Ft[a];
            dtv[a] = -Ft[a] / kt;
        }
        o->capped = 1;
    }
    double F[3];
    for (int a = 0; a < 3; ++a) F[a] = Fn[a] + Ft[a];
    /* T = r (n x F), lever arm the full radius of particle i */
    double nxF[3];
    cross3(n, F, nxF);
    for (int a = 0; a < 3; ++a) {
        o->F[a] = F[a];
        o->T[a] = ri * nxF[a];
        o->dt[a] = dtv[a];
    }
    o->dn = dn;
}

/* ----------------------------------------------------- images and shifts */
/* Shear offset of the periodic images along x at time t. */
double orc_le_offset(const orc_params *P, double t) {
    if (P->shear_rate == 0.0) return 0.0;
    double Lx = P->hi[0] - P->lo[0], Ly = P->hi[1] - P->lo[1];
    double u = P->shear_rate * Ly;
    return fmod(u * t, Lx);
}

typedef struct {
    int k[3];
    double S[3];  /* position shift of the partner's image */
    double dvx;   /* velocity of the partner's image along x, added to v_j */
} orc_image;

/* All images of a partner that may touch: (0,0,0) plus periodic copies.
 * Image (kx, ky, kz) sits at x_j + (kx Lx + ky D, ky Ly, kz Lz) and moves
 * with v_j + ky shear_rate Ly e_x (Lees-Edwards). */
static int orc_images(const orc_params *P, double t, orc_image *out) {
    double L[3];
    for (int a = 0; a < 3; ++a) L[a] = P->hi[a] - P->lo[a];
    double D = orc_le_offset(P, t);
    int rx = (P->periodic & 1u) ? 2 : 0;
    int ry = (P->periodic & 2u) ? 1 : 0;
    int rz = (P->periodic & 4u) ? 1 : 0;
    int m = 0;
    for (int kz = -rz; kz <= rz; ++kz)
        for (int ky = -ry; ky <= ry; ++ky)
            for (int kx = -rx; kx <= rx; ++kx) {
                orc_image *im = &out[m++];
                im->k[0] = kx; im->k[1] = ky; im->k[2] = kz;
                im->S[0] = (double)kx * L[0] + (double)ky * D;
                im->S[1] = (double)ky * L[1];
                im->S[2] = (double)kz * L[2];
                im->dvx = (double)ky * P->shear_rate * L[1];
            }
    return m;
}

/* The contact predicate on FP64 positions, evaluated as written with no
 * fused multiply-add: ((dx^2 + dy^2) + dz^2) < (ri + rj)^2. */
static int orc_touch(const double *dx, double ri, double rj) {
    double d2 = dx[0] * dx[0] + dx[1] * dx[1];
    d2 = d2 + dx[2] * dx[2];
    double s = ri + rj;
    return d2 < s * s;
}

/* ------------------------------------------------------- contact search */
typedef struct {
    uint32_t j;   /* partner index, or ORC_FACE_ID + face */
    int16_t img;  /* index into the image table */
} orc_hit;

typedef struct {
    double lo[3], cell[3];
    int nc[3];
    int *start, *cnt, *item;
} orc_grid;

static int orc_cell_coord(const orc_grid *g, double p, int a) {
    double f = floor((p - g->lo[a]) / g->cell[a]);
    if (!(f >= 0.0)) return 0;   /* also catches NaN */
    if (f >= g->nc[a]) return g->nc[a] - 1;
    return (int)f;
}

/* Plain uniform grid over the box; every cell is at least as wide as the
 * largest contact distance 2 r_max along each axis, so the 27 cells around a
 * point hold every sphere that can touch a sphere centred there.  Positions
 * outside the box fall into the border cells, which keeps that property. */
static void orc_grid_build(orc_grid *g, const orc_params *P, long n, const double *x, const double *r) {
    double rmax = 0.0;
    for (long i = 0; i < n; ++i) if (r[i] > rmax) rmax = r[i];
    double range = 2.0 * rmax;
    for (int a = 0; a < 3; ++a) {
        double L = P->hi[a] - P->lo[a];
        int c = (int)floor(L / (range * 1.000001));
        g->nc[a] = c < 1 ? 1 : c;
        g->lo[a] = P->lo[a];
        g->cell[a] = L / g->nc[a];
    }
    long nc = (long)g->nc[0] * g->nc[1] * g->nc[2];
    g->start = (int *)calloc(nc + 1, sizeof(int));
    g->cnt = (int *)calloc(nc, sizeof(int));
    g->item = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int *cid = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (long i = 0; i < n; ++i) {
        int c0 = orc_cell_coord(g, x[3 * i], 0), c1 = orc_cell_coord(g, x[3 * i + 1], 1);
        int c2 = orc_cell_coord(g, x[3 * i + 2], 2);
        cid[i] = (c2 * g->nc[1] + c1) * g->nc[0] + c0;
        g->cnt[cid[i]]++;
    }
    for (long c = 0; c < nc; ++c) g->start[c + 1] = g->start[c] + g->cnt[c];
    int *fill = (int *)calloc(nc, sizeof(int));
    for (long i = 0; i < n; ++i) g->item[g->start[cid[i]] + fill[cid[i]]++] = (int)i;
    free(fill);
    free(cid);
}

static void orc_grid_free(orc_grid *g) {
    free(g->start); free(g->cnt); free(g->item);
}

static int hit_cmp(const void *a, const void *b) {
    uint32_t x = ((const orc_hit *)a)->j, y = ((const orc_hit *)b)->j;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Contacts of particle i, sorted by partner id (faces last).  mode 0: brute
 * force over all pairs and images; mode 1: cell list.  Returns the count,
 * or -1 if `cap` is too small. */
static int orc_find(const orc_params *P, long n, const double *x, const double *r, long i,
                    int mode, const orc_grid *g, const orc_image *im, int nim, orc_hit *hits,
                    int cap) {
    int m = 0;
    const double *xi = x + 3 * i;
    for (int s = 0; s < nim; ++s) {
        if (mode == 0) {
            for (long j = 0; j < n; ++j) {
                if (j == i) continue;
                double dx[3];
                for (int a = 0; a < 3; ++a) dx[a] = (x[3 * j + a] - xi[a]) + im[s].S[a];
                if (orc_touch(dx, r[i], r[j])) {
                    if (m >= cap) return -1;
                    hits[m].j = (uint32_t)j; hits[m].img = (int16_t)s; ++m;
                }
            }
        } else {
            /* partners j whose image x_j + S lies near x_i: look near x_i - S */
            double p[3];
            int skip = 0, shifted = im[s].k[0] || im[s].k[1] || im[s].k[2];
            for (int a = 0; a < 3; ++a) {
                p[a] = xi[a] - im[s].S[a];
                if (shifted && (p[a] < g->lo[a] - g->cell[a] || p[a] > P->hi[a] + g->cell[a])) skip = 1;
            }
            if (skip) continue;
            int c[3];
            for (int a = 0; a < 3; ++a) c[a] = orc_cell_coord(g, p[a], a);
            for (int oz = -1; oz <= 1; ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int ox = -1; ox <= 1; ++ox) {
                        int q0 = c[0] + ox, q1 = c[1] + oy, q2 = c[2] + oz;
                        if (q0 < 0 || q1 < 0 || q2 < 0 || q0 >= g->nc[0] || q1 >= g->nc[1] || q2 >= g->nc[2])
                            continue;
                        int cid = (q2 * g->nc[1] + q1) * g->nc[0] + q0;
                        for (int k = g->start[cid]; k < g->start[cid + 1]; ++k) {
                            long j = g->item[k];
                            if (j == i) continue;
                            double dx[3];
                            for (int a = 0; a < 3; ++a) dx[a] = (x[3 * j + a] - xi[a]) + im[s].S[a];
                            if (orc_touch(dx, r[i], r[j])) {
                                if (m >= cap) return -1;
                                hits[m].j = (uint32_t)j; hits[m].img = (int16_t)s; ++m;
                            }
                        }
                    }
        }
    }
    qsort(hits, m, sizeof(orc_hit), hit_cmp);
    /* box faces last, in face order: distance from the face < r_i */
    for (int f = 0; f < 6; ++f) {
        if (!(P->walls & (1u << f))) continue;
        int a = f >> 1;
        double dist = (f & 1) ? P->hi[a] - xi[a] : xi[a] - P->lo[a];
        if (dist < r[i]) {
            if (m >= cap) return -1;
            hits[m].j = ORC_FACE_ID + (uint32_t)f; hits[m].img = 0; ++m;
        }
    }
    /* then the extra walls, in order */
    for (int k = 0; k < P->n_extra; ++k) {
        if (orc_wall_touch(&P->extra[k], xi, r[i])) {
            if (m >= cap) return -1;
            hits[m].j = ORC_FACE_ID + 6u + (uint32_t)k; hits[m].img = 0; ++m;
        }
    }
    return m;
}

/* Public: the contact set as ordered pairs (i, j) sorted by (i, j); j is a
 * particle index or ORC_FACE_ID + face.  Returns the number of contacts or
 * -1 when cap is too small, -2 when a pair touches through two images. */
long orc_contacts(const orc_params *P, long n, const double *x, const double *r, int mode,
                  long cap, uint32_t *out_i, uint32_t *out_j) {
    orc_image im[75];
    int nim = orc_images(P, P->time, im);
    orc_grid g;
    memset(&g, 0, sizeof(g));
    if (mode == 1) orc_grid_build(&g, P, n, x, r);
    orc_hit hits[512];
    long m = 0;
    for (long i = 0; i < n; ++i) {
        int c = orc_find(P, n, x, r, i, mode, &g, im, nim, hits, 512);
        if (c < 0) { m = -1; break; }
        for (int k = 1; k < c; ++k)
            if (hits[k].j == hits[k - 1].j) { m = -2; goto done; }
        for (int k = 0; k < c; ++k) {
            if (m < cap) { out_i[m] = (uint32_t)i; out_j[m] = hits[k].j; }
            ++m;
        }
    }
done:
    if (mode == 1) orc_grid_free(&g);
    if (m > cap) return -1;
    return m;
}

/* ---------------------------------------------------------- one pair */
/* Public: the force law for one contact, for unit checks.  Geometry from
 * positions: partner j (face < 0), box face `face` (0..5) or extra wall
 * face - 6.  */
void orc_pair(const orc_params *P, const double *xi, const double *vi, const double *wi, double ri,
              int mi, const double *xj, const double *vj, const double *wj, double rj, int mj,
              int face, const double *dt_old, double *F, double *T, double *dt_new, double *dn_out,
              int *capped) {
    double n[3], dn, v[3], rw[3], rs, ms;
    double massi = orc_mass(P->density[mi], ri);
    if (face < 0) {
        double dx[3];
        for (int a = 0; a < 3; ++a) dx[a] = xj[a] - xi[a];
        double d2 = dx[0] * dx[0] + dx[1] * dx[1];
        d2 = d2 + dx[2] * dx[2];
        double d = sqrt(d2);
        for (int a = 0; a < 3; ++a) n[a] = dx[a] / d;
        dn = (ri + rj) - d;
        for (int a = 0; a < 3; ++a) {
            v[a] = vi[a] - vj[a];
            rw[a] = ri * wi[a] + rj * wj[a];
        }
        rs = ri * rj / (ri + rj);
        double massj = orc_mass(P->density[mj], rj);
        ms = massi * massj / (massi + massj);
    } else {
        if (face < 6) {
            int a0 = face >> 1;
            double dist = (face & 1) ? P->hi[a0] - xi[a0] : xi[a0] - P->lo[a0];
            for (int a = 0; a < 3; ++a) n[a] = 0.0;
            n[a0] = (face & 1) ? 1.0 : -1.0;
            dn = ri - dist;
        } else {
            orc_wall_normal(&P->extra[face - 6], xi, ri, n, &dn);
        }
        for (int a = 0; a < 3; ++a) {
            v[a] = vi[a];
            rw[a] = ri * wi[a];
        }
        rs = ri;
        ms = massi;
        mj = mi;
    }
    orc_pair_out o;
    orc_contact_law(P, mi, mj, ri, rs, ms, n, dn, v, rw, dt_old, &o);
    for (int a = 0; a < 3; ++a) { F[a] = o.F[a]; T[a] = o.T[a]; dt_new[a] = o.dt[a]; }
    *dn_out = o.dn;
    *capped = o.capped;
}

/* ---------------------------------------------------------- one step */
/* history lookup: (hi, hj) sorted by (i, j) */
static long hist_find(long m, const uint32_t *hi, const uint32_t *hj, uint32_t i, uint32_t j) {
    long a = 0, b = m;
    while (a < b) {
        long c = (a + b) / 2;
        if (hi[c] < i || (hi[c] == i && hj[c] < j)) a = c + 1;
        else b = c;
    }
    if (a < m && hi[a] == i && hj[a] == j) return a;
    return -1;
}

/*
 * Public: advance the state one step in place.
 *   x, v, w  (n,3) particle state; r radii; mat material index per particle
 *   history in: m_in contacts (hi, hj, hdt[3*m]) sorted by (i, j)
 *   history out: up to cap_out contacts; *m_out receives the count
 *   F_out, T_out (n,3) optional: per-particle totals used in this step
 *   cF, cT (cap_out,3) optional: per-contact force and torque on i
 *   cQ (cap_out,5) optional: per contact |F_t| before the cap, mu |F_n|,
 *     the rounding scale of the sliding test and that of Eq. (1), and k_t
 *     (orc_pair_out)
 *   mode 0 brute force, 1 cell list; nthreads 0 = OpenMP default
 * Returns 0, -1 (history capacity), -2 (a per-particle contact list over
 * 64) or -3 (a pair touching through two images).
 */
int orc_step(const orc_params *P, long n, double *x, double *v, double *w, const double *r,
             const uint16_t *mat, long m_in, const uint32_t *hi_, const uint32_t *hj_,
             const double *hdt, long cap_out, long *m_out, uint32_t *ho_i, uint32_t *ho_j,
             double *ho_dt, double *F_out, double *T_out, double *cF, double *cT, double *cQ,
             int mode, int nthreads) {
    orc_image im[75];
    int nim = orc_images(P, P->time, im);
    orc_grid g;
    memset(&g, 0, sizeof(g));
    if (mode == 1) orc_grid_build(&g, P, n, x, r);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int *cnt = (int *)calloc(n + 1, sizeof(int));
    orc_hit *allhits = (orc_hit *)malloc(sizeof(orc_hit) * 64 * (size_t)(n > 0 ? n : 1));
    int err = 0;
    /* pass 1: contact lists */
#pragma omp parallel for schedule(dynamic, 256) if (n > 4096)
    for (long i = 0; i < n; ++i) {
        orc_hit hits[512];
        int c = orc_find(P, n, x, r, i, mode, &g, im, nim, hits, 512);
        if (c < 0 || c > 64) {
#pragma omp atomic write
            err = -2;
            c = 0;
        }
        for (int k = 1; k < c; ++k)
            if (hits[k].j == hits[k - 1].j) {
#pragma omp atomic write
                err = -3;
            }
        cnt[i] = c;
        memcpy(allhits + 64 * i, hits, sizeof(orc_hit) * c);
    }
    if (mode == 1) orc_grid_free(&g);
    if (err) { free(cnt); free(allhits); return err; }
    long *off = (long *)malloc(sizeof(long) * (n + 1));
    off[0] = 0;
    for (long i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i];
    long mtot = off[n];
    *m_out = mtot;
    if (mtot > cap_out) { free(cnt); free(allhits); free(off); return -1; }

    double *Fi = (double *)calloc(3 * (size_t)(n > 0 ? n : 1), sizeof(double));
    double *Ti = (double *)calloc(3 * (size_t)(n > 0 ? n : 1), sizeof(double));
    /* pass 2: forces, in ascending partner id, faces last */
#pragma omp parallel for schedule(dynamic, 256) if (n > 4096)
    for (long i = 0; i < n; ++i) {
        int mi = mat ? mat[i] : 0;
        double massi = orc_mass(P->density[mi], r[i]);
        double Fs[3] = {0, 0, 0}, Ts[3] = {0, 0, 0};
        for (int k = 0; k < cnt[i]; ++k) {
            orc_hit h = allhits[64 * i + k];
            double n_[3], dn, vrel[3], rw[3], rs, ms;
            int mj;
            if (h.j < ORC_FACE_ID) {
                long j = h.j;
                mj = mat ? mat[j] : 0;
                double dx[3];
                for (int a = 0; a < 3; ++a) dx[a] = (x[3 * j + a] - x[3 * i + a]) + im[h.img].S[a];
                double d2 = dx[0] * dx[0] + dx[1] * dx[1];
                d2 = d2 + dx[2] * dx[2];
                double d = sqrt(d2);
                for (int a = 0; a < 3; ++a) n_[a] = dx[a] / d;
                dn = (r[i] + r[j]) - d;
                for (int a = 0; a < 3; ++a) {
                    vrel[a] = v[3 * i + a] - v[3 * j + a];
                    rw[a] = r[i] * w[3 * i + a] + r[j] * w[3 * j + a];
                }
                vrel[0] = vrel[0] - im[h.img].dvx;
                rs = r[i] * r[j] / (r[i] + r[j]);
                double massj = orc_mass(P->density[mj], r[j]);
                ms = massi * massj / (massi + massj);
            } else {
                int f = (int)(h.j - ORC_FACE_ID), a0 = f >> 1;
                if (f < 6) {
                    double dist = (f & 1) ? P->hi[a0] - x[3 * i + a0] : x[3 * i + a0] - P->lo[a0];
                    n_[0] = n_[1] = n_[2] = 0.0;
                    n_[a0] = (f & 1) ? 1.0 : -1.0;
                    dn = r[i] - dist;
                } else {
                    orc_wall_normal(&P->extra[f - 6], x + 3 * i, r[i], n_, &dn);
                }
                for (int a = 0; a < 3; ++a) {
                    vrel[a] = v[3 * i + a];
                    rw[a] = r[i] * w[3 * i + a];
                }
                rs = r[i];
                ms = massi;
                mj = mi;
            }
            double dto[3] = {0, 0, 0};
            long hidx = hist_find(m_in, hi_, hj_, (uint32_t)i, h.j);
            if (hidx >= 0) for (int a = 0; a < 3; ++a) dto[a] = hdt[3 * hidx + a];
            orc_pair_out o;
            orc_contact_law(P, mi, mj, r[i], rs, ms, n_, dn, vrel, rw, dto, &o);
            long q = off[i] + k;
            ho_i[q] = (uint32_t)i;
            ho_j[q] = h.j;
            for (int a = 0; a < 3; ++a) {
                ho_dt[3 * q + a] = o.dt[a];
                Fs[a] += o.F[a];
                Ts[a] += o.T[a];
                if (cF) cF[3 * q + a] = o.F[a];
                if (cT) cT[3 * q + a] = o.T[a];
            }
            if (cQ) {
                cQ[5 * q] = o.ft_pre;
                cQ[5 * q + 1] = o.mufn;
                cQ[5 * q + 2] = o.scale;
                cQ[5 * q + 3] = o.fterm;
                cQ[5 * q + 4] = o.kt;
            }
        }
        for (int a = 0; a < 3; ++a) {
            Fi[3 * i + a] = Fs[a] + massi * P->gravity[a];
            Ti[3 * i + a] = Ts[a];
        }
    }
    /* integrate: v += dt F/m; x += dt v; w += dt T/I; then wrap periodic axes */
    double L[3];
    for (int a = 0; a < 3; ++a) L[a] = P->hi[a] - P->lo[a];
    double Dn = orc_le_offset(P, P->time + P->dt);
    double du = P->shear_rate * L[1];
    for (long i = 0; i < n; ++i) {
        int mi = mat ? mat[i] : 0;
        double m = orc_mass(P->density[mi], r[i]);
        double I = orc_inertia(m, r[i]);
        for (int a = 0; a < 3; ++a) {
            v[3 * i + a] += P->dt * Fi[3 * i + a] / m;
            x[3 * i + a] += P->dt * v[3 * i + a];
            w[3 * i + a] += P->dt * Ti[3 * i + a] / I;
        }
        if (P->periodic & 2u) {
            if (x[3 * i + 1] >= P->hi[1]) {
                x[3 * i + 1] -= L[1];
                x[3 * i + 0] -= Dn;
                v[3 * i + 0] -= du;
            } else if (x[3 * i + 1] < P->lo[1]) {
                x[3 * i + 1] += L[1];
                x[3 * i + 0] += Dn;
                v[3 * i + 0] += du;
            }
        }
        for (int a = 0; a < 3; a += 2) {
            if (!(P->periodic & (1u << a))) continue;
            for (int k = 0; k < 4 && x[3 * i + a] >= P->hi[a]; ++k) x[3 * i + a] -= L[a];
            for (int k = 0; k < 4 && x[3 * i + a] < P->lo[a]; ++k) x[3 * i + a] += L[a];
        }
        if (F_out) for (int a = 0; a < 3; ++a) F_out[3 * i + a] = Fi[3 * i + a];
        if (T_out) for (int a = 0; a < 3; ++a) T_out[3 * i + a] = Ti[3 * i + a];
    }
    free(Fi); free(Ti); free(cnt); free(allhits); free(off);
    return 0;
}
