/*
 * oracle.c -- plain FP64 CPU reference of one agitated-soil particle step.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Built with -O2 -ffp-contract=off.
 * Written for readability against the paper, not for speed: every step below
 * names the passage of Servin, Berglund & Nystedt (arXiv 2011.00459) it
 * follows, and the readings taken where the paper is silent or garbled.
 *
 * Conventions (readings taken where the paper is silent, ambiguous or garbled):
 *  - Contact normal n points from body 1 to body 2.  A pair is ordered by id
 *    (body 1 = lower id); for a boundary contact body 1 is the kinematic shape
 *    and body 2 the particle.
 *  - Overlap delta > 0 when penetrating.  The constraint function of Eq.
 *    signCoul1 is read as g_n = -delta^(5/4) (negative when penetrating), so a
 *    positive lambda_n pushes body 2 along +n.
 *  - The Hertz mapping (epsilon_n read as 5/(4 k_n)) is applied to the row
 *    divided by ||G_n|| = (5/4) delta^(1/4): g' = -(4/5) delta,
 *    eps' = 4 / (5 k_n sqrt(delta)), lambda' = impulse along n.  Scaling a row
 *    does not change the MCP solution; the cohesion bound becomes c_p A_p.
 *  - SPOOK (section "Contacting rigid multibodies") as printed:
 *    Upsilon = 1/(1+4 tau/dt), Sigma = (4/dt^2) eps Upsilon,
 *    q = -(4/dt) Upsilon g + Upsilon G v_n.  lambda is an impulse.
 *  - Cohesion: a contact exists while delta > -delta_c with delta_c = kappa_c
 *    (r1 + r2) (pairs) or 2 kappa_c r (walls) when c_p > 0, else delta > 0;
 *    lambda_n >= -c_p pi min(r1,r2)^2 dt.
 *  - Friction disk ||lambda_t|| <= mu |lambda_n| (Eq. signCoul2 literally).
 *  - Contact point at the middle of the overlap: lever arms l_i = r_i - delta/2.
 *  - tau_n = 2 dt for every contact; the impact stage runs only when v_imp > 0.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
/* ------------------------------------------------------------------ */
static double dot3(const double* a, const double* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Rotation matrix of a unit quaternion (w, x, y, z); R[i][j] row-major. */
static void quat_matrix(const double* q, double R[3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

/* splitmix64 (Steele, Lea & Flood 2014; Vigna's published constants). */
static uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double particle_mass(const orc_params* P, const double* rho, int64_t i, const double* r)
{
    double dens = rho ? rho[i] : P->m.rho;
    return dens * (4.0 / 3.0) * PI * r[i] * r[i] * r[i];
}

/* ------------------------------------------------------------------ */
/* Contact detection ("do collision detection", Algorithm 1)            */
/* ------------------------------------------------------------------ */

/* Cohesive range added to the contact distance (reading of "cohesion is
 * active when the overlap is smaller than delta_c = 0.025 d"). */
static double pair_range(const orc_params* P, double ri, double rj)
{
    return P->m.c_p > 0.0 ? P->m.kappa_c * (ri + rj) : 0.0;
}
static double wall_range(const orc_params* P, double r)
{
    return P->m.c_p > 0.0 ? P->m.kappa_c * (2.0 * r) : 0.0;
}

/* Pinned pair predicate: evaluated exactly in this order, no contraction. */
static int pair_touch(const orc_params* P, const double* xi, double ri, const double* xj, double rj, double* d2out)
{
    double dx = xj[0] - xi[0];
    double dy = xj[1] - xi[1];
    double dz = xj[2] - xi[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double R = (ri + rj) + pair_range(P, ri, rj);
    *d2out = d2;
    return d2 < R * R;
}

/* World-frame plane of a PLANE shape: normal nw and offset dw. */
static void plane_world(const orc_shape* s, const orc_body* b, double nw[3], double* dw)
{
    double R[3][3];
    quat_matrix(b->quat, R);
    for (int k = 0; k < 3; ++k) nw[k] = (R[k][0] * s->n[0] + R[k][1] * s->n[1]) + R[k][2] * s->n[2];
    *dw = s->d + ((nw[0] * b->pos[0] + nw[1] * b->pos[1]) + nw[2] * b->pos[2]);
}

/* Boundary geometry of one sphere against one shape.  Returns 1 if in contact
 * and fills delta, normal (shape -> particle). */
static int shape_touch(const orc_params* P, const orc_shape* s, const orc_body* bodies,
                       const double* x, double r, double* delta, double nrm[3])
{
    double Rr = r + wall_range(P, r);
    if (s->type == ORC_PLANE) {
        double nw[3], dw;
        plane_world(s, &bodies[s->body], nw, &dw);
        double sd = ((nw[0] * x[0] + nw[1] * x[1]) + nw[2] * x[2]) - dw;
        if (!(sd < 0.0 || sd * sd < Rr * Rr)) return 0;
        *delta = r - sd;
        nrm[0] = nw[0]; nrm[1] = nw[1]; nrm[2] = nw[2];
        return 1;
    }
    if (s->type == ORC_BOX) {
        const orc_body* b = &bodies[s->body];
        double R[3][3];
        quat_matrix(b->quat, R);
        double c[3];
        for (int k = 0; k < 3; ++k) c[k] = b->pos[k] + ((R[k][0] * s->off[0] + R[k][1] * s->off[1]) + R[k][2] * s->off[2]);
        double dx = x[0] - c[0], dy = x[1] - c[1], dz = x[2] - c[2];
        double l[3];
        for (int k = 0; k < 3; ++k) l[k] = (R[0][k] * dx + R[1][k] * dy) + R[2][k] * dz;
        int inside = 1;
        double q[3];
        for (int k = 0; k < 3; ++k) {
            q[k] = l[k];
            if (q[k] > s->half[k]) { q[k] = s->half[k]; inside = 0; }
            if (q[k] < -s->half[k]) { q[k] = -s->half[k]; inside = 0; }
        }
        if (inside) {
            /* centre inside the box: least-penetration face, ties to the lower
             * axis, + side when the coordinate is >= 0 */
            int kbest = 0;
            double pbest = s->half[0] - fabs(l[0]);
            for (int k = 1; k < 3; ++k) {
                double p = s->half[k] - fabs(l[k]);
                if (p < pbest) { pbest = p; kbest = k; }
            }
            double sg = l[kbest] >= 0.0 ? 1.0 : -1.0;
            for (int k = 0; k < 3; ++k) nrm[k] = sg * R[k][kbest];
            *delta = r + pbest;
            return 1;
        }
        double e0 = l[0] - q[0], e1 = l[1] - q[1], e2 = l[2] - q[2];
        double d2 = (e0 * e0 + e1 * e1) + e2 * e2;
        if (!(d2 < Rr * Rr)) return 0;
        double dist = sqrt(d2);
        double nl[3] = {e0 / dist, e1 / dist, e2 / dist};
        for (int k = 0; k < 3; ++k) nrm[k] = (R[k][0] * nl[0] + R[k][1] * nl[1]) + R[k][2] * nl[2];
        *delta = r - dist;
        return 1;
    }
    if (s->type == ORC_HFIELD) {
        /* Eq. surface: heights interpolated linearly between grid points,
         * read as bilinear; local tangent-plane distance. */
        double inv = 1.0 / s->l0;
        double fx = (x[0] - s->ox) * inv;
        double fy = (x[1] - s->oy) * inv;
        double fi = floor(fx), fj = floor(fy);
        if (fi < 0.0) fi = 0.0;
        if (fi > (double)(s->nx - 2)) fi = (double)(s->nx - 2);
        if (fj < 0.0) fj = 0.0;
        if (fj > (double)(s->ny - 2)) fj = (double)(s->ny - 2);
        int i = (int)fi, j = (int)fj;
        double t = fx - fi, u = fy - fj;
        double h00 = s->h[j * s->nx + i], h10 = s->h[j * s->nx + i + 1];
        double h01 = s->h[(j + 1) * s->nx + i], h11 = s->h[(j + 1) * s->nx + i + 1];
        double h = (h00 * (1.0 - t) + h10 * t) * (1.0 - u) + (h01 * (1.0 - t) + h11 * t) * u;
        double hx = ((h10 - h00) * (1.0 - u) + (h11 - h01) * u) * inv;
        double hy = ((h01 - h00) * (1.0 - t) + (h11 - h10) * t) * inv;
        double dz = x[2] - h;
        double m2 = (1.0 + hx * hx) + hy * hy;
        if (!(dz < 0.0 || dz * dz < (Rr * Rr) * m2)) return 0;
        double nz = 1.0 / sqrt(m2);
        nrm[0] = -hx * nz; nrm[1] = -hy * nz; nrm[2] = nz;
        *delta = r - dz * nz;
        return 1;
    }
    return 0;
}

typedef struct {
    uint64_t key;
    int64_t a, b;   /* particle indices; a = -1 for a boundary contact */
    int32_t shape;  /* shape index for a boundary contact */
} raw_contact;

static int cmp_raw(const void* p, const void* q)
{
    uint64_t a = ((const raw_contact*)p)->key, b = ((const raw_contact*)q)->key;
    return a < b ? -1 : (a > b ? 1 : 0);
}

typedef struct { int64_t cell; int64_t idx; } cell_entry;
static int cmp_cell(const void* p, const void* q)
{
    const cell_entry* a = (const cell_entry*)p;
    const cell_entry* b = (const cell_entry*)q;
    if (a->cell != b->cell) return a->cell < b->cell ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

/* Append a pair (i, j) if it touches; keys ordered by id. */
static int add_pair(const orc_params* P, const int64_t* id, const double* x, const double* r,
                    int64_t i, int64_t j, raw_contact** buf, int64_t* nc, int64_t* capb)
{
    int64_t lo = id[i] < id[j] ? i : j, hi = id[i] < id[j] ? j : i;
    double d2;
    if (!pair_touch(P, &x[3 * lo], r[lo], &x[3 * hi], r[hi], &d2)) return 0;
    if (*nc == *capb) {
        *capb = *capb ? 2 * *capb : 1024;
        *buf = (raw_contact*)realloc(*buf, (size_t)*capb * sizeof(raw_contact));
    }
    raw_contact* c = &(*buf)[(*nc)++];
    c->key = ((uint64_t)id[lo] << 32) | (uint64_t)(uint32_t)id[hi];
    c->a = lo; c->b = hi; c->shape = -1;
    return 1;
}

/* Detect all contacts, return them sorted by key (caller frees *out). */
static int64_t detect_all(const orc_params* P, int64_t n, const int64_t* id, const double* x, const double* r,
                          int32_t nb, const orc_body* bodies, int32_t ns, const orc_shape* shapes,
                          raw_contact** out)
{
    raw_contact* buf = NULL;
    int64_t nc = 0, capb = 0;
    (void)nb;
    if (P->detect == ORC_BRUTE || n < 2) {
        /* the plain definition: every unordered pair */
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) add_pair(P, id, x, r, i, j, &buf, &nc, &capb);
    } else {
        /* uniform cell list with cell size = the largest contact distance */
        double rmax = 0.0, lo[3] = {1e300, 1e300, 1e300};
        for (int64_t i = 0; i < n; ++i) {
            if (r[i] > rmax) rmax = r[i];
            for (int k = 0; k < 3; ++k) if (x[3 * i + k] < lo[k]) lo[k] = x[3 * i + k];
        }
        double h = 2.0 * rmax + pair_range(P, rmax, rmax);
        h *= 1.0000001; /* margin: any touching pair lies in adjacent cells */
        int64_t dim[3] = {1, 1, 1};
        int64_t* cx = (int64_t*)malloc((size_t)n * 3 * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) {
                cx[3 * i + k] = (int64_t)floor((x[3 * i + k] - lo[k]) / h);
                if (cx[3 * i + k] + 1 > dim[k]) dim[k] = cx[3 * i + k] + 1;
            }
        cell_entry* ce = (cell_entry*)malloc((size_t)n * sizeof(cell_entry));
        for (int64_t i = 0; i < n; ++i) {
            ce[i].cell = (cx[3 * i + 2] * dim[1] + cx[3 * i + 1]) * dim[0] + cx[3 * i];
            ce[i].idx = i;
        }
        qsort(ce, (size_t)n, sizeof(cell_entry), cmp_cell);
        for (int64_t s = 0; s < n; ++s) {
            int64_t i = ce[s].idx;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int64_t c0 = cx[3 * i] + dx, c1 = cx[3 * i + 1] + dy, c2 = cx[3 * i + 2] + dz;
                        if (c0 < 0 || c1 < 0 || c2 < 0 || c0 >= dim[0] || c1 >= dim[1] || c2 >= dim[2]) continue;
                        int64_t cell = (c2 * dim[1] + c1) * dim[0] + c0;
                        /* binary search for the first entry of that cell */
                        int64_t a = 0, b = n;
                        while (a < b) {
                            int64_t m = (a + b) / 2;
                            if (ce[m].cell < cell) a = m + 1; else b = m;
                        }
                        for (int64_t t = a; t < n && ce[t].cell == cell; ++t) {
                            int64_t j = ce[t].idx;
                            if (id[j] > id[i]) add_pair(P, id, x, r, i, j, &buf, &nc, &capb);
                        }
                    }
        }
        free(ce);
        free(cx);
    }
    for (int64_t i = 0; i < n; ++i)
        for (int32_t s = 0; s < ns; ++s) {
            double dl, nr[3];
            if (!shape_touch(P, &shapes[s], bodies, &x[3 * i], r[i], &dl, nr)) continue;
            if (nc == capb) {
                capb = capb ? 2 * capb : 1024;
                buf = (raw_contact*)realloc(buf, (size_t)capb * sizeof(raw_contact));
            }
            raw_contact* c = &buf[nc++];
            c->key = ((uint64_t)id[i] << 32) | 0x80000000ull | (uint64_t)(uint32_t)s;
            c->a = -1; c->b = i; c->shape = s;
        }
    if (nc > 1) qsort(buf, (size_t)nc, sizeof(raw_contact), cmp_raw);
    *out = buf;
    return nc;
}

/* ------------------------------------------------------------------ */
/* Contact rows                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t key;
    int64_t a, b;        /* body 1 (particle index or -1), body 2 (particle index) */
    int32_t shape, body; /* kinematic side (boundary contacts) */
    double n[3];         /* body 1 -> body 2 */
    double delta;
    double l1, l2;       /* lever arms from the centres to the contact point */
    double p[3];         /* contact point */
    double vk[3];        /* kinematic velocity at p (boundary contacts) */
    double Wn, Wt, Dn, Dt, Sig, q, lo, mu;
    double qg;           /* the overlap part of q (q = qg + Upsilon G_n v) */
    double Wr, rlim;     /* rolling rows: 1/I_1 + 1/I_2, and r mu_r (0: no rolling rows) */
    double wk[3];        /* angular velocity of the kinematic side (boundary contacts) */
    double ln, lt[3];    /* impulses */
    double lr[3];        /* rolling (torque) impulse, on body 2; -lr on body 1 */
    int persistent;
    int colour;
} row;

typedef struct {
    double* im;   /* 1/m per particle */
    double* iI;   /* 1/I per particle */
} inv_mass;

/* Relative velocity at the contact point, body 2 minus body 1. */
static void rel_vel(const row* c, const double* v, const double* w, double u[3])
{
    double n[3] = {c->n[0], c->n[1], c->n[2]};
    double u2[3], u1[3], t[3], arm[3];
    /* body 2: v2 + w2 x (p - x2), p - x2 = -l2 n */
    for (int k = 0; k < 3; ++k) arm[k] = -c->l2 * n[k];
    cross3(&w[3 * c->b], arm, t);
    for (int k = 0; k < 3; ++k) u2[k] = v[3 * c->b + k] + t[k];
    if (c->a >= 0) {
        for (int k = 0; k < 3; ++k) arm[k] = c->l1 * n[k];
        cross3(&w[3 * c->a], arm, t);
        for (int k = 0; k < 3; ++k) u1[k] = v[3 * c->a + k] + t[k];
    } else {
        for (int k = 0; k < 3; ++k) u1[k] = c->vk[k];
    }
    for (int k = 0; k < 3; ++k) u[k] = u2[k] - u1[k];
}

/* Apply impulse J (vector, on body 2; -J on body 1) at the contact point. */
static void apply_impulse(const row* c, const inv_mass* M, double* v, double* w, const double J[3])
{
    double arm[3], t[3];
    int64_t b = c->b;
    for (int k = 0; k < 3; ++k) v[3 * b + k] += M->im[b] * J[k];
    for (int k = 0; k < 3; ++k) arm[k] = -c->l2 * c->n[k];
    cross3(arm, J, t);
    for (int k = 0; k < 3; ++k) w[3 * b + k] += M->iI[b] * t[k];
    if (c->a >= 0) {
        int64_t a = c->a;
        for (int k = 0; k < 3; ++k) v[3 * a + k] -= M->im[a] * J[k];
        for (int k = 0; k < 3; ++k) arm[k] = c->l1 * c->n[k];
        cross3(arm, J, t);
        for (int k = 0; k < 3; ++k) w[3 * a + k] -= M->iI[a] * t[k];
    }
}

/* Geometry and SPOOK/Hertz scalars of every contact (v = start-of-step). */
static void build_rows(const orc_params* P, const int64_t* id, const double* r, const inv_mass* M,
                       const double* x, const double* v, const double* w,
                       const orc_body* bodies, const orc_shape* shapes,
                       const raw_contact* rc, int64_t nc, row* rows)
{
    const orc_material* m = &P->m;
    double dt = P->dt;
    double tau = m->tau_n > 0.0 ? m->tau_n : 2.0 * dt;
    double Ups = 1.0 / (1.0 + 4.0 * tau / dt);
    double a_coef = (4.0 / dt) * Ups;
    double b_coef = Ups;
    double Estar = m->E / (2.0 * (1.0 - m->nu * m->nu)); /* same material both sides */
    (void)id;
    for (int64_t c = 0; c < nc; ++c) {
        row* R = &rows[c];
        memset(R, 0, sizeof(row));
        R->key = rc[c].key;
        R->a = rc[c].a;
        R->b = rc[c].b;
        R->shape = rc[c].shape;
        R->body = -1;
        double dstar, dref, rmin;
        int64_t b = R->b;
        if (R->a >= 0) {
            int64_t a = R->a;
            double e[3] = {x[3 * b] - x[3 * a], x[3 * b + 1] - x[3 * a + 1], x[3 * b + 2] - x[3 * a + 2]};
            double d = sqrt(dot3(e, e));
            if (d > 0.0) { for (int k = 0; k < 3; ++k) R->n[k] = e[k] / d; }
            else { R->n[0] = 0.0; R->n[1] = 0.0; R->n[2] = 1.0; }
            R->delta = (r[a] + r[b]) - d;
            R->l1 = r[a] - 0.5 * R->delta;
            R->l2 = r[b] - 0.5 * R->delta;
            double da = 2.0 * r[a], db = 2.0 * r[b];
            dstar = 1.0 / (1.0 / da + 1.0 / db);
            dref = r[a] + r[b];
            rmin = r[a] < r[b] ? r[a] : r[b];
        } else {
            const orc_shape* s = &shapes[R->shape];
            shape_touch(P, s, bodies, &x[3 * b], r[b], &R->delta, R->n);
            R->body = s->body;
            R->l1 = 0.0;
            R->l2 = r[b] - 0.5 * R->delta;
            dstar = 2.0 * r[b];
            dref = 2.0 * r[b];
            rmin = r[b];
        }
        for (int k = 0; k < 3; ++k) R->p[k] = x[3 * b + k] - R->l2 * R->n[k];
        if (R->a < 0) {
            const orc_body* B = &bodies[R->body];
            double arm[3] = {R->p[0] - B->pos[0], R->p[1] - B->pos[1], R->p[2] - B->pos[2]};
            double t[3];
            cross3(B->angvel, arm, t);
            for (int k = 0; k < 3; ++k) R->vk[k] = B->linvel[k] + t[k];
        }
        /* Hertz stiffness k_n = E* sqrt(d*) / 3 and the scaled row */
        double kn = Estar * sqrt(dstar) / 3.0;
        double de = R->delta > m->kappa_min * dref ? R->delta : m->kappa_min * dref;
        double eps = 4.0 / (5.0 * kn * sqrt(de));
        double gq = -0.8 * R->delta;
        R->Sig = (4.0 / (dt * dt)) * eps * Ups;
        double u[3];
        rel_vel(R, v, w, u);
        double un = dot3(R->n, u);
        R->qg = -a_coef * gq;
        R->q = R->qg + b_coef * un;
        double ima = R->a >= 0 ? M->im[R->a] : 0.0, imb = M->im[b];
        double iIa = R->a >= 0 ? M->iI[R->a] : 0.0, iIb = M->iI[b];
        R->Wn = ima + imb;
        R->Wt = ima + imb + R->l1 * R->l1 * iIa + R->l2 * R->l2 * iIb;
        R->Dn = R->Wn + R->Sig;
        R->Dt = R->Wt + m->gamma_t / dt;
        R->lo = -m->c_p * PI * rmin * rmin * dt;
        R->mu = m->mu_t;
        /* rolling resistance (Eq. signCoul3): zero relative angular velocity,
         * the torque impulse bounded by r mu_r |lambda_n|, r the smaller radius */
        R->Wr = iIa + iIb;
        R->rlim = m->mu_r * rmin;
        if (R->a < 0)
            for (int k = 0; k < 3; ++k) R->wk[k] = bodies[R->body].angvel[k];
    }
}

/* Project (ln, lt) onto {ln >= lo, |lt| <= mu |ln|}. */
static void project(const row* R, double* ln, double lt[3])
{
    if (*ln < R->lo) *ln = R->lo;
    double tn = dot3(R->n, lt);
    for (int k = 0; k < 3; ++k) lt[k] -= tn * R->n[k];
    double lim = R->mu * fabs(*ln);
    double m = sqrt(dot3(lt, lt));
    if (m > lim) {
        double s = m > 0.0 ? lim / m : 0.0;
        for (int k = 0; k < 3; ++k) lt[k] *= s;
    }
}

/* Project lr onto the disk {|lr| <= r mu_r |ln|}. */
static void project_r(const row* R, double lr[3])
{
    double lim = R->rlim * fabs(R->ln);
    double m = sqrt(dot3(lr, lr));
    if (m > lim) {
        double s = m > 0.0 ? lim / m : 0.0;
        for (int k = 0; k < 3; ++k) lr[k] *= s;
    }
}

/* Apply the torque impulse L (on body 2; -L on body 1). */
static void apply_torque(const row* R, const inv_mass* M, double* w, const double L[3])
{
    for (int k = 0; k < 3; ++k) w[3 * R->b + k] += M->iI[R->b] * L[k];
    if (R->a >= 0)
        for (int k = 0; k < 3; ++k) w[3 * R->a + k] -= M->iI[R->a] * L[k];
}

/* One projected Gauss-Seidel update of one contact (normal row, then the
 * tangential disk row, then the rolling row when mu_r > 0).  Adds the
 * D-weighted change and value to acc. */
static void pgs_contact(row* R, const inv_mass* M, double* v, double* w, double gamma_dt, double acc[2])
{
    double u[3];
    /* normal row */
    rel_vel(R, v, w, u);
    double un = dot3(R->n, u);
    double ln_new = R->ln - (un + R->Sig * R->ln - R->q) / R->Dn;
    if (ln_new < R->lo) ln_new = R->lo;
    double dn = ln_new - R->ln;
    R->ln = ln_new;
    double J[3] = {dn * R->n[0], dn * R->n[1], dn * R->n[2]};
    apply_impulse(R, M, v, w, J);
    /* tangential row */
    rel_vel(R, v, w, u);
    un = dot3(R->n, u);
    double ut[3] = {u[0] - un * R->n[0], u[1] - un * R->n[1], u[2] - un * R->n[2]};
    double lt[3];
    for (int k = 0; k < 3; ++k) lt[k] = R->lt[k] - (ut[k] + gamma_dt * R->lt[k]) / R->Dt;
    double lim = R->mu * fabs(R->ln);
    double mag = sqrt(dot3(lt, lt));
    if (mag > lim) {
        double s = mag > 0.0 ? lim / mag : 0.0;
        for (int k = 0; k < 3; ++k) lt[k] *= s;
    }
    double dtv[3] = {lt[0] - R->lt[0], lt[1] - R->lt[1], lt[2] - R->lt[2]};
    for (int k = 0; k < 3; ++k) R->lt[k] = lt[k];
    apply_impulse(R, M, v, w, dtv);
    acc[0] += R->Dn * dn * dn + R->Dt * dot3(dtv, dtv);
    acc[1] += R->Dn * R->ln * R->ln + R->Dt * dot3(R->lt, R->lt);
    if (R->rlim > 0.0) {
        /* rolling row: relative angular velocity, body 2 minus body 1 */
        double ur[3];
        for (int k = 0; k < 3; ++k) ur[k] = w[3 * R->b + k] - (R->a >= 0 ? w[3 * R->a + k] : R->wk[k]);
        double lr[3];
        for (int k = 0; k < 3; ++k) lr[k] = R->lr[k] - ur[k] / R->Wr;
        project_r(R, lr);
        double dr[3] = {lr[0] - R->lr[0], lr[1] - R->lr[1], lr[2] - R->lr[2]};
        for (int k = 0; k < 3; ++k) R->lr[k] = lr[k];
        apply_torque(R, M, w, dr);
        acc[0] += R->Wr * dot3(dr, dr);
        acc[1] += R->Wr * dot3(R->lr, R->lr);
    }
}

/* ------------------------------------------------------------------ */
/* Colouring: greedy in decreasing (splitmix64(key), key) order.  This is the */
/* unique result of Jones-Plassmann with that priority.                  */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t h, key; int64_t idx; } prio;
static int cmp_prio_desc(const void* p, const void* q)
{
    const prio* a = (const prio*)p;
    const prio* b = (const prio*)q;
    if (a->h != b->h) return a->h > b->h ? -1 : 1;
    if (a->key != b->key) return a->key > b->key ? -1 : 1;
    return 0;
}

static int colour_contacts(row* rows, int64_t nc, int64_t n)
{
    /* incidence lists of dynamic particles */
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t c = 0; c < nc; ++c) {
        cnt[rows[c].b + 1]++;
        if (rows[c].a >= 0) cnt[rows[c].a + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t* fill = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    memcpy(fill, cnt, (size_t)(n + 1) * sizeof(int64_t));
    int64_t* inc = (int64_t*)malloc((size_t)(cnt[n] > 0 ? cnt[n] : 1) * sizeof(int64_t));
    for (int64_t c = 0; c < nc; ++c) {
        inc[fill[rows[c].b]++] = c;
        if (rows[c].a >= 0) inc[fill[rows[c].a]++] = c;
    }
    prio* order = (prio*)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(prio));
    for (int64_t c = 0; c < nc; ++c) {
        order[c].h = splitmix64(rows[c].key);
        order[c].key = rows[c].key;
        order[c].idx = c;
        rows[c].colour = -1;
    }
    qsort(order, (size_t)nc, sizeof(prio), cmp_prio_desc);
    int maxc = 0;
    for (int64_t t = 0; t < nc; ++t) {
        row* R = &rows[order[t].idx];
        unsigned char used[256];
        memset(used, 0, sizeof(used));
        int64_t parts[2] = {R->b, R->a};
        for (int s = 0; s < 2; ++s) {
            if (parts[s] < 0) continue;
            for (int64_t e = cnt[parts[s]]; e < cnt[parts[s] + 1]; ++e) {
                int col = rows[inc[e]].colour;
                if (col >= 0 && col < 256) used[col] = 1;
            }
        }
        int col = 0;
        while (col < 256 && used[col]) ++col;
        R->colour = col;
        if (col + 1 > maxc) maxc = col + 1;
    }
    free(order);
    free(inc);
    free(fill);
    free(cnt);
    return maxc;
}

/* ------------------------------------------------------------------ */
/* MLP (learned warm start)                                             */
/* ------------------------------------------------------------------ */
static double silu(double z) { return z / (1.0 + exp(-z)); }
static double dsilu(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

/* bfloat16 rounding of a value held in single precision: the upper 16 bits
 * of the IEEE binary32 pattern, rounded to nearest with ties to even (the
 * published bfloat16 conversion; finite inputs only). */
static double to_bf16(double a)
{
    float f = (float)a;
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

/* The network 12 -> 64 -> 64 -> 3 with SiLU.  With net->bf16 the inference
 * takes the precision the learned start is specified in: the scaled inputs,
 * the three weight matrices and both hidden layers are bfloat16 values (the
 * hidden layers first held in single precision), biases and sums in double. */
void orc_mlp_forward(const orc_mlp* net, int64_t B, const double* feat, double* out)
{
    const int q = net->bf16;
    for (int64_t b = 0; b < B; ++b) {
        double x0[12], h1[64], h2[64];
        for (int i = 0; i < 12; ++i) {
            x0[i] = feat[12 * b + i] * net->in_scale[i];
            if (q) x0[i] = to_bf16(x0[i]);
        }
        for (int o = 0; o < 64; ++o) {
            double z = net->b1[o];
            for (int i = 0; i < 12; ++i) z += (q ? to_bf16(net->W1[o * 12 + i]) : net->W1[o * 12 + i]) * x0[i];
            h1[o] = q ? to_bf16(silu(z)) : silu(z);
        }
        for (int o = 0; o < 64; ++o) {
            double z = net->b2[o];
            for (int i = 0; i < 64; ++i) z += (q ? to_bf16(net->W2[o * 64 + i]) : net->W2[o * 64 + i]) * h1[i];
            h2[o] = q ? to_bf16(silu(z)) : silu(z);
        }
        for (int o = 0; o < 3; ++o) {
            double z = net->b3[o];
            for (int i = 0; i < 64; ++i) z += (q ? to_bf16(net->W3[o * 64 + i]) : net->W3[o * 64 + i]) * h2[i];
            out[3 * b + o] = z;
        }
    }
}

double orc_mlp_loss_grad(const orc_mlp* net, int64_t B, const double* feat, const double* label, double* grads)
{
    double* gW1 = grads;
    double* gb1 = gW1 + 64 * 12;
    double* gW2 = gb1 + 64;
    double* gb2 = gW2 + 64 * 64;
    double* gW3 = gb2 + 64;
    double* gb3 = gW3 + 3 * 64;
    memset(grads, 0, sizeof(double) * (64 * 12 + 64 + 64 * 64 + 64 + 3 * 64 + 3));
    double loss = 0.0;
    for (int64_t b = 0; b < B; ++b) {
        double x0[12], z1[64], h1[64], z2[64], h2[64], y[3];
        for (int i = 0; i < 12; ++i) x0[i] = feat[12 * b + i] * net->in_scale[i];
        for (int o = 0; o < 64; ++o) {
            double z = net->b1[o];
            for (int i = 0; i < 12; ++i) z += net->W1[o * 12 + i] * x0[i];
            z1[o] = z; h1[o] = silu(z);
        }
        for (int o = 0; o < 64; ++o) {
            double z = net->b2[o];
            for (int i = 0; i < 64; ++i) z += net->W2[o * 64 + i] * h1[i];
            z2[o] = z; h2[o] = silu(z);
        }
        double gy[3];
        for (int o = 0; o < 3; ++o) {
            double z = net->b3[o];
            for (int i = 0; i < 64; ++i) z += net->W3[o * 64 + i] * h2[i];
            y[o] = z;
            double e = y[o] - label[3 * b + o];
            loss += 0.5 * e * e;
            gy[o] = e / (double)B;
        }
        double gh2[64], gz2[64], gh1[64], gz1[64];
        for (int i = 0; i < 64; ++i) gh2[i] = 0.0;
        for (int o = 0; o < 3; ++o) {
            gb3[o] += gy[o];
            for (int i = 0; i < 64; ++i) {
                gW3[o * 64 + i] += gy[o] * h2[i];
                gh2[i] += net->W3[o * 64 + i] * gy[o];
            }
        }
        for (int i = 0; i < 64; ++i) { gz2[i] = gh2[i] * dsilu(z2[i]); gh1[i] = 0.0; }
        for (int o = 0; o < 64; ++o) {
            gb2[o] += gz2[o];
            for (int i = 0; i < 64; ++i) {
                gW2[o * 64 + i] += gz2[o] * h1[i];
                gh1[i] += net->W2[o * 64 + i] * gz2[o];
            }
        }
        for (int i = 0; i < 64; ++i) gz1[i] = gh1[i] * dsilu(z1[i]);
        for (int o = 0; o < 64; ++o) {
            gb1[o] += gz1[o];
            for (int i = 0; i < 12; ++i) gW1[o * 12 + i] += gz1[o] * x0[i];
        }
    }
    return loss / (double)B;
}

/* ------------------------------------------------------------------ */
/* Learned-start features (12 per contact) and the contact frame.       */
/* ------------------------------------------------------------------ */
static void contact_frame(const row* R, const double u[3], const double ltp[3], double t1[3], double t2[3])
{
    double un = dot3(R->n, u);
    double ut[3] = {u[0] - un * R->n[0], u[1] - un * R->n[1], u[2] - un * R->n[2]};
    double m = sqrt(dot3(ut, ut));
    double src[3];
    if (m > 1e-12) { for (int k = 0; k < 3; ++k) src[k] = ut[k] / m; }
    else {
        double lm = sqrt(dot3(ltp, ltp));
        if (lm > 0.0) { for (int k = 0; k < 3; ++k) src[k] = ltp[k] / lm; }
        else {
            /* any unit vector orthogonal to n: the axis least aligned with n */
            double ax[3] = {0.0, 0.0, 0.0};
            int k0 = 0;
            for (int k = 1; k < 3; ++k) if (fabs(R->n[k]) < fabs(R->n[k0])) k0 = k;
            ax[k0] = 1.0;
            double dn = dot3(ax, R->n);
            for (int k = 0; k < 3; ++k) src[k] = ax[k] - dn * R->n[k];
            double sm = sqrt(dot3(src, src));
            for (int k = 0; k < 3; ++k) src[k] /= sm;
        }
    }
    for (int k = 0; k < 3; ++k) t1[k] = src[k];
    cross3(R->n, t1, t2);
}

/* Column of a particle for the depth feature (reading R42): the (x, y) index
 * of the detection cell grid, cell width h = 2 r_max (1 + kappa_c) * 1.001
 * from the grid's low corner, clamped to the grid.  The index is an integer
 * decided by floating point, so it is taken in single precision on the
 * single-precision state, the precision of the measured path. */
static void column_of(const orc_params* P, double rmax, const double* x, int64_t* cx, int64_t* cy)
{
    double h = 2.0 * rmax * (1.0 + (P->m.c_p > 0.0 ? P->m.kappa_c : 0.0)) * 1.001;
    float inv = (float)(1.0 / h);
    int64_t dims[2];
    for (int k = 0; k < 2; ++k) {
        double ext = P->grid_hi[k] - P->grid_lo[k];
        double dd = ceil(ext / h);
        dims[k] = dd < 1.0 ? 1 : (int64_t)dd;
    }
    float lo0 = (float)P->grid_lo[0], lo1 = (float)P->grid_lo[1];
    float f0 = ((float)x[0] - lo0) * inv, f1 = ((float)x[1] - lo1) * inv;
    float g0 = floorf(f0), g1 = floorf(f1);
    if (!(g0 >= 0.0f)) g0 = 0.0f;
    if (!(g1 >= 0.0f)) g1 = 0.0f;
    if (g0 > (float)(dims[0] - 1)) g0 = (float)(dims[0] - 1);
    if (g1 > (float)(dims[1] - 1)) g1 = (float)(dims[1] - 1);
    *cx = (int64_t)g0;
    *cy = (int64_t)g1;
}

/* depth_i = max over the particle's column of (z + r) minus z_i */
static void column_depths(const orc_params* P, int64_t n, const double* x, const double* r, double* depth)
{
    double rmax = 0.0;
    for (int64_t i = 0; i < n; ++i) if (r[i] > rmax) rmax = r[i];
    cell_entry* ce = (cell_entry*)malloc((size_t)(n > 0 ? n : 1) * sizeof(cell_entry));
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx, cy;
        column_of(P, rmax, &x[3 * i], &cx, &cy);
        ce[i].cell = cy * 1048576 + cx;
        ce[i].idx = i;
    }
    qsort(ce, (size_t)n, sizeof(cell_entry), cmp_cell);
    for (int64_t s0 = 0; s0 < n;) {
        int64_t s1 = s0;
        double top = -1e300;
        while (s1 < n && ce[s1].cell == ce[s0].cell) {
            int64_t j = ce[s1].idx;
            if (x[3 * j + 2] + r[j] > top) top = x[3 * j + 2] + r[j];
            ++s1;
        }
        for (int64_t t = s0; t < s1; ++t) depth[ce[t].idx] = top - x[3 * ce[t].idx + 2];
        s0 = s1;
    }
    free(ce);
}

/* The 12 inputs of the learned start (one reading of the configuration's
 * "overlap, normal/tangential relative velocity, previous-step impulses,
 * depth below free surface, radii"), the frame and the impulse scale. */
static void learned_features(const orc_params* P, int64_t n, const double* x, const double* r,
                             const double* v, const double* w, const row* rows, int64_t nc,
                             const double* lnprev, const double* ltprev, double* F, double (*frames)[6],
                             double* scale)
{
    double* depth = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    column_depths(P, n, x, r, depth);
    double gmag = sqrt(dot3(P->g, P->g));
    double gdt = gmag * P->dt;
    for (int64_t c = 0; c < nc; ++c) {
        const row* R = &rows[c];
        double u[3];
        rel_vel(R, v, w, u);
        double un = dot3(R->n, u);
        double ut[3] = {u[0] - un * R->n[0], u[1] - un * R->n[1], u[2] - un * R->n[2]};
        double t1[3], t2[3];
        contact_frame(R, u, &ltprev[3 * c], t1, t2);
        double ls = (1.0 / R->Wn) * gdt;
        double rbar = R->a >= 0 ? 0.5 * (r[R->a] + r[R->b]) : r[R->b];
        double* f = &F[12 * c];
        f[0] = R->delta / rbar;
        f[1] = un / gdt;
        f[2] = sqrt(dot3(ut, ut)) / gdt;
        f[3] = lnprev[c] / ls;
        f[4] = dot3(&ltprev[3 * c], t1) / ls;
        f[5] = dot3(&ltprev[3 * c], t2) / ls;
        f[6] = R->a >= 0 ? depth[R->a] / rbar : 0.0;
        f[7] = depth[R->b] / rbar;
        f[8] = R->a >= 0 ? r[R->a] / P->r_ref : 0.0;
        f[9] = r[R->b] / P->r_ref;
        f[10] = R->a >= 0 ? 0.0 : 1.0;
        f[11] = R->persistent ? 1.0 : 0.0;
        for (int k = 0; k < 3; ++k) { frames[c][k] = t1[k]; frames[c][3 + k] = t2[k]; }
        scale[c] = ls;
    }
    free(depth);
}

/* ------------------------------------------------------------------ */
/* Public entry points                                                  */
/* ------------------------------------------------------------------ */
int64_t orc_detect(const orc_params* P, int64_t n, const int64_t* id, const double* x, const double* r,
                   int32_t nb, const orc_body* bodies, int32_t ns, const orc_shape* shapes,
                   int64_t cap, uint64_t* keys, double* delta)
{
    raw_contact* rc = NULL;
    int64_t nc = detect_all(P, n, id, x, r, nb, bodies, ns, shapes, &rc);
    if (nc > cap) { free(rc); return -5; }
    for (int64_t c = 0; c < nc; ++c) {
        keys[c] = rc[c].key;
        if (delta) {
            if (rc[c].a >= 0) {
                int64_t a = rc[c].a, b = rc[c].b;
                double e[3] = {x[3 * b] - x[3 * a], x[3 * b + 1] - x[3 * a + 1], x[3 * b + 2] - x[3 * a + 2]};
                delta[c] = (r[a] + r[b]) - sqrt(dot3(e, e));
            } else {
                double nr[3];
                shape_touch(P, &shapes[rc[c].shape], bodies, &x[3 * rc[c].b], r[rc[c].b], &delta[c], nr);
            }
        }
    }
    free(rc);
    return nc;
}

static void make_inv_mass(const orc_params* P, int64_t n, const double* r, const double* rho, inv_mass* M)
{
    M->im = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    M->iI = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double m = particle_mass(P, rho, i, r);
        M->im[i] = 1.0 / m;
        M->iI[i] = 1.0 / (0.4 * m * r[i] * r[i]);
    }
}

/* Look up key in the previous cache (sorted); returns index or -1. */
static int64_t find_prev(int64_t nprev, const uint64_t* keys, uint64_t k)
{
    int64_t a = 0, b = nprev;
    while (a < b) {
        int64_t m = (a + b) / 2;
        if (keys[m] < k) a = m + 1; else b = m;
    }
    return (a < nprev && keys[a] == k) ? a : -1;
}

/* Aggregate body of every zone (Eqs. aggregate_mass .. aggregate_rot_vel):
 * particles are labelled with the first body (in order) whose zone contains
 * them; sums over particles only, with the spheres' own inertia 2/5 m r^2
 * and spin (the inertia formula as printed is read as the standard
 * parallel-axis sum about x_A). */
/* Height and gradient of a heightfield at (x, y): Eq. surface, the grid
 * heights interpolated linearly in each direction (bilinear), clamped to the
 * border cells. */
static double hf_eval(const orc_shape* s, double x, double y, double* hx, double* hy)
{
    double inv = 1.0 / s->l0;
    double fx = (x - s->ox) * inv;
    double fy = (y - s->oy) * inv;
    double fi = floor(fx), fj = floor(fy);
    if (fi < 0.0) fi = 0.0;
    if (fi > (double)(s->nx - 2)) fi = (double)(s->nx - 2);
    if (fj < 0.0) fj = 0.0;
    if (fj > (double)(s->ny - 2)) fj = (double)(s->ny - 2);
    int i = (int)fi, j = (int)fj;
    double t = fx - fi, u = fy - fj;
    double h00 = s->h[j * s->nx + i], h10 = s->h[j * s->nx + i + 1];
    double h01 = s->h[(j + 1) * s->nx + i], h11 = s->h[(j + 1) * s->nx + i + 1];
    *hx = ((h10 - h00) * (1.0 - u) + (h11 - h01) * u) * inv;
    *hy = ((h01 - h00) * (1.0 - t) + (h11 - h10) * t) * inv;
    return (h00 * (1.0 - t) + h10 * t) * (1.0 - u) + (h01 * (1.0 - t) + h11 * t) * u;
}

static void normalize3(double* a)
{
    double m = sqrt(dot3(a, a));
    for (int k = 0; k < 3; ++k) a[k] /= m;
}

/* The active zone of a cutting edge: for each lateral slice, the wedge
 * between the separation plate through the edge and the failure plane that
 * rises from the edge at theta(phi, beta) = pi/2 - (phi + beta)/2 against
 * the terrain surface (Eq. failure_plane), up to where it meets the surface
 * (plus the heap allowance), between the slice's lateral planes.  beta is the
 * angle from the surface to the separation plate, both taken in the plane
 * normal to the edge; the plate's normal is interpolated between the primary
 * plate and the inner face by the fill ratio. */
int32_t orc_predict_wedges(const orc_tool* t, const orc_body* bodies, const orc_shape* terrain, orc_wedge* out)
{
    if (t->n_wedges < 1 || t->n_wedges > ORC_MAX_WEDGES || !(t->fill >= 0.0 && t->fill <= 1.0)) return -1;
    const orc_body* B = &bodies[t->body];
    double R[3][3];
    quat_matrix(B->quat, R);
    double E0[3], E1[3], nc[3], ntc[3];
    for (int k = 0; k < 3; ++k) {
        E0[k] = B->pos[k] + ((R[k][0] * t->edge0[0] + R[k][1] * t->edge0[1]) + R[k][2] * t->edge0[2]);
        E1[k] = B->pos[k] + ((R[k][0] * t->edge1[0] + R[k][1] * t->edge1[1]) + R[k][2] * t->edge1[2]);
        nc[k] = (R[k][0] * t->n_c[0] + R[k][1] * t->n_c[1]) + R[k][2] * t->n_c[2];
        ntc[k] = (R[k][0] * t->n_tc[0] + R[k][1] * t->n_tc[1]) + R[k][2] * t->n_tc[2];
    }
    for (int w = 0; w < t->n_wedges; ++w) out[w].n = 0;
    if (!terrain) return t->n_wedges;
    if (t->v_min > 0.0) {
        /* a deformer resolves its zone only while its edge moves fast enough */
        double mid[3], arm[3], ve[3];
        for (int k = 0; k < 3; ++k) { mid[k] = 0.5 * (E0[k] + E1[k]); arm[k] = mid[k] - B->pos[k]; }
        cross3(B->angvel, arm, ve);
        for (int k = 0; k < 3; ++k) ve[k] += B->linvel[k];
        if (!(sqrt(dot3(ve, ve)) > t->v_min)) return t->n_wedges;
    }
    double nf[3], L[3], l[3];
    for (int k = 0; k < 3; ++k) {
        nf[k] = (1.0 - t->fill) * nc[k] + t->fill * ntc[k];
        L[k] = E1[k] - E0[k];
        l[k] = L[k];
    }
    normalize3(nf);
    normalize3(l);
    const double zh[3] = {0.0, 0.0, 1.0};
    double u[3], p[3];
    cross3(zh, l, u);        /* horizontal, normal to the edge */
    normalize3(u);
    if (dot3(u, nf) < 0.0) for (int k = 0; k < 3; ++k) u[k] = -u[k];
    cross3(l, nf, p);        /* the plate's direction away from the edge */
    normalize3(p);
    if (p[2] < 0.0) for (int k = 0; k < 3; ++k) p[k] = -p[k];
    for (int w = 0; w < t->n_wedges; ++w) {
        double a[3], b[3], m[3];
        double fa = (double)w / t->n_wedges, fb = (double)(w + 1) / t->n_wedges, fm = (w + 0.5) / t->n_wedges;
        for (int k = 0; k < 3; ++k) { a[k] = E0[k] + L[k] * fa; b[k] = E0[k] + L[k] * fb; m[k] = E0[k] + L[k] * fm; }
        double hx, hy;
        double h0 = hf_eval(terrain, m[0], m[1], &hx, &hy);
        if (!(m[2] < h0)) continue;  /* the edge is not below the surface */
        /* surface tangent and its upward normal in the plane normal to the edge */
        double s[3] = {u[0], u[1], u[2] + (hx * u[0] + hy * u[1])};
        double sl = dot3(s, l);
        for (int k = 0; k < 3; ++k) s[k] -= sl * l[k];
        normalize3(s);
        double ns[3];
        cross3(l, s, ns);
        if (ns[2] < 0.0) for (int k = 0; k < 3; ++k) ns[k] = -ns[k];
        double beta = atan2(dot3(p, ns), dot3(p, s));
        double theta = 0.5 * PI - 0.5 * (t->phi + beta);
        if (!(theta > 0.0 && theta < 0.5 * PI)) continue;
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = cos(theta) * s[k] + sin(theta) * ns[k];
        /* where the failure line from the edge meets the surface: bracket by
         * doubling from one grid spacing, then 60 bisections */
        double lo = 0.0, hi = terrain->l0;
        int found = 0;
        for (int it = 0; it < 40; ++it) {
            double q[3] = {m[0] + hi * d[0], m[1] + hi * d[1], m[2] + hi * d[2]};
            if (q[2] - hf_eval(terrain, q[0], q[1], &hx, &hy) >= 0.0) { found = 1; break; }
            lo = hi;
            hi *= 2.0;
        }
        if (!found) continue;
        for (int it = 0; it < 60; ++it) {
            double mid = 0.5 * (lo + hi);
            double q[3] = {m[0] + mid * d[0], m[1] + mid * d[1], m[2] + mid * d[2]};
            if (q[2] - hf_eval(terrain, q[0], q[1], &hx, &hy) >= 0.0) hi = mid;
            else lo = mid;
        }
        double ztop = (m[2] + hi * d[2]) + t->heap;
        double c[3];
        cross3(l, d, c);
        normalize3(c);
        if (dot3(c, p) > 0.0) for (int k = 0; k < 3; ++k) c[k] = -c[k];
        orc_wedge* W = &out[w];
        for (int k = 0; k < 3; ++k) {
            W->planes[0][k] = -nf[k];   /* in front of the separation plate */
            W->planes[1][k] = c[k];     /* above the failure plane */
            W->planes[2][k] = zh[k];    /* below the top */
            W->planes[3][k] = -l[k];    /* between the slice's lateral planes */
            W->planes[4][k] = l[k];
        }
        W->planes[0][3] = -dot3(nf, m);
        W->planes[1][3] = dot3(c, m);
        W->planes[2][3] = ztop;
        W->planes[3][3] = -dot3(l, a);
        W->planes[4][3] = dot3(l, b);
        W->n = 5;
    }
    return t->n_wedges;
}

static int in_planes(const double (*pl)[4], int np, const double* x)
{
    for (int p = 0; p < np; ++p)
        if (dot3(pl[p], x) - pl[p][3] > 0.0) return 0;
    return 1;
}

/* Aggregates with, per body, either its half-space zone or the union of its
 * tool's wedges (wedges[b] non-NULL, nw[b] of them). */
static int32_t aggregates_impl(int64_t n, const double* r, const double* inv_m, const double* x, const double* v,
                               const double* w, int32_t nb, const orc_body* bodies, orc_wedge* const* wedges,
                               const int32_t* nw, orc_aggregate* agg)
{
    int32_t na = 0;
    int32_t* zone_of = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    double (*wp)[8][4] = malloc((size_t)(nb > 0 ? nb : 1) * sizeof(double[8][4]));
    for (int32_t b = 0; b < nb; ++b) {
        double Rm[3][3];
        quat_matrix(bodies[b].quat, Rm);
        for (int p = 0; p < bodies[b].nplanes; ++p) {
            const double* pl = bodies[b].planes[p];
            double nw[3];
            for (int k = 0; k < 3; ++k) nw[k] = (Rm[k][0] * pl[0] + Rm[k][1] * pl[1]) + Rm[k][2] * pl[2];
            for (int k = 0; k < 3; ++k) wp[b][p][k] = nw[k];
            wp[b][p][3] = pl[3] + dot3(nw, bodies[b].pos);
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        zone_of[i] = -1;
        for (int32_t b = 0; b < nb && zone_of[i] < 0; ++b) {
            int in = 0;
            if (wedges && wedges[b]) {
                for (int32_t k = 0; k < nw[b] && !in; ++k)
                    in = wedges[b][k].n > 0 && in_planes(wedges[b][k].planes, wedges[b][k].n, &x[3 * i]);
            } else if (bodies[b].nplanes > 0) {
                in = in_planes(wp[b], bodies[b].nplanes, &x[3 * i]);
            }
            if (in) zone_of[i] = b;
        }
    }
    for (int32_t b = 0; b < nb; ++b) {
        if (!(wedges && wedges[b]) && bodies[b].nplanes <= 0) continue;
        orc_aggregate* A = &agg[na++];
        memset(A, 0, sizeof(*A));
        A->zone = b;
        double Mt = 0.0, mx[3] = {0, 0, 0}, mv[3] = {0, 0, 0};
        for (int64_t i = 0; i < n; ++i) {
            if (zone_of[i] != b) continue;
            double m = 1.0 / inv_m[i];
            A->n_particles++;
            Mt += m;
            for (int k = 0; k < 3; ++k) { mx[k] += m * x[3 * i + k]; mv[k] += m * v[3 * i + k]; }
        }
        A->M = Mt;
        if (Mt <= 0.0) continue;
        for (int k = 0; k < 3; ++k) { A->x[k] = mx[k] / Mt; A->v[k] = mv[k] / Mt; }
        double I[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, L[3] = {0, 0, 0};
        for (int64_t i = 0; i < n; ++i) {
            if (zone_of[i] != b) continue;
            double m = 1.0 / inv_m[i];
            double rho_[3] = {x[3 * i] - A->x[0], x[3 * i + 1] - A->x[1], x[3 * i + 2] - A->x[2]};
            double rr = dot3(rho_, rho_);
            double Is = 0.4 * m * r[i] * r[i];
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q)
                    I[p][q] += (p == q ? Is + m * rr : 0.0) - m * rho_[p] * rho_[q];
            double cxv[3];
            cross3(rho_, &v[3 * i], cxv);
            for (int k = 0; k < 3; ++k) L[k] += m * cxv[k] + Is * w[3 * i + k];
        }
        A->I[0] = I[0][0]; A->I[1] = I[1][1]; A->I[2] = I[2][2];
        A->I[3] = I[0][1]; A->I[4] = I[0][2]; A->I[5] = I[1][2];
        for (int k = 0; k < 3; ++k) A->L[k] = L[k];
        /* omega_A = I^-1 L by Cramer's rule */
        double det = I[0][0] * (I[1][1] * I[2][2] - I[1][2] * I[2][1])
                   - I[0][1] * (I[1][0] * I[2][2] - I[1][2] * I[2][0])
                   + I[0][2] * (I[1][0] * I[2][1] - I[1][1] * I[2][0]);
        for (int k = 0; k < 3; ++k) {
            double Mk[3][3];
            memcpy(Mk, I, sizeof(Mk));
            for (int p = 0; p < 3; ++p) Mk[p][k] = L[p];
            double dk = Mk[0][0] * (Mk[1][1] * Mk[2][2] - Mk[1][2] * Mk[2][1])
                      - Mk[0][1] * (Mk[1][0] * Mk[2][2] - Mk[1][2] * Mk[2][0])
                      + Mk[0][2] * (Mk[1][0] * Mk[2][1] - Mk[1][1] * Mk[2][0]);
            A->w[k] = det != 0.0 ? dk / det : 0.0;
        }
    }
    free(wp);
    free(zone_of);
    return na;
}

int32_t orc_aggregates(int64_t n, const double* r, const double* inv_m, const double* x, const double* v,
                       const double* w, int32_t nb, const orc_body* bodies, orc_aggregate* agg)
{
    return aggregates_impl(n, r, inv_m, x, v, w, nb, bodies, NULL, NULL, agg);
}

int32_t orc_aggregates_tools(int64_t n, const double* r, const double* inv_m, const double* x, const double* v,
                             const double* w, int32_t nb, const orc_body* bodies, int32_t ntools,
                             const orc_tool* tools, const orc_shape* terrain, orc_aggregate* agg)
{
    orc_wedge** wedges = (orc_wedge**)calloc((size_t)(nb > 0 ? nb : 1), sizeof(orc_wedge*));
    int32_t* nw = (int32_t*)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int32_t));
    orc_wedge* pool = (orc_wedge*)calloc((size_t)(ntools > 0 ? ntools : 1) * ORC_MAX_WEDGES, sizeof(orc_wedge));
    int32_t na = -1;
    for (int32_t k = 0; k < ntools; ++k) {
        const orc_tool* T = &tools[k];
        if (T->body < 0 || T->body >= nb || wedges[T->body]) goto done;  /* one tool per body */
        orc_wedge* W = pool + (size_t)k * ORC_MAX_WEDGES;
        if (orc_predict_wedges(T, bodies, terrain, W) < 0) goto done;
        wedges[T->body] = W;
        nw[T->body] = T->n_wedges;
    }
    na = aggregates_impl(n, r, inv_m, x, v, w, nb, bodies, wedges, nw, agg);
done:
    free(pool); free(nw); free(wedges);
    return na;
}

/* Run one sweep over all colours; returns the residual of that sweep. */
static double sweep(row* rows, int64_t nc, int ncol, const int64_t* cstart, const int64_t* corder,
                    const inv_mass* M, double* v, double* w, double gamma_dt)
{
    double acc[2] = {0.0, 0.0};
    for (int col = 0; col < ncol; ++col)
        for (int64_t t = cstart[col]; t < cstart[col + 1]; ++t)
            pgs_contact(&rows[corder[t]], M, v, w, gamma_dt, acc);
    (void)nc;
    if (acc[1] > 0.0) return sqrt(acc[0]) / sqrt(acc[1]);
    return acc[0] > 0.0 ? 1.0 : 0.0;
}

/* Warm-start values lambda^0 for every contact into (ln0, lt0). */
static void apply_start(row* rows, int64_t nc, const inv_mass* M, double* v, double* w)
{
    for (int64_t c = 0; c < nc; ++c) {
        row* R = &rows[c];
        project(R, &R->ln, R->lt);
        double J[3];
        for (int k = 0; k < 3; ++k) J[k] = R->ln * R->n[k] + R->lt[k];
        apply_impulse(R, M, v, w, J);
        if (R->rlim > 0.0) {
            project_r(R, R->lr);
            apply_torque(R, M, w, R->lr);
        } else {
            R->lr[0] = R->lr[1] = R->lr[2] = 0.0;
        }
    }
}

/* Impact stage, solved before the main solve (the paper's separation of
 * impacts from resting contacts).  A contact whose normal velocity at the
 * start of the step approaches faster than v_imp is an impact and gets the
 * Newton law G_n v+ = -e G_n v-; every other contact keeps its velocity-level
 * constraints G v+ = 0: a unilateral normal row, Coulomb friction and the
 * rolling bound, with the stage's own impulses.  The rows are the step's
 * rows without compliance, regularisation or cohesion, cold-started and
 * swept in the same colour order as the main solve, with its sweep cap and
 * tolerance.  v, w are updated in place; the stage's impulses are returned
 * in li (4 per contact) and lri (3 per contact).  Returns the number of
 * impacts (0: nothing was done). */
static int64_t impact_stage(const orc_params* P, const row* rows, int64_t nc, int ncol, const int64_t* cstart,
                            const int64_t* corder, const inv_mass* M, double* v, double* w, double* li,
                            double* lri, int* sweeps_out)
{
    *sweeps_out = 0;
    if (!(P->m.v_imp > 0.0) || nc == 0) return 0;
    int64_t nimp = 0;
    row* ri = (row*)malloc((size_t)nc * sizeof(row));
    memcpy(ri, rows, (size_t)nc * sizeof(row));
    for (int64_t c = 0; c < nc; ++c) {
        row* R = &ri[c];
        double u[3];
        rel_vel(R, v, w, u);
        double un = dot3(R->n, u);
        int impact = un < -P->m.v_imp;
        nimp += impact;
        R->Sig = 0.0;
        R->Dn = R->Wn;
        R->Dt = R->Wt;
        R->lo = 0.0;
        R->q = impact ? -P->m.restitution * un : 0.0;
        R->ln = 0.0;
        for (int k = 0; k < 3; ++k) R->lt[k] = R->lr[k] = 0.0;
    }
    if (nimp > 0) {
        int k = 0;
        double Rk = 1.0;
        while (k < P->max_sweeps) {
            if (k > 0 && P->tol > 0.0 && Rk <= P->tol) break;
            Rk = sweep(ri, nc, ncol, cstart, corder, M, v, w, 0.0);
            ++k;
        }
        *sweeps_out = k;
        for (int64_t c = 0; c < nc; ++c) {
            li[4 * c] = ri[c].ln;
            for (int j = 0; j < 3; ++j) { li[4 * c + 1 + j] = ri[c].lt[j]; lri[3 * c + j] = ri[c].lr[j]; }
        }
    }
    free(ri);
    return nimp;
}

int64_t orc_step(const orc_params* P,
                 int64_t n, const int64_t* id, const double* r, const double* rho,
                 double* x, double* v, double* w,
                 int32_t nb, orc_body* bodies,
                 int32_t ns, const orc_shape* shapes,
                 int64_t nprev, const uint64_t* prev_keys, const double* prev_lam, const double* prev_lr,
                 const orc_mlp* mlp,
                 int64_t cap, uint64_t* keys_out, double* lam_out, double* lr_out, int32_t* colour_out,
                 orc_stats* st, double* body_ft,
                 orc_aggregate* agg, int32_t* n_agg, double* resid)
{
    if (P->m.mu_r < 0.0 || !(P->m.restitution >= 0.0 && P->m.restitution <= 1.0)) return -1;
    double dt = P->dt;
    inv_mass M;
    make_inv_mass(P, n, r, rho, &M);

    /* 1-2. detection and canonical order */
    raw_contact* rc = NULL;
    int64_t nc = detect_all(P, n, id, x, r, nb, bodies, ns, shapes, &rc);
    if (nc > cap) {
        free(rc); free(M.im); free(M.iI);
        return -5;
    }
    row* rows = (row*)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(row));

    /* 3-5. rows from the start-of-step state */
    build_rows(P, id, r, &M, x, v, w, bodies, shapes, rc, nc, rows);
    free(rc);

    /* previous-step impulses, matched by key */
    double* ltprev = (double*)calloc((size_t)(nc > 0 ? nc : 1) * 3, sizeof(double));
    double* lnprev = (double*)calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    double* lrprev = (double*)calloc((size_t)(nc > 0 ? nc : 1) * 3, sizeof(double));
    for (int64_t c = 0; c < nc; ++c) {
        int64_t k = nprev > 0 ? find_prev(nprev, prev_keys, rows[c].key) : -1;
        rows[c].persistent = k >= 0;
        if (k >= 0 && prev_lr)
            for (int j = 0; j < 3; ++j) lrprev[3 * c + j] = prev_lr[3 * k + j];
        if (k >= 0) {
            lnprev[c] = prev_lam[4 * k];
            for (int j = 0; j < 3; ++j) ltprev[3 * c + j] = prev_lam[4 * k + 1 + j];
            /* re-project onto the new tangent plane */
            double tn = dot3(rows[c].n, &ltprev[3 * c]);
            for (int j = 0; j < 3; ++j) ltprev[3 * c + j] -= tn * rows[c].n[j];
        }
    }

    /* start-of-step velocities (the learned start's inputs) */
    double* v0 = (double*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    double* w0 = (double*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    memcpy(v0, v, (size_t)n * 3 * sizeof(double));
    memcpy(w0, w, (size_t)n * 3 * sizeof(double));

    /* colouring and colour-ordered contact list */
    int ncol = colour_contacts(rows, nc, n);
    int64_t* cstart = (int64_t*)calloc((size_t)ncol + 2, sizeof(int64_t));
    int64_t* corder = (int64_t*)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    for (int64_t c = 0; c < nc; ++c) cstart[rows[c].colour + 1]++;
    for (int k = 0; k < ncol; ++k) cstart[k + 1] += cstart[k];
    {
        int64_t* f = (int64_t*)malloc((size_t)(ncol + 1) * sizeof(int64_t));
        memcpy(f, cstart, (size_t)(ncol + 1) * sizeof(int64_t));
        for (int64_t c = 0; c < nc; ++c) corder[f[rows[c].colour]++] = c;
        free(f);
    }

    /* impact stage on the start-of-step velocities; the main rows' velocity
     * term then takes the post-impact velocities */
    double* li = (double*)calloc((size_t)(nc > 0 ? nc : 1) * 4, sizeof(double));
    double* lri = (double*)calloc((size_t)(nc > 0 ? nc : 1) * 3, sizeof(double));
    int impact_sweeps = 0;
    int64_t nimp = impact_stage(P, rows, nc, ncol, cstart, corder, &M, v, w, li, lri, &impact_sweeps);
    if (nimp > 0) {
        double tau = P->m.tau_n > 0.0 ? P->m.tau_n : 2.0 * dt;
        double Ups = 1.0 / (1.0 + 4.0 * tau / dt);
        for (int64_t c = 0; c < nc; ++c) {
            double u[3];
            rel_vel(&rows[c], v, w, u);
            rows[c].q = rows[c].qg + Ups * dot3(rows[c].n, u);
        }
    }

    /* 6. prediction v* = v + dt g */
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) v[3 * i + k] += dt * P->g[k];

    double gamma_dt = P->m.gamma_t / dt;
    int sweeps_done = 0;
    double R = 1.0;
    int fallback = 0, learned_used = 0;
    double r1 = 0.0, r1_trial[2] = {0.0, 0.0};

    /* warm start (A8): cold, previous-step, or learned with fallback */
    for (int64_t c = 0; c < nc; ++c) {
        rows[c].ln = 0.0;
        for (int j = 0; j < 3; ++j) rows[c].lt[j] = rows[c].lr[j] = 0.0;
    }
    int have_prev = 0;
    for (int64_t c = 0; c < nc; ++c) have_prev |= rows[c].persistent;
    if (P->warm == ORC_PREV || P->warm == ORC_LEARNED) {
        for (int64_t c = 0; c < nc; ++c) {
            rows[c].ln = lnprev[c];
            for (int j = 0; j < 3; ++j) rows[c].lt[j] = ltprev[3 * c + j];
            for (int j = 0; j < 3; ++j) rows[c].lr[j] = lrprev[3 * c + j];
        }
    }
    if (P->warm == ORC_LEARNED && mlp && nc > 0 && P->max_sweeps > 0) {
        /* trial: learned start and its first sweep */
        double* F = (double*)malloc((size_t)nc * 12 * sizeof(double));
        double (*fr)[6] = malloc((size_t)nc * sizeof(double[6]));
        double* lsc = (double*)malloc((size_t)nc * sizeof(double));
        double* y = (double*)malloc((size_t)nc * 3 * sizeof(double));
        learned_features(P, n, x, r, v0, w0, rows, nc, lnprev, ltprev, F, fr, lsc);
        orc_mlp_forward(mlp, nc, F, y);
        int finite = 1;
        row* rl = (row*)malloc((size_t)nc * sizeof(row));
        memcpy(rl, rows, (size_t)nc * sizeof(row));
        for (int64_t c = 0; c < nc; ++c) {
            /* residual form: the output corrects the previous-step impulse
             * (inputs 3-5, in the contact frame), so a zero output gives the
             * previous-step start */
            double ls = lsc[c];
            const double* f = &F[12 * c];
            double yn = f[3] + y[3 * c], y1 = f[4] + y[3 * c + 1], y2 = f[5] + y[3 * c + 2];
            rl[c].ln = yn * ls;
            for (int k = 0; k < 3; ++k) rl[c].lt[k] = (y1 * fr[c][k] + y2 * fr[c][3 + k]) * ls;
            if (!isfinite(rl[c].ln) || !isfinite(rl[c].lt[0]) || !isfinite(rl[c].lt[1]) || !isfinite(rl[c].lt[2])) finite = 0;
        }
        double* vl = (double*)malloc((size_t)n * 3 * sizeof(double));
        double* wl = (double*)malloc((size_t)n * 3 * sizeof(double));
        memcpy(vl, v, (size_t)n * 3 * sizeof(double));
        memcpy(wl, w, (size_t)n * 3 * sizeof(double));
        double r1l = 1e300;
        if (finite) {
            apply_start(rl, nc, &M, vl, wl);
            r1l = sweep(rl, nc, ncol, cstart, corder, &M, vl, wl, gamma_dt);
            if (!isfinite(r1l)) finite = 0;
        }
        /* reference: previous-step start (cold when there is no cache) */
        apply_start(rows, nc, &M, v, w);
        double r1p = sweep(rows, nc, ncol, cstart, corder, &M, v, w, gamma_dt);
        r1_trial[0] = r1l;
        r1_trial[1] = r1p;
        if (finite && !(r1l > r1p)) {
            memcpy(rows, rl, (size_t)nc * sizeof(row));
            memcpy(v, vl, (size_t)n * 3 * sizeof(double));
            memcpy(w, wl, (size_t)n * 3 * sizeof(double));
            R = r1l;
            learned_used = 1;
        } else {
            R = r1p;
            fallback = 1;
        }
        (void)have_prev;
        r1 = R;
        if (resid) resid[0] = R;
        sweeps_done = 1;
        free(vl); free(wl); free(rl); free(y); free(lsc); free(fr); free(F);
    } else {
        apply_start(rows, nc, &M, v, w);
    }

    /* 7. PGS sweeps in colour order */
    while (sweeps_done < P->max_sweeps) {
        if (sweeps_done > 0 && P->tol > 0.0 && R <= P->tol) break;
        R = sweep(rows, nc, ncol, cstart, corder, &M, v, w, gamma_dt);
        if (resid) resid[sweeps_done] = R;
        if (sweeps_done == 0) r1 = R;
        ++sweeps_done;
    }

    /* 8. symplectic position update and kinematic poses */
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) x[3 * i + k] += dt * v[3 * i + k];

    /* 9. contact force and torque on each kinematic body (start-of-step pose) */
    if (body_ft) {
        for (int32_t b = 0; b < nb; ++b) for (int k = 0; k < 6; ++k) body_ft[6 * b + k] = 0.0;
        for (int64_t c = 0; c < nc; ++c) {
            const row* Rw = &rows[c];
            if (Rw->a >= 0) continue;
            const orc_body* B = &bodies[Rw->body];
            double f[3], arm[3], t[3];
            /* the step's impulses: main solve and impact stage */
            double ln = Rw->ln + li[4 * c];
            for (int k = 0; k < 3; ++k) f[k] = -(ln * Rw->n[k] + Rw->lt[k] + li[4 * c + 1 + k]) / dt;
            for (int k = 0; k < 3; ++k) arm[k] = Rw->p[k] - B->pos[k];
            cross3(arm, f, t);
            for (int k = 0; k < 3; ++k) t[k] -= (Rw->lr[k] + lri[3 * c + k]) / dt;  /* the rolling couple */
            for (int k = 0; k < 3; ++k) { body_ft[6 * Rw->body + k] += f[k]; body_ft[6 * Rw->body + 3 + k] += t[k]; }
        }
    }
    for (int32_t b = 0; b < nb; ++b) {
        orc_body* B = &bodies[b];
        for (int k = 0; k < 3; ++k) B->pos[k] += dt * B->linvel[k];
        /* q <- normalize(q + dt/2 (0, w) (x) q) */
        double q0 = B->quat[0], q1 = B->quat[1], q2 = B->quat[2], q3 = B->quat[3];
        double wx = B->angvel[0], wy = B->angvel[1], wz = B->angvel[2];
        double h = 0.5 * dt;
        double n0 = q0 + h * (-wx * q1 - wy * q2 - wz * q3);
        double n1 = q1 + h * (wx * q0 + wy * q3 - wz * q2);
        double n2 = q2 + h * (-wx * q3 + wy * q0 + wz * q1);
        double n3 = q3 + h * (wx * q2 - wy * q1 + wz * q0);
        double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2 + n3 * n3);
        B->quat[0] = n0 / nn; B->quat[1] = n1 / nn; B->quat[2] = n2 / nn; B->quat[3] = n3 / nn;
    }

    /* 10. aggregate bodies of the active zones (Eqs. aggregate_mass..rot_vel) */
    if (agg && n_agg) {
        if (P->ntools > 0) {
            const orc_shape* terrain = NULL;
            for (int32_t k = 0; k < ns && !terrain; ++k)
                if (shapes[k].type == ORC_HFIELD) terrain = &shapes[k];
            *n_agg = orc_aggregates_tools(n, r, M.im, x, v, w, nb, bodies, P->ntools, P->tools, terrain, agg);
        } else {
            *n_agg = orc_aggregates(n, r, M.im, x, v, w, nb, bodies, agg);
        }
    }

    /* 11. outputs and the cache of this step */
    for (int64_t c = 0; c < nc; ++c) {
        keys_out[c] = rows[c].key;
        if (lam_out) {
            lam_out[4 * c] = rows[c].ln;
            for (int k = 0; k < 3; ++k) lam_out[4 * c + 1 + k] = rows[c].lt[k];
        }
        if (lr_out)
            for (int k = 0; k < 3; ++k) lr_out[3 * c + k] = rows[c].lr[k];
        if (colour_out) colour_out[c] = rows[c].colour;
    }
    if (st) {
        int64_t np = 0;
        for (int64_t c = 0; c < nc; ++c) np += rows[c].a >= 0;
        st->contacts = nc;
        st->pair_contacts = np;
        st->colours = ncol;
        st->sweeps = sweeps_done;
        st->residual = R;
        st->fallback_used = fallback;
        st->learned_used = learned_used;
        st->r1_first = r1;
        st->r1_trial[0] = r1_trial[0];
        st->r1_trial[1] = r1_trial[1];
        st->impacts = (int32_t)nimp;
        st->impact_sweeps = impact_sweeps;
    }
    free(ltprev); free(lnprev); free(lrprev); free(v0); free(w0); free(li); free(lri);
    free(cstart); free(corder); free(rows);
    free(M.im); free(M.iI);
    return nc;
}

int64_t orc_features(const orc_params* P, int64_t n, const int64_t* id, const double* r, const double* rho,
                     const double* x, const double* v, const double* w,
                     int32_t nb, const orc_body* bodies, int32_t ns, const orc_shape* shapes,
                     int64_t nprev, const uint64_t* prev_keys, const double* prev_lam,
                     int64_t cap, double* feat, double* frame, double* scale)
{
    inv_mass M;
    make_inv_mass(P, n, r, rho, &M);
    raw_contact* rc = NULL;
    int64_t nc = detect_all(P, n, id, x, r, nb, bodies, ns, shapes, &rc);
    if (nc > cap) { free(rc); free(M.im); free(M.iI); return -5; }
    row* rows = (row*)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(row));
    build_rows(P, id, r, &M, x, v, w, bodies, shapes, rc, nc, rows);
    free(rc);
    double* lt = (double*)calloc((size_t)(nc > 0 ? nc : 1) * 3, sizeof(double));
    double* ln = (double*)calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    for (int64_t c = 0; c < nc; ++c) {
        int64_t k = nprev > 0 ? find_prev(nprev, prev_keys, rows[c].key) : -1;
        rows[c].persistent = k >= 0;
        if (k >= 0) {
            ln[c] = prev_lam[4 * k];
            for (int j = 0; j < 3; ++j) lt[3 * c + j] = prev_lam[4 * k + 1 + j];
            double tn = dot3(rows[c].n, &lt[3 * c]);
            for (int j = 0; j < 3; ++j) lt[3 * c + j] -= tn * rows[c].n[j];
        }
    }
    double (*fr)[6] = malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double[6]));
    learned_features(P, n, x, r, v, w, rows, nc, ln, lt, feat, fr, scale);
    for (int64_t c = 0; c < nc; ++c) for (int k = 0; k < 6; ++k) frame[6 * c + k] = fr[c][k];
    free(fr); free(lt); free(ln); free(rows); free(M.im); free(M.iI);
    return nc;
}

double orc_natural_residual(const orc_params* P,
                            int64_t n, const int64_t* id, const double* r, const double* rho,
                            const double* x, const double* v, const double* w,
                            int32_t nb, const orc_body* bodies,
                            int32_t ns, const orc_shape* shapes,
                            int64_t nc_in, const double* lam)
{
    inv_mass M;
    make_inv_mass(P, n, r, rho, &M);
    raw_contact* rc = NULL;
    int64_t nc = detect_all(P, n, id, x, r, nb, bodies, ns, shapes, &rc);
    if (nc != nc_in) { free(rc); free(M.im); free(M.iI); return -1.0; }
    row* rows = (row*)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(row));
    build_rows(P, id, r, &M, x, v, w, bodies, shapes, rc, nc, rows);
    free(rc);
    double* vv = (double*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    double* ww = (double*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) { vv[3 * i + k] = v[3 * i + k] + P->dt * P->g[k]; ww[3 * i + k] = w[3 * i + k]; }
    for (int64_t c = 0; c < nc; ++c) {
        rows[c].ln = lam[4 * c];
        for (int k = 0; k < 3; ++k) rows[c].lt[k] = lam[4 * c + 1 + k];
        double J[3];
        for (int k = 0; k < 3; ++k) J[k] = rows[c].ln * rows[c].n[k] + rows[c].lt[k];
        apply_impulse(&rows[c], &M, vv, ww, J);
    }
    double num = 0.0, den = 0.0, gdt = P->m.gamma_t / P->dt;
    for (int64_t c = 0; c < nc; ++c) {
        row* R = &rows[c];
        double u[3];
        rel_vel(R, vv, ww, u);
        double un = dot3(R->n, u);
        double ln2 = R->ln - (un + R->Sig * R->ln - R->q) / R->Dn;
        if (ln2 < R->lo) ln2 = R->lo;
        double ut[3] = {u[0] - un * R->n[0], u[1] - un * R->n[1], u[2] - un * R->n[2]};
        double lt2[3];
        for (int k = 0; k < 3; ++k) lt2[k] = R->lt[k] - (ut[k] + gdt * R->lt[k]) / R->Dt;
        double lim = R->mu * fabs(R->ln);
        double mag = sqrt(dot3(lt2, lt2));
        if (mag > lim) { double s = mag > 0.0 ? lim / mag : 0.0; for (int k = 0; k < 3; ++k) lt2[k] *= s; }
        double en = R->ln - ln2, et[3] = {R->lt[0] - lt2[0], R->lt[1] - lt2[1], R->lt[2] - lt2[2]};
        num += R->Dn * en * en + R->Dt * dot3(et, et);
        den += R->Dn * R->ln * R->ln + R->Dt * dot3(R->lt, R->lt);
    }
    free(vv); free(ww); free(rows); free(M.im); free(M.iI);
    if (den > 0.0) return sqrt(num) / sqrt(den);
    return num > 0.0 ? 1.0 : 0.0;
}

/* ------------------------------------------------------------------ */
/* Conversion between resting solid and fluidized mass (the passage on   */
/* converting overlapping soil, Eq. surface)                            */
/* ------------------------------------------------------------------ */
static int grid_ok(const orc_voxel_grid* g);

int32_t orc_surface_heights(const orc_voxel_grid* g, const double* phi, double* h)
{
    if (!grid_ok(g)) return -1;
    const int64_t nxy = (int64_t)g->nx * g->ny;
    for (int64_t c = 0; c < nxy; ++c) {
        h[c] = g->origin[2];
        for (int k = g->nz - 1; k >= 0; --k) {
            double f = phi[(int64_t)k * nxy + c];
            if (f > 0.0) {
                double zc = g->origin[2] + (k + 0.5) * g->l0;  /* the voxel's centre */
                h[c] = zc + (f - 0.5) * g->l0;
                break;
            }
        }
    }
    return 0;
}

/* The z interval of the vertical line through (x, y) inside one wedge; 0 if
 * the line misses it or the wedge has no lower bound there. */
static int wedge_vertical(const orc_wedge* w, double x, double y, double* zlo, double* zhi)
{
    double lo = -INFINITY, hi = INFINITY;
    if (w->n == 0) return 0;
    for (int p = 0; p < w->n; ++p) {
        const double* P = w->planes[p];
        double a = P[2], b = P[3] - P[0] * x - P[1] * y;  /* a z <= b */
        if (a > 0.0) { double z = b / a; if (z < hi) hi = z; }
        else if (a < 0.0) { double z = b / a; if (z > lo) lo = z; }
        else if (b < 0.0) return 0;
    }
    if (!(lo <= hi) || lo == -INFINITY) return 0;
    *zlo = lo;
    *zhi = hi;
    return 1;
}

static int inside_any_wedge(int32_t nw, const orc_wedge* w, const double x[3])
{
    for (int k = 0; k < nw; ++k) {
        if (w[k].n == 0) continue;
        int in = 1;
        for (int p = 0; p < w[k].n && in; ++p)
            if (w[k].planes[p][0] * x[0] + w[k].planes[p][1] * x[1] + w[k].planes[p][2] * x[2] - w[k].planes[p][3] > 0.0)
                in = 0;
        if (in) return 1;
    }
    return 0;
}

double orc_convert_cut(const orc_voxel_grid* g, double rho_b, int32_t n_wedges, const orc_wedge* wedges,
                       double* phi, const double* wc, double* mf)
{
    if (!grid_ok(g) || n_wedges < 0) return -1.0;
    const int64_t nxy = (int64_t)g->nx * g->ny;
    const double V0 = g->l0 * g->l0 * g->l0;
    double total = 0.0;
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            double x = g->origin[0] + (i + 0.5) * g->l0, y = g->origin[1] + (j + 0.5) * g->l0;
            double zcut = INFINITY, lo, hi;
            for (int w = 0; w < n_wedges; ++w)
                if (wedge_vertical(&wedges[w], x, y, &lo, &hi) && lo < zcut) zcut = lo;
            if (zcut == INFINITY) continue;
            for (int k = 0; k < g->nz; ++k) {
                int64_t id = (int64_t)k * nxy + (int64_t)j * g->nx + i;
                double t = (zcut - (g->origin[2] + k * g->l0)) / g->l0;  /* occupancy below the cut */
                if (t < 0.0) t = 0.0;
                if (t > 1.0) t = 1.0;
                if (phi[id] > t) {
                    double dm = wc[id] * rho_b * V0 * (phi[id] - t);
                    mf[id] += dm;
                    total += dm;
                    phi[id] = t;
                }
            }
        }
    return total;
}

double orc_convert_deposit(const orc_voxel_grid* g, double rho_b, double w_dep, int32_t n_wedges,
                           const orc_wedge* wedges, const double* rho_p, double* phi, double* wc, double* mf)
{
    if (!grid_ok(g) || n_wedges < 0 || !(w_dep > 0.0)) return -1.0;
    const int64_t nxy = (int64_t)g->nx * g->ny;
    const double V0 = g->l0 * g->l0 * g->l0;
    double total = 0.0;
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            const int64_t c = (int64_t)j * g->nx + i;
            for (int k = 0; k < g->nz; ++k) {
                const int64_t src = (int64_t)k * nxy + c;
                double x[3] = {g->origin[0] + (i + 0.5) * g->l0, g->origin[1] + (j + 0.5) * g->l0,
                               g->origin[2] + (k + 0.5) * g->l0};
                if (!(mf[src] > 0.0) || rho_p[src] != 0.0 || inside_any_wedge(n_wedges, wedges, x)) continue;
                double m = mf[src];
                mf[src] = 0.0;
                /* the first voxel of the column that is not full */
                int kk = 0;
                while (kk < g->nz && phi[(int64_t)kk * nxy + c] >= 1.0) ++kk;
                while (m > 0.0 && kk < g->nz) {
                    const int64_t id = (int64_t)kk * nxy + c;
                    double cap = (1.0 - phi[id]) * w_dep * rho_b * V0;
                    double take = m < cap ? m : cap;
                    double f = take == cap ? 1.0 : phi[id] + take / (w_dep * rho_b * V0);
                    double before = wc[id] * rho_b * V0 * phi[id];
                    wc[id] = phi[id] > 0.0 ? (before + take) / (rho_b * V0 * f) : w_dep;
                    phi[id] = f;
                    total += take;
                    m -= take;
                    ++kk;
                }
                mf[src] += m;  /* a full column: the rest stays fluid */
            }
        }
    return total;
}

static int64_t voxel_of(const orc_voxel_grid* g, const double* x)
{
    const int dims[3] = {g->nx, g->ny, g->nz};
    int c[3];
    for (int k = 0; k < 3; ++k) {
        double f = floor((x[k] - g->origin[k]) / g->l0);
        if (!(f >= 0.0 && f < (double)dims[k])) return -1;
        c[k] = (int)f;
    }
    return ((int64_t)c[2] * g->ny + c[1]) * g->nx + c[0];
}

double orc_grow_particles(int64_t n, const double* x, double* r, double rho, const orc_voxel_grid* g, double dt,
                          double dprime_max, double d_max, double* mf)
{
    if (!grid_ok(g) || !(rho > 0.0) || !(dt >= 0.0) || !(dprime_max >= 0.0) || !(d_max > 0.0)) return -1.0;
    const int64_t nv = (int64_t)g->nx * g->ny * g->nz;
    double* cap_sum = (double*)calloc((size_t)nv, sizeof(double));
    double* cap = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    const double k_m = rho * (4.0 / 3.0) * PI;  /* m = k_m r^3 */
    const double m_max = k_m * (0.5 * d_max) * (0.5 * d_max) * (0.5 * d_max);
    /* each particle's bound over dt, summed per voxel */
    for (int64_t a = 0; a < n; ++a) {
        cap[a] = 0.0;
        int64_t v = voxel_of(g, &x[3 * a]);
        if (v < 0) continue;
        double m = k_m * r[a] * r[a] * r[a];
        double c = 3.0 * m * dprime_max * dt / (2.0 * r[a]);
        if (m + c > m_max) c = m_max > m ? m_max - m : 0.0;
        cap[a] = c;
        cap_sum[v] += c;
    }
    double total = 0.0;
    double* used = (double*)calloc((size_t)nv, sizeof(double));
    for (int64_t a = 0; a < n; ++a) {
        if (cap[a] <= 0.0) continue;
        int64_t v = voxel_of(g, &x[3 * a]);
        double A = mf[v] > 0.0 ? mf[v] : 0.0;
        double share = cap_sum[v] <= A ? cap[a] : cap[a] * (A / cap_sum[v]);
        if (!(share > 0.0)) continue;  /* a particle that gains nothing keeps its radius */
        double m = k_m * r[a] * r[a] * r[a];
        r[a] = cbrt((m + share) / k_m);
        used[v] += share;
        total += share;
    }
    for (int64_t v = 0; v < nv; ++v) mf[v] -= used[v];
    free(cap_sum); free(cap); free(used);
    return total;
}

int64_t orc_form_particles(const orc_voxel_grid* g, double rho, double d_min, double d_max, double phi_max,
                           int32_t n_wedges, const orc_wedge* wedges, const double* rho_p, const double* u,
                           double* mf, int64_t cap, int64_t* voxel, double* x, double* v, double* r)
{
    if (!grid_ok(g) || !(rho > 0.0) || !(d_min > 0.0) || !(d_max >= d_min) || !(phi_max > 0.0) || n_wedges < 0)
        return -1;
    const int64_t nxy = (int64_t)g->nx * g->ny;
    const double V0 = g->l0 * g->l0 * g->l0;
    const double k_m = rho * PI / 6.0;  /* m = k_m d^3 */
    const double m_min = k_m * d_min * d_min * d_min;
    int64_t n = 0;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                const int64_t id = (int64_t)k * nxy + (int64_t)j * g->nx + i;
                if (!(mf[id] >= m_min)) continue;
                double c[3] = {g->origin[0] + (i + 0.5) * g->l0, g->origin[1] + (j + 0.5) * g->l0,
                               g->origin[2] + (k + 0.5) * g->l0};
                if (!inside_any_wedge(n_wedges, wedges, c)) continue;
                double d = cbrt(mf[id] / k_m);
                if (d > d_max) d = d_max;
                double m = k_m * d * d * d;
                /* room for the new particle: particle volume fraction after it */
                if (rho_p[id] / rho + m / (rho * V0) > phi_max) continue;
                mf[id] -= m;
                if (n < cap) {
                    voxel[n] = id;
                    for (int q = 0; q < 3; ++q) { x[3 * n + q] = c[q]; v[3 * n + q] = u[3 * id + q]; }
                    r[n] = 0.5 * d;
                }
                ++n;
            }
    return n;
}

double orc_settle_particles(int64_t n, const double* x, const double* v, const double* m, const orc_voxel_grid* g,
                            double v_rest, int32_t n_wedges, const orc_wedge* wedges, double* mf, int32_t* gone)
{
    if (!grid_ok(g) || !(v_rest >= 0.0) || n_wedges < 0) return -1.0;
    double total = 0.0;
    for (int64_t a = 0; a < n; ++a) {
        gone[a] = 0;
        const double* va = &v[3 * a];
        if (!(sqrt(dot3(va, va)) < v_rest)) continue;
        int64_t vox = voxel_of(g, &x[3 * a]);
        if (vox < 0 || inside_any_wedge(n_wedges, wedges, &x[3 * a])) continue;
        mf[vox] += m[a];
        total += m[a];
        gone[a] = 1;
    }
    return total;
}

/* Eq. failure_plane: theta(phi, beta) = pi/2 - (phi + beta)/2. */
double orc_failure_angle(double phi, double beta) { return 0.5 * PI - 0.5 * (phi + beta); }

/* ------------------------------------------------------------------ */
/* Mesoscale fields on voxels: coarse-graining (Eq. cg_velocity) and the */
/* conserved advection of fluidized mass (Eq. advection)                 */
/* ------------------------------------------------------------------ */
static int grid_ok(const orc_voxel_grid* g)
{
    return g && g->l0 > 0.0 && g->nx > 0 && g->ny > 0 && g->nz > 0;
}

int32_t orc_coarse_grain(int64_t n, const double* x, const double* v, const double* m, const orc_voxel_grid* g,
                         int32_t kernel, double R, double* rho, double* mom, double* u)
{
    if (!grid_ok(g) || (kernel != ORC_CG_HEAVISIDE && kernel != ORC_CG_GAUSS) ||
        (kernel == ORC_CG_GAUSS && !(R > 0.0)))
        return -1;
    const int64_t nv = (int64_t)g->nx * g->ny * g->nz;
    const double V0 = g->l0 * g->l0 * g->l0;
    for (int64_t i = 0; i < nv; ++i) {
        rho[i] = 0.0;
        for (int k = 0; k < 3; ++k) mom[3 * i + k] = 0.0;
    }
    const int dims[3] = {g->nx, g->ny, g->nz};
    for (int64_t a = 0; a < n; ++a) {
        const double* xa = &x[3 * a];
        if (kernel == ORC_CG_HEAVISIDE) {
            int c[3], in = 1;
            for (int k = 0; k < 3; ++k) {
                double f = floor((xa[k] - g->origin[k]) / g->l0);
                if (!(f >= 0.0 && f < (double)dims[k])) in = 0;
                c[k] = in ? (int)f : 0;
            }
            if (!in) continue;
            int64_t id = ((int64_t)c[2] * g->ny + c[1]) * g->nx + c[0];
            rho[id] += m[a] / V0;
            for (int k = 0; k < 3; ++k) mom[3 * id + k] += m[a] * v[3 * a + k] / V0;
        } else {
            const double norm = 1.0 / ((sqrt(2.0 * PI) * R) * (sqrt(2.0 * PI) * R) * (sqrt(2.0 * PI) * R));
            int lo[3], hi[3];
            for (int k = 0; k < 3; ++k) {
                /* voxel centres within 3R of the particle */
                double fl = ceil((xa[k] - 3.0 * R - g->origin[k]) / g->l0 - 0.5);
                double fh = floor((xa[k] + 3.0 * R - g->origin[k]) / g->l0 - 0.5);
                lo[k] = fl < 0.0 ? 0 : (int)fl;
                hi[k] = fh > (double)(dims[k] - 1) ? dims[k] - 1 : (int)fh;
            }
            for (int kz = lo[2]; kz <= hi[2]; ++kz)
                for (int jy = lo[1]; jy <= hi[1]; ++jy)
                    for (int ix = lo[0]; ix <= hi[0]; ++ix) {
                        double y[3] = {g->origin[0] + (ix + 0.5) * g->l0 - xa[0],
                                       g->origin[1] + (jy + 0.5) * g->l0 - xa[1],
                                       g->origin[2] + (kz + 0.5) * g->l0 - xa[2]};
                        double r2 = dot3(y, y);
                        if (r2 > 9.0 * R * R) continue;
                        double z = norm * exp(-r2 / (2.0 * R * R));
                        int64_t id = ((int64_t)kz * g->ny + jy) * g->nx + ix;
                        rho[id] += m[a] * z;
                        for (int k = 0; k < 3; ++k) mom[3 * id + k] += m[a] * v[3 * a + k] * z;
                    }
        }
    }
    if (u)
        for (int64_t i = 0; i < nv; ++i)
            for (int k = 0; k < 3; ++k) u[3 * i + k] = rho[i] > 0.0 ? mom[3 * i + k] / rho[i] : 0.0;
    return 0;
}

double orc_advect(const orc_voxel_grid* g, double dt, const double* u, double* mf)
{
    if (!grid_ok(g)) return -1.0;
    const int64_t nv = (int64_t)g->nx * g->ny * g->nz;
    const int dims[3] = {g->nx, g->ny, g->nz};
    const int64_t strides[3] = {1, g->nx, (int64_t)g->nx * g->ny};
    double* out = (double*)malloc((size_t)nv * sizeof(double));
    double cfl = 0.0;
    for (int64_t i = 0; i < nv; ++i) out[i] = mf[i];
    /* every interior face once: the flux leaves the donor and enters the other voxel */
    for (int64_t i = 0; i < nv; ++i) {
        int64_t c[3] = {i % g->nx, (i / g->nx) % g->ny, i / ((int64_t)g->nx * g->ny)};
        for (int d = 0; d < 3; ++d) {
            if (c[d] + 1 >= dims[d]) continue;  /* closed outer face */
            int64_t j = i + strides[d];
            double uf = 0.5 * (u[3 * i + d] + u[3 * j + d]);
            double a = fabs(uf) * dt / g->l0;
            if (a > cfl) cfl = a;
            double phi = uf > 0.0 ? dt * uf * mf[i] / g->l0 : dt * uf * mf[j] / g->l0;  /* + : i -> j */
            out[i] -= phi;
            out[j] += phi;
        }
    }
    for (int64_t i = 0; i < nv; ++i) mf[i] = out[i];
    free(out);
    return cfl;
}

/* ------------------------------------------------------------------ */
/* Macroscale model (section "Macroscale model"): the aggregate body A   */
/* of a zone under Eq. mdb:eqAgg with the velocity constraints of Eqs.  */
/* aggregateNormal and aggregateTangent at its interfaces to the        */
/* equipment (AB) and the failure surface (AC), four points each.       */
/* ------------------------------------------------------------------ */

/* World-frame half-space p of body b: normal nw, offset dw (inside: nw.x <= dw). */
static void zone_plane_world(const orc_body* B, int p, double nw[3], double* dw)
{
    double Rm[3][3];
    quat_matrix(B->quat, Rm);
    const double* pl = B->planes[p];
    for (int k = 0; k < 3; ++k) nw[k] = (Rm[k][0] * pl[0] + Rm[k][1] * pl[1]) + Rm[k][2] * pl[2];
    *dw = pl[3] + dot3(nw, B->pos);
}

/* In-plane axes of a plane with unit normal n: e1 the normalised projection
 * of the world axis least aligned with n (the lower axis on ties), e2 = n x e1. */
static void plane_axes(const double n[3], double e1[3], double e2[3])
{
    int k0 = 0;
    for (int k = 1; k < 3; ++k) if (fabs(n[k]) < fabs(n[k0])) k0 = k;
    double a[3] = {0.0, 0.0, 0.0};
    a[k0] = 1.0;
    double an = dot3(a, n);
    for (int k = 0; k < 3; ++k) e1[k] = a[k] - an * n[k];
    double m = sqrt(dot3(e1, e1));
    for (int k = 0; k < 3; ++k) e1[k] /= m;
    cross3(n, e1, e2);
}

int32_t orc_reduce4(int64_t n, const double* pts, const double nrm[3], int64_t idx[4])
{
    if (n <= 0) return 0;
    double e1[3], e2[3];
    plane_axes(nrm, e1, e2);
    int64_t best[4] = {0, 0, 0, 0};
    double bv[4];
    for (int64_t i = 0; i < n; ++i) {
        double s1 = dot3(&pts[3 * i], e1), s2 = dot3(&pts[3 * i], e2);
        double val[4] = {s1, -s1, s2, -s2};
        for (int d = 0; d < 4; ++d)
            if (i == 0 || val[d] > bv[d]) { bv[d] = val[d]; best[d] = i; }  /* strict: ties keep the smaller index */
    }
    int32_t m = 0;
    for (int d = 0; d < 4; ++d) {
        int dup = 0;
        for (int q = 0; q < m; ++q) dup |= idx[q] == best[d];
        if (!dup) idx[m++] = best[d];
    }
    return m;
}

/* Inverse of a symmetric 3x3 matrix by cofactors. */
static void inv3(const double A[3][3], double B[3][3])
{
    double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    B[0][0] = c00 / det;
    B[1][0] = c01 / det;
    B[2][0] = c02 / det;
    B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

static void mat3_vec(const double A[3][3], const double x[3], double y[3])
{
    for (int k = 0; k < 3; ++k) y[k] = (A[k][0] * x[0] + A[k][1] * x[1]) + A[k][2] * x[2];
}

/* Velocity change of the point at arm rr per unit impulse along a, projected
 * on b: (1/M) a.b + (rr x a) . Iinv (rr x b). */
static double point_w(double invM, const double Iinv[3][3], const double rr[3], const double a[3], const double b[3])
{
    double ra[3], rb[3], t[3];
    cross3(rr, a, ra);
    cross3(rr, b, rb);
    mat3_vec(Iinv, rb, t);
    return invM * dot3(a, b) + dot3(ra, t);
}

int32_t orc_macro_step(const orc_params* P, int64_t n, const double* r, const double* rho,
                       const double* x, const double* v, const double* w,
                       int32_t nb, const orc_body* bodies, int32_t ns, const orc_shape* shapes,
                       const orc_macro_params* mp, int32_t neq, const orc_macro_equipment* eq,
                       int32_t cap, orc_macro_out* out)
{
    const double dt = P->dt;
    double* inv_m = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t i = 0; i < n; ++i) inv_m[i] = 1.0 / particle_mass(P, rho, i, r);
    orc_aggregate* agg = (orc_aggregate*)calloc((size_t)(nb > 0 ? nb : 1), sizeof(orc_aggregate));
    int32_t na = orc_aggregates(n, r, inv_m, x, v, w, nb, bodies, agg);
    /* zone membership: the first body (in order) whose half-spaces all contain x */
    int32_t* zone_of = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        zone_of[i] = -1;
        for (int32_t b = 0; b < nb && zone_of[i] < 0; ++b) {
            if (bodies[b].nplanes <= 0) continue;
            int in = 1;
            for (int p = 0; p < bodies[b].nplanes && in; ++p) {
                double nw[3], dw;
                zone_plane_world(&bodies[b], p, nw, &dw);
                if (dot3(nw, &x[3 * i]) - dw > 0.0) in = 0;
            }
            if (in) zone_of[i] = b;
        }
    }
    double* cand = (double*)malloc((size_t)(2 * n + 1) * 3 * sizeof(double));
    int64_t* csrc = (int64_t*)malloc((size_t)(2 * n + 1) * sizeof(int64_t));
    int32_t nout = 0;
    for (int32_t ai = 0; ai < na && nout < cap; ++ai) {
        const orc_aggregate* A = &agg[ai];
        const int32_t b = A->zone;
        const orc_body* B = &bodies[b];
        if (B->nplanes < 2 || A->M <= 0.0) continue;
        orc_macro_out* o = &out[nout++];
        memset(o, 0, sizeof(*o));
        o->zone = b;
        o->M = A->M;
        for (int k = 0; k < 3; ++k) { o->x[k] = A->x[k]; o->v0[k] = A->v[k]; o->w0[k] = A->w[k]; }
        double I[3][3] = {{A->I[0], A->I[3], A->I[4]}, {A->I[3], A->I[1], A->I[5]}, {A->I[4], A->I[5], A->I[2]}};
        double Iinv[3][3];
        inv3(I, Iinv);
        const double invM = 1.0 / A->M;
        /* the aggregate's length scale: cube root of its solid volume */
        double vol = 0.0;
        for (int64_t i = 0; i < n; ++i)
            if (zone_of[i] == b) vol += (4.0 / 3.0) * PI * r[i] * r[i] * r[i];
        const double L = cbrt(vol);
        double nsep[3], dsep, nfail[3], dfail;
        zone_plane_world(B, 0, nsep, &dsep);
        zone_plane_world(B, 1, nfail, &dfail);
        for (int q = 0; q < 2; ++q) {
            /* interface normals point from B or C into A: against the zone's
             * outward normals of the separation plate and the failure plane */
            double nI[3];
            for (int k = 0; k < 3; ++k) nI[k] = -(q == 0 ? nsep[k] : nfail[k]);
            int64_t nc = 0;
            double area = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                if (zone_of[i] != b) continue;
                if (q == 0) {
                    for (int32_t s = 0; s < ns; ++s) {
                        if (shapes[s].body != b) continue;
                        double delta, nrm[3];
                        if (!shape_touch(P, &shapes[s], bodies, &x[3 * i], r[i], &delta, nrm)) continue;
                        double l2 = r[i] - 0.5 * delta;
                        for (int k = 0; k < 3; ++k) cand[3 * nc + k] = x[3 * i + k] - l2 * nrm[k];
                        csrc[nc++] = i;
                        area += PI * r[i] * r[i];
                    }
                } else {
                    double d = dot3(nfail, &x[3 * i]) - dfail;  /* <= 0 inside the zone */
                    if (!(d >= -r[i])) continue;
                    for (int k = 0; k < 3; ++k) cand[3 * nc + k] = x[3 * i + k] - d * nfail[k];
                    csrc[nc++] = i;
                    area += PI * r[i] * r[i];
                }
            }
            o->n_cand[q] = nc;
            o->area[q] = area;
            int64_t idx[4];
            int32_t m = orc_reduce4(nc, cand, nI, idx);
            o->n_points[q] = m;
            o->gamma[q] = area > 0.0 ? L / ((q == 0 ? mp->cas_ab : mp->cas_ac) * mp->E_b * area * dt * dt) : 0.0;
            for (int j = 0; j < m; ++j) {
                for (int k = 0; k < 3; ++k) { o->p[4 * q + j][k] = cand[3 * idx[j] + k]; o->n[4 * q + j][k] = nI[k]; }
                o->src[4 * q + j] = csrc[idx[j]];
            }
        }
        /* Eq. mdb:eqAgg in impulse form: M (v+ - v) = dt M g + sum G^T lambda,
         * I (w+ - w) = sum (p - x_A) x (G^T lambda); each point's normal row
         * gamma lambda_n + n.u >= 0 with lambda_n >= -c_b A dt / points, its
         * tangential rows gamma lambda_t + u_t = 0 on the disk
         * |lambda_t| <= mu |lambda_n|, u the velocity of A at the point minus
         * that of B (or 0 on the terrain).  With the equipment dynamic (Eq.
         * mdb:eqEq) B is a second body: M_B (v_B+ - v_B) = dt M_B g -
         * sum_AB G^T lambda + lambda_d, I_B (w_B+ - w_B) = -sum_AB (p - x_B) x
         * (G^T lambda) + tau_d, with the drive's rows gamma_d lambda_d +
         * (v_B - v_target) = 0 per world axis (linear, then angular),
         * |lambda_d| <= f_max dt (t_max dt).  Projected Gauss-Seidel, normal
         * then tangential rows of each point in turn (AB, then AC), then the
         * drive rows, until no impulse changes. */
        const orc_macro_equipment* E = NULL;
        for (int32_t k = 0; k < neq; ++k)
            if (eq[k].body == b) E = &eq[k];
        double vv[3], ww[3], vB[3], wB[3], IBinv[3][3], invMB = 0.0, ld[6] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < 3; ++k) { vv[k] = A->v[k] + dt * P->g[k]; ww[k] = A->w[k]; }
        memset(IBinv, 0, sizeof(IBinv));
        if (E) {
            invMB = 1.0 / E->mass;
            double Rm[3][3], Iw[3][3];
            quat_matrix(B->quat, Rm);
            const double* J6 = E->inertia;
            double Ib[3][3] = {{J6[0], J6[3], J6[4]}, {J6[3], J6[1], J6[5]}, {J6[4], J6[5], J6[2]}};
            for (int p = 0; p < 3; ++p)          /* world inertia R I R^T */
                for (int q = 0; q < 3; ++q) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k)
                        for (int l = 0; l < 3; ++l) acc += Rm[p][k] * Ib[k][l] * Rm[q][l];
                    Iw[p][q] = acc;
                }
            inv3(Iw, IBinv);
            for (int k = 0; k < 3; ++k) { vB[k] = B->linvel[k] + dt * P->g[k]; wB[k] = B->angvel[k]; }
        } else {
            for (int k = 0; k < 3; ++k) { vB[k] = B->linvel[k]; wB[k] = B->angvel[k]; }
        }
        int np = 0;
        int map[8];
        for (int q = 0; q < 2; ++q)
            for (int j = 0; j < o->n_points[q]; ++j) map[np++] = 4 * q + j;
        double rr[8][3], rb[8][3], uo[8][3], Wn[8], Wt[8], lo[8], mu[8], gam[8], t1[8][3], t2[8][3];
        int onB[8];
        for (int c = 0; c < np; ++c) {
            int k8 = map[c], q = k8 / 4;
            onB[c] = q == 0 && E != NULL;
            for (int k = 0; k < 3; ++k) { rr[c][k] = o->p[k8][k] - A->x[k]; rb[c][k] = o->p[k8][k] - B->pos[k]; }
            for (int k = 0; k < 3; ++k) uo[c][k] = 0.0;
            if (q == 0 && !E) {
                double t[3];
                cross3(B->angvel, rb[c], t);
                for (int k = 0; k < 3; ++k) uo[c][k] = B->linvel[k] + t[k];
            }
            plane_axes(o->n[k8], t1[c], t2[c]);
            Wn[c] = point_w(invM, Iinv, rr[c], o->n[k8], o->n[k8]);
            /* one scalar for both tangential rows (the disk's fixed point does
             * not depend on it): their mean effective inverse mass */
            Wt[c] = 0.5 * (point_w(invM, Iinv, rr[c], t1[c], t1[c]) + point_w(invM, Iinv, rr[c], t2[c], t2[c]));
            if (onB[c]) {
                Wn[c] += point_w(invMB, (const double(*)[3])IBinv, rb[c], o->n[k8], o->n[k8]);
                Wt[c] += 0.5 * (point_w(invMB, (const double(*)[3])IBinv, rb[c], t1[c], t1[c]) +
                                point_w(invMB, (const double(*)[3])IBinv, rb[c], t2[c], t2[c]));
            }
            lo[c] = -mp->c_b * o->area[q] * dt / (double)o->n_points[q];
            mu[c] = q == 0 ? mp->mu_ab : mp->mu_ac;
            gam[c] = o->gamma[q];
        }
        double lam[8][4];
        memset(lam, 0, sizeof(lam));
        int sweep = 0;
        for (; sweep < 200000; ++sweep) {
            double dmax = 0.0, lmax = 0.0;
            for (int c = 0; c < np; ++c) {
                const double* nn = o->n[map[c]];
                for (int row = 0; row < 2; ++row) {
                    double u[3], t[3];
                    cross3(ww, rr[c], t);
                    for (int k = 0; k < 3; ++k) u[k] = vv[k] + t[k] - uo[c][k];
                    if (onB[c]) {
                        cross3(wB, rb[c], t);
                        for (int k = 0; k < 3; ++k) u[k] -= vB[k] + t[k];
                    }
                    double J[3];
                    if (row == 0) {
                        double un = dot3(nn, u);
                        double ln = lam[c][0] - (un + gam[c] * lam[c][0]) / (Wn[c] + gam[c]);
                        if (ln < lo[c]) ln = lo[c];
                        double d = ln - lam[c][0];
                        lam[c][0] = ln;
                        for (int k = 0; k < 3; ++k) J[k] = d * nn[k];
                        if (fabs(d) > dmax) dmax = fabs(d);
                    } else {
                        double un = dot3(nn, u);
                        double lt[3];
                        for (int k = 0; k < 3; ++k) {
                            double ut = u[k] - un * nn[k];
                            lt[k] = lam[c][1 + k] - (ut + gam[c] * lam[c][1 + k]) / (Wt[c] + gam[c]);
                        }
                        double ltn = dot3(lt, nn);
                        for (int k = 0; k < 3; ++k) lt[k] -= ltn * nn[k];
                        double lim = mu[c] * fabs(lam[c][0]);
                        double m2 = sqrt(dot3(lt, lt));
                        if (m2 > lim) {
                            double s = m2 > 0.0 ? lim / m2 : 0.0;
                            for (int k = 0; k < 3; ++k) lt[k] *= s;
                        }
                        for (int k = 0; k < 3; ++k) {
                            J[k] = lt[k] - lam[c][1 + k];
                            if (fabs(J[k]) > dmax) dmax = fabs(J[k]);
                            lam[c][1 + k] = lt[k];
                        }
                    }
                    double tj[3], dw[3];
                    cross3(rr[c], J, tj);
                    mat3_vec(Iinv, tj, dw);
                    for (int k = 0; k < 3; ++k) { vv[k] += invM * J[k]; ww[k] += dw[k]; }
                    if (onB[c]) {
                        cross3(rb[c], J, tj);
                        mat3_vec((const double(*)[3])IBinv, tj, dw);
                        for (int k = 0; k < 3; ++k) { vB[k] -= invMB * J[k]; wB[k] -= dw[k]; }
                    }
                }
                for (int k = 0; k < 4; ++k) if (fabs(lam[c][k]) > lmax) lmax = fabs(lam[c][k]);
            }
            if (E) {
                for (int k = 0; k < 6; ++k) {
                    const int ax = k % 3;
                    const double u = k < 3 ? vB[ax] - E->v_target[ax] : wB[ax] - E->w_target[ax];
                    const double W = k < 3 ? invMB : IBinv[ax][ax];
                    const double lim = (k < 3 ? E->f_max : E->t_max) * dt;
                    double l = ld[k] - (u + E->gamma_drive * ld[k]) / (W + E->gamma_drive);
                    if (l > lim) l = lim;
                    if (l < -lim) l = -lim;
                    const double d = l - ld[k];
                    ld[k] = l;
                    if (k < 3) vB[ax] += invMB * d;
                    else for (int j = 0; j < 3; ++j) wB[j] += IBinv[j][ax] * d;
                    if (fabs(d) > dmax) dmax = fabs(d);
                    if (fabs(l) > lmax) lmax = fabs(l);
                }
            }
            if (dmax <= 1e-15 * lmax || lmax == 0.0) { ++sweep; break; }
        }
        o->sweeps = sweep;
        for (int k = 0; k < 3; ++k) {
            o->v[k] = vv[k]; o->w[k] = ww[k]; o->force_b[k] = 0.0; o->torque_b[k] = 0.0;
            o->v_b[k] = vB[k]; o->w_b[k] = wB[k];
        }
        for (int k = 0; k < 6; ++k) o->lam_drive[k] = ld[k];
        for (int c = 0; c < np; ++c) {
            int k8 = map[c];
            for (int k = 0; k < 4; ++k) o->lam[k8][k] = lam[c][k];
            if (k8 >= 4) continue;
            double J[3], t[3];
            for (int k = 0; k < 3; ++k) J[k] = lam[c][0] * o->n[k8][k] + lam[c][1 + k];
            for (int k = 0; k < 3; ++k) o->force_b[k] -= J[k] / dt;
            cross3(rb[c], J, t);
            for (int k = 0; k < 3; ++k) o->torque_b[k] -= t[k] / dt;
        }
    }
    free(cand); free(csrc); free(zone_of); free(agg); free(inv_m);
    return nout;
}
