/*
 * Non-sequential Monte Carlo polarization ray trace through a geometric
 * waveguide, its adjoint, and brute-force deterministic splitting.
 * Test infrastructure (oracle); see oracle.h.
 *
 * Follows the paper's Methods:
 *   - "Polarization ray tracing" (Eq. 5): at every coated interface the complex
 *     field vector is projected on the local s and p unit vectors, scaled by the
 *     effective coefficients, and re-assembled on the outgoing basis; the basis
 *     is recomputed at every interface;
 *   - "Differentiable Monte Carlo non-sequential ray tracing" (Eq. 6): at each
 *     partially reflective mirror one branch is sampled with the mirror's
 *     reflection probability omega and the field is divided by sqrt(omega) or
 *     sqrt(1 - omega); the choice depends only on the random number and omega,
 *     never on the coefficients, so the path is independent of the layer
 *     thicknesses and the gradient is the pathwise derivative;
 *   - the eyebox intensity is the incoherent sum of |E|^2 over rays.
 *
 * Geometry (a synthetic stand-in; the paper's exact layout is not given):
 * slab 0 <= z <= T, 0 <= x <= Lx, unbounded in y; M planar mirrors across the
 * full thickness with common normal n = (-sin b, 0, cos b) through
 * (x_m, ., T/2); the cells between mirrors are convex and a ray leaves its
 * cell through the nearest of its four bounding planes.  Slab faces are bare
 * glass/air interfaces (Eq. 3): total internal reflection keeps the ray;
 * otherwise the top face emits it towards the eyebox (its Fresnel-reflected
 * part is dropped and tallied), the bottom face loses it.  End faces absorb.
 *
 * The geometric operations below are written in a fixed order with no fused
 * multiply-add so that a second implementation performing the same IEEE
 * operations reproduces every path decision bit for bit.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

void orc__tmm_coeffs(int L, const double* thk, const double* nre, const double* nim,
                     double n_glass, double lambda_nm, double kappa, double complex c[4]);

enum { SURF_TOP = 1000, SURF_BOTTOM = 1001, SURF_END0 = 1002, SURF_END1 = 1003 };
enum { EV_TIR = 1, EV_EXIT = 2, EV_LEAK = 3, EV_END = 4, EV_MIRROR = 5 };

typedef struct { double x, y, z; } vec3;
typedef struct { double complex x, y, z; } cvec3;

static double dot3(vec3 a, vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static vec3 cross3(vec3 a, vec3 b)
{
    vec3 r = { a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x };
    return r;
}
static vec3 scale3(vec3 a, double s) { vec3 r = { a.x * s, a.y * s, a.z * s }; return r; }
static double complex cdot3(cvec3 e, vec3 u) { return e.x * u.x + e.y * u.y + e.z * u.z; }
static double norm2c(cvec3 e)
{
    double ax = creal(e.x) * creal(e.x) + cimag(e.x) * cimag(e.x);
    double ay = creal(e.y) * creal(e.y) + cimag(e.y) * cimag(e.y);
    double az = creal(e.z) * creal(e.z) + cimag(e.z) * cimag(e.z);
    return (ax + ay) + az;
}

static double u24(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

/* ------------------------------------------------------------ scene setup */
typedef struct {
    const orc_scene* sc;
    double nx, nz;          /* mirror normal (-sin b, 0, cos b) */
    double* h;              /* plane offsets n . c_m */
    uint32_t* thr;          /* reflect iff word < thr */
    double* p_eff;          /* thr / 2^32 */
    uint32_t key[2];
    int64_t id_base;        /* added to a ray's id in its random stream */
    /* per point */
    int d, li, f, lam;
    double ng, na, lambda_nm;
    /* per mirror stacks in incidence order: [M][2 sides][Lmax] */
    double* s_thk;
    double* s_nre;
    double* s_nim;
    int* s_len;
} ctx_t;

static int ctx_init(ctx_t* c, const orc_scene* sc)
{
    memset(c, 0, sizeof(*c));
    c->sc = sc;
    double beta = sc->tilt_deg * (M_PI / 180.0);
    c->nx = -sin(beta);
    c->nz = cos(beta);
    int M = sc->n_mirrors;
    c->h = (double*)malloc(sizeof(double) * (size_t)M);
    c->thr = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)M);
    c->p_eff = (double*)malloc(sizeof(double) * (size_t)M);
    for (int m = 0; m < M; ++m) {
        double xm = sc->center_x + ((double)m - (double)(M - 1) * 0.5) * sc->pitch;
        c->h[m] = c->nx * xm + c->nz * (sc->T * 0.5);
        double t = floor(sc->omega[m] * 4294967296.0);
        if (t > 4294967295.0) t = 4294967295.0;
        if (t < 0.0) t = 0.0;
        c->thr[m] = (uint32_t)t;
        c->p_eff[m] = (double)c->thr[m] / 4294967296.0;
    }
    c->id_base = (int64_t)sc->first_design * sc->n_lsel * (sc->fov_mode == 1 ? 1 : sc->n_fov) * sc->rays_per_point;
    c->key[0] = (uint32_t)sc->seed;
    c->key[1] = (uint32_t)(sc->seed >> 32) ^ (uint32_t)sc->step;
    size_t n = (size_t)M * 2 * (size_t)(sc->max_layers > 0 ? sc->max_layers : 1);
    c->s_thk = (double*)malloc(sizeof(double) * n);
    c->s_nre = (double*)malloc(sizeof(double) * n);
    c->s_nim = (double*)malloc(sizeof(double) * n);
    c->s_len = (int*)malloc(sizeof(int) * (size_t)M);
    return (c->h && c->thr && c->p_eff && c->s_thk && c->s_nre && c->s_nim && c->s_len) ? 0 : -1;
}

static void ctx_free(ctx_t* c)
{
    free(c->h); free(c->thr); free(c->p_eff);
    free(c->s_thk); free(c->s_nre); free(c->s_nim); free(c->s_len);
}

/* Select point (design d, selected wavelength li, fov f): glass index and the
 * per-mirror stacks in both incidence orders.  Layer 0 faces the +n side, so
 * a hit from that side (front) sees layers 0..L-1 and a back hit the reverse. */
static void ctx_point(ctx_t* c, int d, int li, int f)
{
    const orc_scene* sc = c->sc;
    c->d = d; c->li = li; c->f = f;
    c->lam = sc->lambda_sel[li];
    const double* nre = sc->n_re + (size_t)c->lam * sc->n_mat;
    const double* nim = sc->n_im + (size_t)c->lam * sc->n_mat;
    c->ng = nre[sc->mat_glass];
    c->na = nre[sc->mat_air];
    c->lambda_nm = sc->lambda_nm[c->lam];
    int Lm = sc->max_layers;
    for (int m = 0; m < sc->n_mirrors; ++m) {
        int L = sc->n_layers[d * sc->n_mirrors + m];
        c->s_len[m] = L;
        const double* thk = sc->thk + ((size_t)d * sc->n_mirrors + m) * Lm;
        const uint8_t* mat = sc->mat + ((size_t)d * sc->n_mirrors + m) * Lm;
        for (int side = 0; side < 2; ++side) {
            size_t base = ((size_t)m * 2 + side) * Lm;
            for (int j = 0; j < L; ++j) {
                int src = side == 0 ? j : L - 1 - j;
                c->s_thk[base + j] = thk[src];
                c->s_nre[base + j] = nre[mat[src]];
                c->s_nim[base + j] = nim[mat[src]];
            }
        }
    }
}

/* ------------------------------------------------------------- ray state */
typedef struct {
    vec3 p, d;
    cvec3 E;
    int cell, last;
    int n_events, n_prma;
    /* Philox cache for event words */
    uint32_t words[4];
    int64_t ray_id;
} ray_t;

/* Tape entry of one field-changing event (for the adjoint). */
typedef struct {
    int type;
    int mirror, front, reflect;
    double kappa;
    vec3 s, pin, pout;
    double complex cs, cp;
    double scale;
    cvec3 E_before;
} tape_t;

static void philox_words(const ctx_t* c, int64_t ray_id, uint32_t block, uint32_t tag, uint32_t out[4])
{
    const int64_t gid = ray_id + c->id_base;
    uint32_t ctr[4] = { (uint32_t)(uint64_t)gid, (uint32_t)((uint64_t)gid >> 32), block, tag };
    orc_philox4x32_10(ctr, c->key, out);
}

/* Birth (injection) of ray ray_id at the current point. */
static void ray_birth(const ctx_t* c, int64_t ray_id, ray_t* r)
{
    const orc_scene* sc = c->sc;
    uint32_t w[4];
    philox_words(c, ray_id, 0u, 0u, w);
    memset(r, 0, sizeof(*r));
    r->ray_id = ray_id;
    r->p.x = sc->pupil_x0 + u24(w[0]) * sc->pupil_w;
    r->p.y = u24(w[1]) * sc->pupil_h - 0.5 * sc->pupil_h;
    r->p.z = sc->T;
    double thx, thy;
    if (sc->fov_mode == 1) {
        const double* b = sc->fov_deg;
        thx = b[0] + u24(w[2]) * (b[1] - b[0]);
        thy = b[2] + u24(w[3]) * (b[3] - b[2]);
    } else {
        thx = sc->fov_deg[2 * c->f + 0];
        thy = sc->fov_deg[2 * c->f + 1];
    }
    /* direction at the eye (air), refracted into the glass through the top
     * face (Snell), then mirrored by an in-coupler parallel to the mirrors */
    double tx = tan(thx * (M_PI / 180.0));
    double ty = tan(thy * (M_PI / 180.0));
    double inv = 1.0 / sqrt(tx * tx + ty * ty + 1.0);
    vec3 a = { tx * inv, ty * inv, inv };
    double ng = c->ng;
    vec3 g = { a.x / ng, a.y / ng, sqrt(1.0 - (a.x * a.x + a.y * a.y) / (ng * ng)) };
    double gn = c->nx * g.x + c->nz * g.z;
    double t2 = 2.0 * gn;
    r->d.x = g.x - t2 * c->nx;
    r->d.y = g.y;
    r->d.z = g.z - t2 * c->nz;
    /* polarization: pure s or pure p w.r.t. the slab-face basis */
    vec3 zhat = { 0.0, 0.0, 1.0 };
    vec3 s0 = cross3(r->d, zhat);
    s0 = scale3(s0, 1.0 / sqrt(dot3(s0, s0)));
    vec3 p0 = cross3(r->d, s0);
    vec3 e = (w[0] & 1u) ? p0 : s0;
    r->E.x = e.x; r->E.y = e.y; r->E.z = e.z;
    r->cell = 0;
    r->last = SURF_TOP;
}

/* s unit vector for direction d and surface normal n; falls back to the
 * y axis projected orthogonal to d when d is (nearly) parallel to n, where
 * s and p are physically equivalent. */
static vec3 s_basis(vec3 d, vec3 n)
{
    vec3 c = cross3(d, n);
    double l = sqrt(dot3(c, c));
    if (l < 1e-6) {
        vec3 y = { 0.0, 1.0, 0.0 };
        double yd = dot3(y, d);
        vec3 v = { -yd * d.x, 1.0 - yd * d.y, -yd * d.z };
        return scale3(v, 1.0 / sqrt(dot3(v, v)));
    }
    return scale3(c, 1.0 / l);
}

/* Eq. 5: E' = scale * (c_s (E.s) s + c_p (E.p_in) p_out). */
static cvec3 apply_sp(cvec3 E, vec3 s, vec3 pin, vec3 pout, double complex cs, double complex cp, double sc)
{
    double complex es = cdot3(E, s), ep = cdot3(E, pin);
    double complex as = sc * cs * es, ap = sc * cp * ep;
    cvec3 o = { as * s.x + ap * pout.x, as * s.y + ap * pout.y, as * s.z + ap * pout.z };
    return o;
}

/* Find the nearest bounding plane of the current cell, move there.
 * Returns the surface id (mirror index, or SURF_*), -1 if none. */
static int next_surface(const ctx_t* c, ray_t* r)
{
    const orc_scene* sc = c->sc;
    int M = sc->n_mirrors;
    double best = 0.0;
    int hit = -1;
    /* top */
    if (r->d.z > 0.0 && r->last != SURF_TOP) {
        double t = (sc->T - r->p.z) / r->d.z;
        if (hit < 0 || t < best) { best = t; hit = SURF_TOP; }
    }
    /* bottom */
    if (r->d.z < 0.0 && r->last != SURF_BOTTOM) {
        double t = (0.0 - r->p.z) / r->d.z;
        if (hit < 0 || t < best) { best = t; hit = SURF_BOTTOM; }
    }
    double dn = c->nx * r->d.x + c->nz * r->d.z;
    double pn = c->nx * r->p.x + c->nz * r->p.z;
    /* left boundary: end face or mirror cell-1 (cell lies on its -n side) */
    if (r->cell == 0) {
        if (r->d.x < 0.0 && r->last != SURF_END0) {
            double t = (0.0 - r->p.x) / r->d.x;
            if (hit < 0 || t < best) { best = t; hit = SURF_END0; }
        }
    } else {
        int m = r->cell - 1;
        if (dn > 0.0 && r->last != m) {
            double t = (c->h[m] - pn) / dn;
            if (hit < 0 || t < best) { best = t; hit = m; }
        }
    }
    /* right boundary: mirror cell (cell lies on its +n side) or end face */
    if (r->cell == M) {
        if (r->d.x > 0.0 && r->last != SURF_END1) {
            double t = (sc->Lx - r->p.x) / r->d.x;
            if (hit < 0 || t < best) { best = t; hit = SURF_END1; }
        }
    } else {
        int m = r->cell;
        if (dn < 0.0 && r->last != m) {
            double t = (c->h[m] - pn) / dn;
            if (hit < 0 || t < best) { best = t; hit = m; }
        }
    }
    if (hit < 0) return -1;
    r->p.x = r->p.x + best * r->d.x;
    r->p.y = r->p.y + best * r->d.y;
    r->p.z = r->p.z + best * r->d.z;
    if (hit == SURF_TOP) r->p.z = sc->T;
    if (hit == SURF_BOTTOM) r->p.z = 0.0;
    if (hit == SURF_END0) r->p.x = 0.0;
    if (hit == SURF_END1) r->p.x = sc->Lx;
    return hit;
}

/* Bare glass/air face coefficients (Eq. 3) for a ray inside the glass with
 * direction d hitting a face normal to z.  Returns 1 when totally reflected. */
static int face_coeffs(const ctx_t* c, vec3 d, double complex* rs, double complex* rp,
                       double complex* ts, double complex* tp, double* flux)
{
    double ng = c->ng, na = c->na;
    double ng2 = ng * ng, na2 = na * na;
    double st2 = ng2 * (d.x * d.x + d.y * d.y);       /* kappa^2 */
    double qi = ng * fabs(d.z);
    int tir = st2 > na2;
    double complex qt = tir ? CMPLX(0.0, sqrt(st2 - na2)) : CMPLX(sqrt(na2 - st2), 0.0);
    double complex Ni = ng, Nt = na;
    *rs = (qi - qt) / (qi + qt);
    *ts = 2.0 * qi / (qi + qt);
    *rp = (Nt * Nt * qi - Ni * Ni * qt) / (Nt * Nt * qi + Ni * Ni * qt);
    *tp = 2.0 * Ni * Nt * qi / (Nt * Nt * qi + Ni * Ni * qt);
    *flux = tir ? 0.0 : sqrt(creal(qt) / qi);
    return tir;
}

/* Face event at the top or bottom face (Eq. 3 at a bare glass/air
 * interface, Eq. 5 for the field, basis recomputed for this interface).
 * Total internal reflection keeps the ray in the glass: the field's s and p
 * components are multiplied by r_s and r_p and re-assembled on the reflected
 * basis.  Otherwise the top face emits the ray: the components are
 * multiplied by t_s and t_p and by the square root of the flux ratio, so
 * |E|^2 is the transmitted power, and the direction becomes the refracted
 * one in air; the bottom face loses the ray with its field unchanged.
 * Returns EV_TIR, EV_EXIT or EV_LEAK; t (optional) receives the tape entry
 * of a field-changing event. */
static int face_event(const ctx_t* c, ray_t* r, int s, tape_t* t)
{
    double complex rs, rp, ts, tp;
    double flux;
    int tir = face_coeffs(c, r->d, &rs, &rp, &ts, &tp, &flux);
    vec3 zhat = { 0.0, 0.0, 1.0 };
    vec3 sv = s_basis(r->d, zhat);
    vec3 pin = cross3(r->d, sv);
    if (tir) {
        vec3 dnew = { r->d.x, r->d.y, -r->d.z };
        vec3 pout = cross3(dnew, sv);
        if (t) {
            memset(t, 0, sizeof(*t));
            t->type = EV_TIR; t->s = sv; t->pin = pin; t->pout = pout;
            t->cs = rs; t->cp = rp; t->scale = 1.0; t->E_before = r->E;
        }
        r->E = apply_sp(r->E, sv, pin, pout, rs, rp, 1.0);
        r->d = dnew;
        r->last = s;
        return EV_TIR;
    }
    if (s != SURF_TOP) return EV_LEAK;
    double rn = c->ng / c->na;
    double st2 = (c->ng * c->ng) * (r->d.x * r->d.x + r->d.y * r->d.y);
    vec3 a = { rn * r->d.x, rn * r->d.y, sqrt(1.0 - st2 / (c->na * c->na)) };
    vec3 pout = cross3(a, sv);
    if (t) {
        memset(t, 0, sizeof(*t));
        t->type = EV_EXIT; t->s = sv; t->pin = pin; t->pout = pout;
        t->cs = ts; t->cp = tp; t->scale = flux; t->E_before = r->E;
    }
    r->E = apply_sp(r->E, sv, pin, pout, ts, tp, flux);
    r->d = a;
    return EV_EXIT;
}

/* Outcome of one event. */
typedef struct {
    int terminal;      /* 0 continue, else category + 1 */
    int bin;
    double w;
    vec3 a;            /* air direction at exit */
} outcome_t;

typedef struct {
    int mode;              /* 0 Philox, 1 forced bits, 2 branch callback (splitter) */
    uint64_t bits;
    int n_bits;
    double prob;
    int used;
} decider_t;

/* Eyebox binning of a ray leaving the top face at p with air direction a:
 * its crossing of the eyebox plane falls in a bin of the grid, or (with eye
 * pupils) inside one pupil's circle. */
static int eyebox_bin(const orc_scene* sc, vec3 p, vec3 a)
{
    double xe = p.x + sc->eye_relief * (a.x / a.z);
    double ye = p.y + sc->eye_relief * (a.y / a.z);
    if (sc->n_eye_pupils > 0) {
        double r2 = sc->eye_pupil_r * sc->eye_pupil_r;
        for (int q = 0; q < sc->n_eye_pupils; ++q) {
            double dx = xe - sc->eye_pupil_xy[2 * q];
            double dy = ye - sc->eye_pupil_xy[2 * q + 1];
            if (dx * dx + dy * dy < r2) return q;
        }
        return -1;
    }
    double fx = ((xe - sc->eye_x0) / sc->eye_w) * (double)sc->bins_x;
    double fy = ((ye - sc->eye_y0) / sc->eye_h) * (double)sc->bins_y;
    if (!(fx >= 0.0 && fx < (double)sc->bins_x && fy >= 0.0 && fy < (double)sc->bins_y)) return -1;
    int bx = (int)fx, by = (int)fy;
    return by * sc->bins_x + bx;
}

/* Mirror event: stack response for this side, branch, Eq. 5/6 update. */
void orc_table_weights(double theta, int n, int idx[4], double w[4])
{
    double h = (M_PI / 2.0) / (double)(n - 1);
    double x = theta / h;
    int j = (int)floor(x);
    if (j > n - 2) j = n - 2;
    if (j < 0) j = 0;
    double t = x - (double)j;
    /* cubic Hermite on [theta_j, theta_j+1] with central-difference slopes */
    w[0] = 0.5 * (-t * t * t + 2.0 * t * t - t);
    w[1] = 0.5 * (3.0 * t * t * t - 5.0 * t * t + 2.0);
    w[2] = 0.5 * (-3.0 * t * t * t + 4.0 * t * t + t);
    w[3] = 0.5 * (t * t * t - t * t);
    idx[0] = j == 0 ? 1 : j - 1;
    idx[1] = j;
    idx[2] = j + 1;
    idx[3] = j + 2 < n ? j + 2 : n - 1;
}

/* Incidence angle in the glass of a hit with kappa = n_g sin(theta). */
static double hit_theta(double kappa, double ng)
{
    double s = kappa / ng;
    return asin(s < 1.0 ? s : 1.0);
}

/* Node kappa of table angle j. */
static double node_kappa(const ctx_t* c, int j)
{
    return c->ng * sin((double)j * ((M_PI / 2.0) / (double)(c->sc->table_nodes - 1)));
}

/* The four coefficients of mirror m's stack seen from `side` at kappa:
 * exact, or interpolated from the angle table. */
static void hit_coeffs(const ctx_t* c, int m, int side, double kappa, double complex co[4])
{
    size_t base = ((size_t)m * 2 + side) * c->sc->max_layers;
    if (c->sc->table_nodes <= 0) {
        orc__tmm_coeffs(c->s_len[m], c->s_thk + base, c->s_nre + base, c->s_nim + base,
                        c->ng, c->lambda_nm, kappa, co);
        return;
    }
    int idx[4];
    double w[4];
    orc_table_weights(hit_theta(kappa, c->ng), c->sc->table_nodes, idx, w);
    for (int q = 0; q < 4; ++q) co[q] = 0.0;
    for (int i = 0; i < 4; ++i) {
        double complex ci[4];
        orc__tmm_coeffs(c->s_len[m], c->s_thk + base, c->s_nre + base, c->s_nim + base,
                        c->ng, c->lambda_nm, node_kappa(c, idx[i]), ci);
        for (int q = 0; q < 4; ++q) co[q] += w[i] * ci[q];
    }
}

/* d c / d thk_j of the same coefficients (orc_tmm_dthk layout), exact or
 * through the interpolation (linear in the table entries). */
static void hit_dthk(const ctx_t* c, int m, int side, double kappa, double* dd, double* tmp)
{
    size_t base = ((size_t)m * 2 + side) * c->sc->max_layers;
    int L = c->s_len[m];
    if (c->sc->table_nodes <= 0) {
        orc_tmm_dthk(L, c->s_thk + base, c->s_nre + base, c->s_nim + base, c->ng, c->ng, 0.0,
                     c->lambda_nm, kappa, dd);
        return;
    }
    int idx[4];
    double w[4];
    orc_table_weights(hit_theta(kappa, c->ng), c->sc->table_nodes, idx, w);
    memset(dd, 0, sizeof(double) * 16 * (size_t)(L > 0 ? L : 1));
    for (int i = 0; i < 4; ++i) {
        orc_tmm_dthk(L, c->s_thk + base, c->s_nre + base, c->s_nim + base, c->ng, c->ng, 0.0,
                     c->lambda_nm, node_kappa(c, idx[i]), tmp);
        for (int k = 0; k < 16 * L; ++k) dd[k] += w[i] * tmp[k];
    }
}

static void mirror_event(const ctx_t* c, ray_t* r, int m, int reflect, int mc_scale, tape_t* tp_out)
{
    vec3 n = { c->nx, 0.0, c->nz };
    double dn = c->nx * r->d.x + c->nz * r->d.z;
    int front = dn < 0.0;
    vec3 cr = cross3(r->d, n);
    double sin_i = sqrt(dot3(cr, cr));
    double kappa = c->ng * sin_i;
    int side = front ? 0 : 1;
    double complex co[4];
    hit_coeffs(c, m, side, kappa, co);
    double p = c->p_eff[m];
    vec3 dnew = r->d;
    if (reflect) {
        double t2 = 2.0 * dn;
        dnew.x = r->d.x - t2 * c->nx;
        dnew.z = r->d.z - t2 * c->nz;
    }
    vec3 s = s_basis(r->d, n);
    vec3 pin = cross3(r->d, s);
    vec3 pout = cross3(dnew, s);
    double complex cs = reflect ? co[0] : co[2];
    double complex cp = reflect ? co[1] : co[3];
    double sc = !mc_scale ? 1.0 : (reflect ? 1.0 / sqrt(p) : 1.0 / sqrt(1.0 - p));
    if (tp_out) {
        tp_out->type = EV_MIRROR; tp_out->mirror = m; tp_out->front = front;
        tp_out->reflect = reflect; tp_out->kappa = kappa;
        tp_out->s = s; tp_out->pin = pin; tp_out->pout = pout;
        tp_out->cs = cs; tp_out->cp = cp; tp_out->scale = sc; tp_out->E_before = r->E;
    }
    r->E = apply_sp(r->E, s, pin, pout, cs, cp, sc);
    r->d = dnew;
    if (!reflect) r->cell += (m == r->cell) ? 1 : -1;
    r->last = m;
}

/* Decision at the k-th mirror hit. */
static int decide(const ctx_t* c, ray_t* r, int m, decider_t* dc)
{
    int h = r->n_prma;
    if (dc->mode == 0) {
        if ((h & 3) == 0) philox_words(c, r->ray_id, (uint32_t)(h >> 2), 1u, r->words);
        return r->words[h & 3] < c->thr[m];
    }
    int bit = (h < 64) ? (int)((dc->bits >> h) & 1u) : 0;
    dc->prob *= bit ? c->p_eff[m] : 1.0 - c->p_eff[m];
    dc->used = h + 1;
    return bit;
}

/* One full Monte Carlo trace.  tape (optional) gets up to max_events entries;
 * evlog (optional) gets 10 doubles per event. */
static outcome_t trace_one(const ctx_t* c, int64_t ray_id, decider_t* dc,
                           tape_t* tape, int* n_tape, double* evlog, int evcap, ray_t* rout,
                           orc_stats* st)
{
    const orc_scene* sc = c->sc;
    ray_t r;
    ray_birth(c, ray_id, &r);
    outcome_t o = { 0, -1, 0.0, { 0, 0, 0 } };
    int nt = 0;
    for (int k = 0; k < sc->max_events; ++k) {
        int s = next_surface(c, &r);
        if (s < 0) { o.terminal = ORC_LOST + 1; break; }
        r.n_events++;
        double aoi = 0.0;
        int branch = -1;
        int evtype = EV_MIRROR;
        if (s == SURF_TOP || s == SURF_BOTTOM) {
            double w_in = norm2c(r.E);
            evtype = face_event(c, &r, s, tape ? &tape[nt] : NULL);
            if (tape && evtype != EV_LEAK) nt++;
            if (evtype == EV_EXIT) {
                o.a = r.d;
                o.w = norm2c(r.E);
                if (st) st->power[ORC_FACE_R] += w_in - o.w;
                o.bin = eyebox_bin(sc, r.p, r.d);
                o.terminal = (o.bin >= 0 ? ORC_EYEBOX : ORC_MISS) + 1;
            } else if (evtype == EV_LEAK) {
                o.terminal = ORC_LEAK + 1;
                o.w = norm2c(r.E);
            }
        } else if (s == SURF_END0 || s == SURF_END1) {
            evtype = EV_END;
            o.terminal = ORC_END + 1;
            o.w = norm2c(r.E);
        } else {
            int m = s;
            double dn = c->nx * r.d.x + c->nz * r.d.z;
            aoi = acos(fabs(dn)) * (180.0 / M_PI);
            int refl = decide(c, &r, m, dc);
            branch = refl;
            mirror_event(c, &r, m, refl, 1, tape ? &tape[nt] : NULL);
            if (tape) nt++;
            r.n_prma++;
        }
        if (evlog && r.n_events <= evcap) {
            double* e = evlog + (size_t)(r.n_events - 1) * 10;
            e[0] = (double)evtype;
            e[1] = (double)s;
            e[2] = r.p.x; e[3] = r.p.y; e[4] = r.p.z;
            e[5] = r.d.x; e[6] = r.d.y; e[7] = r.d.z;
            e[8] = aoi; e[9] = (double)branch;
        }
        if (o.terminal) break;
    }
    if (!o.terminal) {
        o.terminal = ORC_TRUNC + 1;
        o.w = norm2c(r.E);
    }
    if (n_tape) *n_tape = nt;
    if (rout) *rout = r;
    return o;
}

static int point_of(const orc_scene* sc, int64_t ray_id, int* d, int* li, int* f)
{
    int64_t pt = ray_id / sc->rays_per_point;
    int F = sc->fov_mode == 1 ? 1 : sc->n_fov;
    *f = (int)(pt % F); pt /= F;
    *li = (int)(pt % sc->n_lsel); pt /= sc->n_lsel;
    *d = (int)pt;
    return (*d < sc->n_designs) ? 0 : -1;
}

int orc_trace_forward(const orc_scene* sc, uint64_t* q_bins, uint32_t* counts,
                      double* wsum, orc_stats* stats)
{
    ctx_t c;
    if (ctx_init(&c, sc)) return -1;
    int F = sc->fov_mode == 1 ? 1 : sc->n_fov;
    int B = sc->bins_x * sc->bins_y;
    size_t n_bins = (size_t)sc->n_designs * sc->n_lsel * F * B;
    if (q_bins) memset(q_bins, 0, sizeof(uint64_t) * n_bins);
    if (counts) memset(counts, 0, sizeof(uint32_t) * n_bins);
    if (wsum) memset(wsum, 0, sizeof(double) * n_bins);
    orc_stats local;
    memset(&local, 0, sizeof(local));
    double cap = ldexp(1.0, 40);
    double scale = ldexp(1.0, sc->fp_shift);
    for (int d = 0; d < sc->n_designs; ++d)
        for (int li = 0; li < sc->n_lsel; ++li)
            for (int f = 0; f < F; ++f) {
                ctx_point(&c, d, li, f);
                size_t pt = ((size_t)d * sc->n_lsel + li) * F + f;
                for (int64_t i = 0; i < sc->rays_per_point; ++i) {
                    int64_t ray_id = (int64_t)pt * sc->rays_per_point + i;
                    decider_t dc = { 0, 0, 0, 1.0, 0 };
                    ray_t r;
                    outcome_t o = trace_one(&c, ray_id, &dc, NULL, NULL, NULL, 0, &r, &local);
                    local.counters[0] += 1;
                    local.counters[1] += r.n_events;
                    local.counters[2] += r.n_prma;
                    int cat = o.terminal - 1;
                    local.counters[4 + cat] += 1;
                    local.power[cat] += o.w;
                    if (cat == ORC_EYEBOX) {
                        size_t k = pt * B + (size_t)o.bin;
                        double units = o.w * scale;
                        if (units > cap) { units = cap; local.counters[3] += 1; }
                        if (q_bins) q_bins[k] += (uint64_t)llrint(units);
                        if (counts) counts[k] += 1u;
                        if (wsum) wsum[k] += o.w;
                    }
                }
            }
    if (stats) *stats = local;
    ctx_free(&c);
    return 0;
}

int orc_trace_rays(const orc_scene* sc, int64_t n, const int64_t* ray_ids, orc_ray_record* rec)
{
    ctx_t c;
    if (ctx_init(&c, sc)) return -1;
    for (int64_t k = 0; k < n; ++k) {
        int d, li, f;
        if (point_of(sc, ray_ids[k], &d, &li, &f)) { ctx_free(&c); return -2; }
        ctx_point(&c, d, li, f);
        decider_t dc = { 0, 0, 0, 1.0, 0 };
        ray_t r;
        outcome_t o = trace_one(&c, ray_ids[k], &dc, NULL, NULL, NULL, 0, &r, NULL);
        orc_ray_record* q = &rec[k];
        q->ray_id = ray_ids[k];
        q->category = o.terminal - 1;
        q->bin = q->category == ORC_EYEBOX ? o.bin : -1;
        q->n_events = r.n_events;
        q->n_prma = r.n_prma;
        q->w = o.w;
        q->exit_dir[0] = o.a.x; q->exit_dir[1] = o.a.y; q->exit_dir[2] = o.a.z;
        q->exit_pos[0] = r.p.x; q->exit_pos[1] = r.p.y; q->exit_pos[2] = r.p.z;
    }
    ctx_free(&c);
    return 0;
}

int orc_ray_events(const orc_scene* sc, int64_t ray_id, int cap, double* ev10)
{
    ctx_t c;
    if (ctx_init(&c, sc)) return -1;
    int d, li, f;
    if (point_of(sc, ray_id, &d, &li, &f)) { ctx_free(&c); return -2; }
    ctx_point(&c, d, li, f);
    decider_t dc = { 0, 0, 0, 1.0, 0 };
    ray_t r;
    trace_one(&c, ray_id, &dc, NULL, NULL, ev10, cap, &r, NULL);
    ctx_free(&c);
    return r.n_events;
}

int orc_trace_forced(const orc_scene* sc, int64_t ray_id, uint64_t decisions, int n_decisions,
                     double* w, double* prob, int* n_used)
{
    ctx_t c;
    if (ctx_init(&c, sc)) return -1;
    int d, li, f;
    if (point_of(sc, ray_id, &d, &li, &f)) { ctx_free(&c); return -2; }
    ctx_point(&c, d, li, f);
    decider_t dc = { 1, decisions, n_decisions, 1.0, 0 };
    ray_t r;
    outcome_t o = trace_one(&c, ray_id, &dc, NULL, NULL, NULL, 0, &r, NULL);
    *w = (o.terminal - 1 == ORC_EYEBOX) ? o.w : 0.0;
    *prob = dc.prob;
    *n_used = r.n_prma;
    ctx_free(&c);
    return (o.terminal - 1 == ORC_EYEBOX) ? o.bin : -1;
}

int orc_trace_forward_sampled(const orc_scene* sc, int64_t sample_stride, double* irr)
{
    ctx_t c;
    if (ctx_init(&c, sc)) return -1;
    int F = sc->fov_mode == 1 ? 1 : sc->n_fov;
    int B = sc->bins_x * sc->bins_y;
    size_t n_bins = (size_t)sc->n_designs * sc->n_lsel * F * B;
    memset(irr, 0, sizeof(double) * n_bins);
    if (sample_stride < 1) sample_stride = 1;
    for (int d = 0; d < sc->n_designs; ++d)
        for (int li = 0; li < sc->n_lsel; ++li)
            for (int f = 0; f < F; ++f) {
                ctx_point(&c, d, li, f);
                size_t pt = ((size_t)d * sc->n_lsel + li) * F + f;
                for (int64_t i = 0; i < sc->rays_per_point; ++i) {
                    int64_t ray_id = (int64_t)pt * sc->rays_per_point + i;
                    if (ray_id % sample_stride) continue;
                    decider_t dc = { 0, 0, 0, 1.0, 0 };
                    outcome_t o = trace_one(&c, ray_id, &dc, NULL, NULL, NULL, 0, NULL, NULL);
                    if (o.terminal - 1 == ORC_EYEBOX)
                        irr[pt * B + (size_t)o.bin] += o.w / (double)sc->rays_per_point;
                }
            }
    ctx_free(&c);
    return 0;
}

/* ------------------------------------------------------------ the adjoint */
/* w = |E_K|^2 along a fixed path.  With lambda_k the adjoint field after
 * event k (lambda_K = E_K, lambda_{k-1} = A_k^H lambda_k), the holomorphic
 * sensitivities of w to the event's coefficients are
 *   G_s = scale conj(lambda_k . s) (s . E_{k-1}),
 *   G_p = scale conj(lambda_k . p_out) (p_in . E_{k-1}),
 * and dw/dthk = 2 Re(G_s dc_s/dthk + G_p dc_p/dthk). */
int orc_trace_backward(const orc_scene* sc, const double* dL_dI, int64_t sample_stride, double* grad)
{
    ctx_t c;
    if (ctx_init(&c, sc)) return -1;
    int F = sc->fov_mode == 1 ? 1 : sc->n_fov;
    int B = sc->bins_x * sc->bins_y;
    int Lm = sc->max_layers;
    memset(grad, 0, sizeof(double) * (size_t)sc->n_designs * sc->n_mirrors * Lm);
    if (sample_stride < 1) sample_stride = 1;
    tape_t* tape = (tape_t*)malloc(sizeof(tape_t) * (size_t)(sc->max_events + 1));
    double* dd = (double*)malloc(sizeof(double) * 16 * (size_t)(Lm > 0 ? Lm : 1));
    double* tmp = (double*)malloc(sizeof(double) * 16 * (size_t)(Lm > 0 ? Lm : 1));
    for (int d = 0; d < sc->n_designs; ++d)
        for (int li = 0; li < sc->n_lsel; ++li)
            for (int f = 0; f < F; ++f) {
                ctx_point(&c, d, li, f);
                size_t pt = ((size_t)d * sc->n_lsel + li) * F + f;
                for (int64_t i = 0; i < sc->rays_per_point; ++i) {
                    int64_t ray_id = (int64_t)pt * sc->rays_per_point + i;
                    if (ray_id % sample_stride) continue;
                    decider_t dc = { 0, 0, 0, 1.0, 0 };
                    int nt = 0;
                    ray_t r;
                    outcome_t o = trace_one(&c, ray_id, &dc, tape, &nt, NULL, 0, &r, NULL);
                    if (o.terminal - 1 != ORC_EYEBOX) continue;
                    double g = dL_dI[pt * B + (size_t)o.bin] / (double)sc->rays_per_point;
                    if (g == 0.0) continue;
                    cvec3 lam = r.E;
                    for (int k = nt - 1; k >= 0; --k) {
                        const tape_t* t = &tape[k];
                        if (t->type == EV_MIRROR) {
                            double complex Gs = t->scale * conj(cdot3(lam, t->s)) * cdot3(t->E_before, t->s);
                            double complex Gp = t->scale * conj(cdot3(lam, t->pout)) * cdot3(t->E_before, t->pin);
                            int m = t->mirror;
                            int side = t->front ? 0 : 1;
                            int L = c.s_len[m];
                            hit_dthk(&c, m, side, t->kappa, dd, tmp);
                            int cs_i = t->reflect ? 0 : 2, cp_i = t->reflect ? 1 : 3;
                            for (int j = 0; j < L; ++j) {
                                double complex dcs = CMPLX(dd[j * 16 + 4 * cs_i], dd[j * 16 + 4 * cs_i + 1]);
                                double complex dcp = CMPLX(dd[j * 16 + 4 * cp_i], dd[j * 16 + 4 * cp_i + 1]);
                                double dw = 2.0 * creal(Gs * dcs + Gp * dcp);
                                int layer = t->front ? j : L - 1 - j;
                                grad[((size_t)d * sc->n_mirrors + m) * Lm + layer] += g * dw;
                            }
                        }
                        /* lambda <- A^H lambda, A = scale (c_s s s^T + c_p p_out p_in^T) */
                        double complex ls = cdot3(lam, t->s), lp = cdot3(lam, t->pout);
                        double complex as = t->scale * conj(t->cs) * ls;
                        double complex ap = t->scale * conj(t->cp) * lp;
                        cvec3 nl = { as * t->s.x + ap * t->pin.x, as * t->s.y + ap * t->pin.y,
                                     as * t->s.z + ap * t->pin.z };
                        lam = nl;
                    }
                }
            }
    free(tape);
    free(dd);
    free(tmp);
    ctx_free(&c);
    return 0;
}

/* -------------------------------------------------- brute-force splitting */
typedef struct {
    const ctx_t* c;
    double* bin_power;
    int64_t paths;
} split_t;

/* Follow both branches at every mirror (no probabilities, no rescaling);
 * a path truncated at max_events contributes nothing, like the tracer. */
static void split_rec(split_t* S, ray_t r, int k)
{
    const ctx_t* c = S->c;
    const orc_scene* sc = c->sc;
    for (; k < sc->max_events; ++k) {
        int s = next_surface(c, &r);
        if (s < 0) { S->paths++; return; }
        r.n_events++;
        if (s == SURF_TOP || s == SURF_BOTTOM) {
            int ev = face_event(c, &r, s, NULL);
            if (ev == EV_TIR) continue;
            if (ev == EV_EXIT) {
                int b = eyebox_bin(sc, r.p, r.d);
                if (b >= 0) S->bin_power[b] += norm2c(r.E);
            }
            S->paths++;
            return;
        }
        if (s == SURF_END0 || s == SURF_END1) { S->paths++; return; }
        /* mirror: reflect branch recursively, continue with transmit */
        ray_t rr = r;
        mirror_event(c, &rr, s, 1, 0, NULL);
        rr.n_prma++;
        split_rec(S, rr, k + 1);
        mirror_event(c, &r, s, 0, 0, NULL);
        r.n_prma++;
    }
    S->paths++;
}

int orc_split_bruteforce(const orc_scene* sc, int32_t d, int32_t lsel, int32_t f,
                         int64_t first, int64_t n_rays, double* bin_power, int64_t* n_paths)
{
    ctx_t c;
    if (ctx_init(&c, sc)) return -1;
    ctx_point(&c, d, lsel, f);
    int F = sc->fov_mode == 1 ? 1 : sc->n_fov;
    int B = sc->bins_x * sc->bins_y;
    memset(bin_power, 0, sizeof(double) * (size_t)B);
    split_t S = { &c, bin_power, 0 };
    size_t pt = ((size_t)d * sc->n_lsel + lsel) * F + f;
    for (int64_t i = first; i < first + n_rays; ++i) {
        ray_t r;
        ray_birth(&c, (int64_t)pt * sc->rays_per_point + i, &r);
        split_rec(&S, r, 0);
    }
    if (n_paths) *n_paths = S.paths;
    ctx_free(&c);
    return 0;
}

/* ------------------------------------------------------ single-event probe */
/* One field-changing event in isolation, for the polarization pins: a ray of
 * point (d, li, fov 0) in the glass with direction dir_in and complex field
 * E_in (x, y, z as (re, im) pairs) meets `surface` (a mirror index, or
 * ORC_SURF_TOP / ORC_SURF_BOTTOM).  A mirror applies the branch `reflect`
 * without the Monte Carlo 1/sqrt(p) factor; a face reflects totally or emits
 * the ray (top) exactly as in the trace.  Returns the event type (1 TIR,
 * 2 exit, 3 leak, 5 mirror) or a negative value for a bad argument. */
int orc_event_probe(const orc_scene* sc, int32_t d, int32_t li, int32_t surface, int32_t reflect,
                    const double dir_in[3], const double E_in[6], double dir_out[3], double E_out[6])
{
    if (d < 0 || d >= sc->n_designs || li < 0 || li >= sc->n_lsel) return -2;
    if (!(surface == SURF_TOP || surface == SURF_BOTTOM || (surface >= 0 && surface < sc->n_mirrors)))
        return -3;
    ctx_t c;
    if (ctx_init(&c, sc)) return -1;
    ctx_point(&c, d, li, 0);
    ray_t r;
    memset(&r, 0, sizeof(r));
    r.d.x = dir_in[0]; r.d.y = dir_in[1]; r.d.z = dir_in[2];
    r.E.x = CMPLX(E_in[0], E_in[1]);
    r.E.y = CMPLX(E_in[2], E_in[3]);
    r.E.z = CMPLX(E_in[4], E_in[5]);
    r.last = -1;
    int ev;
    if (surface == SURF_TOP || surface == SURF_BOTTOM) {
        ev = face_event(&c, &r, surface, NULL);
    } else {
        r.cell = surface;
        mirror_event(&c, &r, surface, reflect ? 1 : 0, 0, NULL);
        ev = EV_MIRROR;
    }
    dir_out[0] = r.d.x; dir_out[1] = r.d.y; dir_out[2] = r.d.z;
    E_out[0] = creal(r.E.x); E_out[1] = cimag(r.E.x);
    E_out[2] = creal(r.E.y); E_out[3] = cimag(r.E.y);
    E_out[4] = creal(r.E.z); E_out[5] = cimag(r.E.z);
    ctx_free(&c);
    return ev;
}
