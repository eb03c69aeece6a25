/*
 * Thin-film stack response by the recursive Airy (Rouard) method.
 * Test infrastructure (oracle); see oracle.h.
 *
 * Methods, "Multilayer thin-film solver": the single-interface Fresnel
 * coefficients (Eq. 3) and the single-layer Airy sums (Eq. 4) are applied
 * repeatedly from the exit medium outwards: the stack below interface j is
 * replaced by its effective reflection coefficient, and the layer above is
 * then summed with Eq. 4.  The phase thickness of layer j is
 * delta_j = (2 pi / lambda) q_j d_j with q_j = N_j cos(theta_j) = sqrt(N_j^2 - kappa^2)
 * (Snell's law in invariant form).  The exp(-i w t) convention makes the
 * per-pass factor exp(+2 i delta).
 *
 * The derivative routine differentiates the same recursion in reverse mode.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include "oracle.h"

/* Normal-direction wavenumber (units of k0) with Im q >= 0, Re q >= 0 if real. */
static double complex qz(double complex N, double kappa)
{
    double complex z = N * N - kappa * kappa;
    if (cimag(z) == 0.0) {
        double zr = creal(z);
        if (zr >= 0.0) return CMPLX(sqrt(zr), 0.0);
        return CMPLX(0.0, sqrt(-zr));
    }
    double complex q = csqrt(z);
    if (cimag(q) < 0.0) q = -q;
    return q;
}

/* Eq. 3 at the interface a -> b: s and p reflection/transmission. */
static void fresnel(double complex Na, double complex qa, double complex Nb, double complex qb,
                    double complex* rs, double complex* ts, double complex* rp, double complex* tp)
{
    *rs = (qa - qb) / (qa + qb);
    *ts = 2.0 * qa / (qa + qb);
    double complex Na2 = Na * Na, Nb2 = Nb * Nb;
    *rp = (Nb2 * qa - Na2 * qb) / (Nb2 * qa + Na2 * qb);
    *tp = 2.0 * Na * Nb * qa / (Nb2 * qa + Na2 * qb);
}

typedef struct {
    int L;
    double complex* N;    /* media 0..L+1 */
    double complex* q;
    double* d;            /* d[j] for layers 1..L (index j) */
    double k0;            /* 2 pi / lambda, per nm */
} stack_t;

static int stack_init(stack_t* s, int L, const double* thk, const double* nre, const double* nim,
                      double n_in, double nout_re, double nout_im, double lambda_nm, double kappa)
{
    s->L = L;
    s->N = (double complex*)malloc(sizeof(double complex) * (size_t)(L + 2));
    s->q = (double complex*)malloc(sizeof(double complex) * (size_t)(L + 2));
    s->d = (double*)malloc(sizeof(double) * (size_t)(L + 2));
    if (!s->N || !s->q || !s->d) return -1;
    s->N[0] = CMPLX(n_in, 0.0);
    for (int j = 1; j <= L; ++j) {
        s->N[j] = CMPLX(nre[j - 1], nim[j - 1]);
        s->d[j] = thk[j - 1];
    }
    s->N[L + 1] = CMPLX(nout_re, nout_im);
    for (int j = 0; j <= L + 1; ++j) s->q[j] = qz(s->N[j], kappa);
    s->k0 = 2.0 * M_PI / lambda_nm;
    return 0;
}

static void stack_free(stack_t* s)
{
    free(s->N); free(s->q); free(s->d);
}

/* Per-step intermediates of the recursion for layer j+1 sitting under interface j. */
typedef struct {
    double complex r, t;        /* interface j -> j+1 Fresnel */
    double complex e1, e2;      /* exp(i delta), exp(2 i delta) of layer j+1 */
    double complex x, D;        /* x = Gamma_{j+1} e2, D = 1 + r x */
    double complex gam, tau;    /* Gamma_j, tau_j */
} step_t;

/* Forward recursion for one polarization (pol 0 = s, 1 = p).  steps[j] for
 * j = 0..L-1 hold the intermediates; returns Gamma_0, tau_0. */
static void rouard(const stack_t* s, int pol, step_t* steps, double complex* r_out, double complex* t_out)
{
    int L = s->L;
    double complex rs, ts, rp, tp;
    fresnel(s->N[L], s->q[L], s->N[L + 1], s->q[L + 1], &rs, &ts, &rp, &tp);
    double complex gam = pol ? rp : rs;
    double complex tau = pol ? tp : ts;
    for (int j = L - 1; j >= 0; --j) {
        step_t* st = &steps[j];
        fresnel(s->N[j], s->q[j], s->N[j + 1], s->q[j + 1], &rs, &ts, &rp, &tp);
        st->r = pol ? rp : rs;
        st->t = pol ? tp : ts;
        double complex delta = s->k0 * s->q[j + 1] * s->d[j + 1];
        st->e1 = cexp(I * delta);
        st->e2 = cexp(2.0 * I * delta);
        st->x = gam * st->e2;
        st->D = 1.0 + st->r * st->x;
        st->gam = (st->r + st->x) / st->D;
        st->tau = st->t * tau * st->e1 / st->D;
        gam = st->gam;
        tau = st->tau;
    }
    *r_out = gam;
    *t_out = tau;
}

void orc_tmm_rt(int n_layers, const double* thk_nm, const double* nre, const double* nim,
                double n_in, double nout_re, double nout_im,
                double lambda_nm, double kappa, double out[8])
{
    stack_t s;
    step_t* steps = (step_t*)malloc(sizeof(step_t) * (size_t)(n_layers > 0 ? n_layers : 1));
    stack_init(&s, n_layers, thk_nm, nre, nim, n_in, nout_re, nout_im, lambda_nm, kappa);
    double complex r[2], t[2];
    for (int pol = 0; pol < 2; ++pol) rouard(&s, pol, steps, &r[pol], &t[pol]);
    out[0] = creal(r[0]); out[1] = cimag(r[0]);
    out[2] = creal(r[1]); out[3] = cimag(r[1]);
    out[4] = creal(t[0]); out[5] = cimag(t[0]);
    out[6] = creal(t[1]); out[7] = cimag(t[1]);
    stack_free(&s);
    free(steps);
}

/* Reverse mode through rouard(): dc/d delta_{j+1} for every step, then
 * dc/dd = dc/d delta * k0 q.  which = 0 differentiates Gamma_0, 1 tau_0. */
static void rouard_adjoint(const stack_t* s, const step_t* steps, int which, double complex* dc_dd)
{
    double complex a_gam = which == 0 ? 1.0 : 0.0;
    double complex a_tau = which == 0 ? 0.0 : 1.0;
    for (int j = 0; j < s->L; ++j) {
        const step_t* st = &steps[j];
        /* Gamma_j = (r + x) / D,  tau_j = t tau_{j+1} e1 / D,  x = Gamma_{j+1} e2 */
        double complex dgam_dx = (1.0 - st->r * st->r) / (st->D * st->D);
        double complex dtau_dx = -st->tau * st->r / st->D;
        double complex a_x = a_gam * dgam_dx + a_tau * dtau_dx;
        /* d x / d delta = 2 i x ; d tau_j / d delta (through e1) = i tau_j */
        double complex dc_ddelta = a_x * (2.0 * I * st->x) + a_tau * (I * st->tau);
        dc_dd[j] = dc_ddelta * s->k0 * s->q[j + 1];
        /* propagate to Gamma_{j+1}, tau_{j+1} */
        double complex next_gam = a_x * st->e2;
        double complex next_tau = a_tau * st->t * st->e1 / st->D;
        a_gam = next_gam;
        a_tau = next_tau;
    }
}

void orc_tmm_dthk(int n_layers, const double* thk_nm, const double* nre, const double* nim,
                  double n_in, double nout_re, double nout_im,
                  double lambda_nm, double kappa, double* d_out)
{
    if (n_layers <= 0) return;
    stack_t s;
    step_t* steps = (step_t*)malloc(sizeof(step_t) * (size_t)n_layers);
    double complex* dd = (double complex*)malloc(sizeof(double complex) * (size_t)n_layers);
    stack_init(&s, n_layers, thk_nm, nre, nim, n_in, nout_re, nout_im, lambda_nm, kappa);
    for (int pol = 0; pol < 2; ++pol) {
        double complex r, t;
        rouard(&s, pol, steps, &r, &t);
        for (int which = 0; which < 2; ++which) {
            int c = which * 2 + pol;   /* r_s, r_p, t_s, t_p */
            rouard_adjoint(&s, steps, which, dd);
            for (int j = 0; j < n_layers; ++j) {
                d_out[j * 16 + 4 * c + 0] = creal(dd[j]);
                d_out[j * 16 + 4 * c + 1] = cimag(dd[j]);
                d_out[j * 16 + 4 * c + 2] = 0.0;
                d_out[j * 16 + 4 * c + 3] = 0.0;
            }
        }
    }
    stack_free(&s);
    free(steps);
    free(dd);
}

/* ---- internal API used by the tracer: both coefficients and their
 * derivatives for one polarization set, on a stack described by per-layer
 * index arrays (already in incidence order). */
void orc__tmm_coeffs(int L, const double* thk, const double* nre, const double* nim,
                     double n_glass, double lambda_nm, double kappa,
                     double complex c[4])
{
    double out[8];
    orc_tmm_rt(L, thk, nre, nim, n_glass, n_glass, 0.0, lambda_nm, kappa, out);
    for (int k = 0; k < 4; ++k) c[k] = CMPLX(out[2 * k], out[2 * k + 1]);
}

/* Many queries of one stack whose layer indices depend on the wavelength:
 * query q uses wavelength row li[q] of nre/nim ([n_lambda][n_layers]) and of
 * n_in / nout ([n_lambda]; nout as (re, im) pairs), lambda_nm[li[q]] and the
 * angle of incidence theta[q] (rad) in the incident medium.  out[q][8] as
 * orc_tmm_rt.  A plain loop over orc_tmm_rt (callers may split the queries
 * across threads: nothing is shared). */
void orc_tmm_rt_batch(int n_layers, const double* thk, const double* nre, const double* nim,
                      const double* n_in, const double* nout, const double* lambda_nm,
                      int64_t n_q, const int32_t* li, const double* theta, double* out)
{
    for (int64_t q = 0; q < n_q; ++q) {
        const int l = li[q];
        const double kappa = n_in[l] * sin(theta[q]);
        orc_tmm_rt(n_layers, thk, nre + (size_t)l * n_layers, nim + (size_t)l * n_layers, n_in[l],
                   nout[2 * l], nout[2 * l + 1], lambda_nm[l], kappa, out + 8 * q);
    }
}
