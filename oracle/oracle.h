/*
 * FP64 CPU oracle for the differentiable Monte Carlo polarization ray trace
 * through a geometric waveguide (arXiv 2601.04370, Methods).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this code; only the test-suite, the smoke check and the bench's CPU
 * baseline leg do.  It is deliberately plain and slow: one ray at a time,
 * double precision, no blocking or fusion, every step in the order the paper
 * describes it.  It shares no code with the HIP implementation.
 *
 * Conventions (readings of points the paper leaves open):
 *   - time dependence exp(-i w t); complex index N = n + i k, k >= 0 absorbs;
 *     a layer's phase factor is exp(+i delta), so single-layer results are the
 *     complex conjugates of the Airy formulas (Eq. 4) as printed, which use
 *     exp(-2 i delta); intensities are identical;
 *   - Fresnel coefficients exactly as Eq. 3 (s: TE, p: TM with p = k x s for
 *     each ray), so r_p(0 deg) = -r_s(0 deg);
 *   - normal-direction wavenumber q = sqrt(N^2 - kappa^2), kappa = n_0 sin(theta_0),
 *     branch Im q >= 0 (and Re q >= 0 when Im q = 0).
 *
 * Units: lengths in mm for geometry, layer thicknesses and wavelengths in nm.
 */
#ifndef GWG_ORACLE_H
#define GWG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- Philox */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): out = bijection(ctr, key). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* ------------------------------------------------------------- thin film */
/* One stack in incidence order: layer j has index (nre[j], nim[j]) and
 * thickness thk_nm[j]; incident medium n_in (real), exit medium (nout_re, nout_im).
 * kappa = n_in * sin(theta_in).  Output out[8] = r_s, r_p, t_s, t_p as
 * (re, im) pairs in the Eq. 3 amplitude convention.  Recursive Airy (Rouard)
 * evaluation of Eq. 4 from the exit medium outwards. */
void orc_tmm_rt(int n_layers, const double* thk_nm, const double* nre, const double* nim,
                double n_in, double nout_re, double nout_im,
                double lambda_nm, double kappa, double out[8]);

/* Many queries of one stack, the layer indices per wavelength row li[q]
 * ([n_lambda][n_layers] tables; n_in, nout, lambda_nm per row, nout as
 * (re, im)); theta[q] in the incident medium; out[q][8] as orc_tmm_rt. */
void orc_tmm_rt_batch(int n_layers, const double* thk, const double* nre, const double* nim,
                      const double* n_in, const double* nout, const double* lambda_nm,
                      int64_t n_q, const int32_t* li, const double* theta, double* out);

/* Holomorphic derivatives d c / d thk_j (per nm) of the four coefficients,
 * by reverse-mode through the same recursion.  d_out[j*16 + 4*c + 0..3] holds,
 * for c = r_s, r_p, t_s, t_p: (re, im) of dc/dthk_j, then 2 unused slots. */
void orc_tmm_dthk(int n_layers, const double* thk_nm, const double* nre, const double* nim,
                  double n_in, double nout_re, double nout_im,
                  double lambda_nm, double kappa, double* d_out);

/* Angle table (Methods, memory-saving strategies: the thin-film response is
 * precomputed on a discrete set of incidence angles and interpolated,
 * differentiably, in between).  Reading: n angles theta_j = j (pi/2)/(n-1)
 * in the glass, a Catmull-Rom cubic in theta through the four angles around
 * theta; the response is even in theta, so the angle before theta_0 is
 * theta_1, and the last segment repeats theta_{n-1}.  A coefficient is
 * sum_i w[i] c(theta_{idx[i]}).  n >= 4; theta in [0, pi/2]. */
void orc_table_weights(double theta, int n, int idx[4], double w[4]);

/* ------------------------------------------------------------------ scene */
typedef struct {
    /* refractive-index table, [n_lambda][n_mat] */
    int32_t n_lambda, n_mat;
    const double* lambda_nm;
    const double* n_re;
    const double* n_im;
    /* slab */
    double T, Lx, eye_relief;
    int32_t mat_glass, mat_air;
    double pupil_x0, pupil_w, pupil_h;
    double eye_x0, eye_y0, eye_w, eye_h;
    int32_t bins_x, bins_y;
    /* mirrors */
    int32_t n_mirrors;
    double tilt_deg, pitch, center_x;
    const double* omega;            /* [M] reflection probability */
    /* stacks, [D][M][Lmax] */
    int32_t n_designs, max_layers;
    const double* thk;
    const uint8_t* mat;
    const int32_t* n_layers;        /* [D][M] */
    /* rays */
    int32_t n_lsel;
    const int32_t* lambda_sel;      /* [n_lsel] indices into the table */
    int32_t fov_mode;               /* 0 grid, 1 uniform random per ray */
    int32_t n_fov;
    const double* fov_deg;          /* grid: [F][2]; random: [[xlo,xhi],[ylo,yhi]] */
    int64_t rays_per_point;
    int32_t max_events;
    int32_t fp_shift;
    uint64_t seed, step;
    /* thin film per mirror hit: 0 = the exact response at the hit's angle;
     * n >= 4 = interpolated from an n-angle table (orc_table_weights) */
    int32_t table_nodes;
    /* eye pupils (Results, "System Architecture": a grid of pupil positions
     * in the eyebox, one image per pupil).  0: the eyebox is binned on the
     * bins_x x bins_y grid.  n > 0: the eyebox plane holds n circular pupils
     * of radius eye_pupil_r (mm) centred at eye_pupil_xy[2 p], [2 p + 1];
     * a ray whose crossing (x, y) of that plane satisfies
     * (x - cx)^2 + (y - cy)^2 < r^2 lands in pupil p (the pupils must not
     * overlap), and "bin" p is pupil p: bins_x = n, bins_y = 1. */
    int32_t n_eye_pupils;
    double eye_pupil_r;
    const double* eye_pupil_xy;
    /* the designs are designs first_design, ... of a larger batch: a ray's
     * random stream is that of its id in the batch, (((first_design + d)
     * n_lsel + l) F + f) rays_per_point + i; ray ids passed to and returned
     * by these functions stay the call's own */
    int32_t first_design;
} orc_scene;

/* Termination categories. */
enum { ORC_EYEBOX = 0, ORC_MISS = 1, ORC_LEAK = 2, ORC_END = 3, ORC_TRUNC = 4,
       ORC_LOST = 5, ORC_FACE_R = 6, ORC_NCAT = 8 };

/* Per-ray record (sampled parity). */
typedef struct {
    int64_t ray_id;
    int32_t bin;          /* flat bin index within the point, -1 if none */
    int32_t category;
    int32_t n_events;     /* ray-surface interactions */
    int32_t n_prma;       /* mirror hits */
    double w;             /* final |E|^2 (at the eyebox, or where the ray ended) */
    double exit_dir[3];   /* direction in air after leaving the top face */
    double exit_pos[3];
} orc_ray_record;

/* Statistics: counters[0..] = rays, interactions, prma_hits, saturated,
 * then per category counts [4 + c]; power[c] = summed weight per category. */
typedef struct {
    int64_t counters[16];
    double power[ORC_NCAT];
} orc_stats;

/* Full forward: every ray of every (design, lambda, fov) point.
 * q_bins, counts, wsum have shape [D][n_lsel][F][bins_y][bins_x] (any may be NULL). */
int orc_trace_forward(const orc_scene* sc, uint64_t* q_bins, uint32_t* counts,
                      double* wsum, orc_stats* stats);

/* Trace the listed rays only (global ray ids), writing one record each. */
int orc_trace_rays(const orc_scene* sc, int64_t n, const int64_t* ray_ids, orc_ray_record* rec);

/* Event log of one ray for geometry tests: up to cap events of
 * (type, surface, x, y, z, dx, dy, dz, aoi_deg, branch). Returns count. */
int orc_ray_events(const orc_scene* sc, int64_t ray_id, int cap, double* ev10);

/* Adjoint: dL/dthk[D][M][Lmax] for dL/dI given per bin (same shape as bins).
 * Only rays with ray_id % sample_stride == 0 contribute when stride > 1
 * (the matching forward is then the sampled one). */
int orc_trace_backward(const orc_scene* sc, const double* dL_dI, int64_t sample_stride,
                       double* grad);

/* Sampled forward matching orc_trace_backward's sampling: irradiance of the
 * rays with ray_id % stride == 0, normalised by the full per-point ray count. */
int orc_trace_forward_sampled(const orc_scene* sc, int64_t sample_stride, double* irr);

/* Brute-force deterministic splitting of the births [first, first + n) of
 * point (d, l, f): exact expected bin power sum_paths |E_path|^2 (no
 * sampling), summed per bin. */
int orc_split_bruteforce(const orc_scene* sc, int32_t d, int32_t lsel, int32_t f,
                         int64_t first, int64_t n_rays, double* bin_power, int64_t* n_paths);

/* Monte Carlo weight of one birth under a forced decision sequence
 * (bit k = 1 means "reflect" at the k-th mirror hit).  Returns the bin (-1 if
 * none) and writes the weight and the path probability. */
int orc_trace_forced(const orc_scene* sc, int64_t ray_id, uint64_t decisions, int n_decisions,
                     double* w, double* prob, int* n_used);

/* One field-changing event in isolation (polarization pins): a ray of point
 * (d, li, fov 0) with direction dir_in[3] and field E_in[6] ((re, im) of x,
 * y, z) meets `surface`: a mirror index (branch `reflect`, no Monte Carlo
 * rescaling) or ORC_SURF_TOP / ORC_SURF_BOTTOM (total internal reflection,
 * exit or leak, as in the trace).  Writes the outgoing direction and field;
 * returns the event type (1 TIR, 2 exit, 3 leak, 5 mirror), < 0 on a bad
 * argument. */
enum { ORC_SURF_TOP = 1000, ORC_SURF_BOTTOM = 1001 };
int orc_event_probe(const orc_scene* sc, int32_t d, int32_t li, int32_t surface, int32_t reflect,
                    const double dir_in[3], const double E_in[6], double dir_out[3], double E_out[6]);

/* --------------------------------------------------------------- the loss */
/* irr: [D][n_l][F][B] irradiance.  kind 0: -mean eta + w_e Var_eyebox + w_f Var_fov;
 * kind 1: -mean eta + w_f CV_fov + w_e CV_eyebox (Eq. 1); kind 2: Eq. 1 on
 * pupil images (B = pupils): -mean over (wavelength, FoV, pupil) of I +
 * w_f CV_fov + w_e CV_pupils.  Returns L, writes dL/dI. */
double orc_loss(const double* irr, int32_t D, int32_t n_l, int32_t F, int32_t B,
                int32_t kind, double w_f, double w_e, double* dL_dI);

#ifdef __cplusplus
}
#endif
#endif
