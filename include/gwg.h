/*
 * gwg.h — C ABI of the MI355X (gfx950) differentiable Monte Carlo
 * polarization ray trace through a geometric waveguide.
 *
 * The operations follow arXiv 2601.04370 (Methods):
 *   - gwg_tmm_rt: effective Fresnel coefficients of a multilayer coating,
 *     "Multilayer thin-film solver" (Eq. 3 interface coefficients, Eq. 4 Airy
 *     sums, transfer-matrix method);
 *   - gwg_trace_forward: non-sequential Monte Carlo polarization ray trace,
 *     "Polarization ray tracing" (Eq. 5) and "Differentiable Monte Carlo
 *     non-sequential ray tracing" (Eq. 6, incoherent eyebox sum of |E|^2);
 *   - gwg_trace_backward: gradient of a loss on the eyebox irradiance with
 *     respect to every layer thickness through the sampled paths
 *     (reparameterized sampling; two-pass intersection and gradient
 *     checkpointing between the tracer and the thin-film solver);
 *   - gwg_loss: the eyebox loss of Eq. 1 (and its variance form) and its
 *     gradient with respect to the irradiance.
 *
 * Conventions shared by every entry point
 *   - time dependence exp(-i w t); complex index N = n + i k with k >= 0
 *     absorbing.  Lossless results are the complex conjugates of Eq. 4 as
 *     printed (which uses exp(-2 i delta)); |r|^2, |t|^2 are identical.
 *   - r_s, r_p, t_s, t_p are field-amplitude ratios in the convention of
 *     Eq. 3 (p unit vector = k x s for each wave), so r_p(0) = -r_s(0).
 *   - lengths: geometry in mm, wavelengths and thicknesses in nm.
 *   - "device" pointers are HIP device memory of the context's GPU, owned by
 *     the caller; "host" pointers are read during the call only.
 *   - all work is enqueued on `stream` (a hipStream_t, NULL = default
 *     stream) and is asynchronous unless a host output is requested.
 *
 * Errors: every call returns a gwg_status.  Arguments are validated on the
 * host before anything is enqueued; on GWG_E_INVAL nothing was launched.
 * gwg_last_error() gives a message for the last failing call on a context.
 * A context is used by one host thread at a time.
 */
#ifndef GWG_H
#define GWG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GWG_ABI_VERSION 2

typedef struct gwg_ctx gwg_ctx;   /* opaque; owns scratch memory and scene tables */

typedef enum {
    GWG_OK = 0,
    GWG_E_INVAL = 1,        /* invalid argument; nothing was launched */
    GWG_E_NOMEM = 2,        /* device allocation failed */
    GWG_E_HIP = 3,          /* HIP runtime error (message in gwg_last_error) */
    GWG_E_STATE = 4,        /* call out of order (e.g. backward without forward) */
    GWG_E_OVERFLOW = 5,     /* fixed-point bin saturated (only reported with stats) */
    GWG_E_NODEVICE = 6      /* no usable gfx950 device for this context */
} gwg_status;

typedef enum {
    GWG_FP64 = 0,           /* every step in double precision */
    GWG_FP32_MIXED = 1,     /* thin-film solve in single precision, re-solved in
                               double precision for hits within 2 degrees of the
                               critical angle of a layer material (the only
                               re-solve rule); geometry, fields, the adjoint and
                               reductions in double precision.  Does not reach
                               |dR| <= 1e-5 on every hit of long stacks: their
                               resonances, not the critical angle, carry the
                               largest single-precision errors */
    GWG_FP32 = 2            /* thin-film solve in single precision, no re-solve
                               (diagnostics: measures the single-precision error) */
} gwg_precision;

/* Refractive-index table (host): n_re/n_im are [n_lambda][n_mat]. */
typedef struct {
    int32_t n_lambda, n_mat;
    const double* lambda_nm;    /* [n_lambda] vacuum wavelengths, nm, > 0 */
    const double* n_re;         /* [n_lambda][n_mat] real part, > 0 */
    const double* n_im;         /* [n_lambda][n_mat] extinction, >= 0 */
} gwg_materials;

/* ------------------------------------------------------------ lifecycle */
/* Create a context on HIP device `device`.  Returns GWG_E_NODEVICE if the
 * device does not exist or is not gfx950.  *out is NULL on failure. */
int gwg_create(gwg_ctx** out, int32_t device);
/* Release the context and every device buffer it owns (synchronizes). */
int gwg_destroy(gwg_ctx* ctx);
/* Message of the last failing call on ctx (never NULL; "" if none).  Valid
 * until the next call on ctx.  With ctx == NULL, the last gwg_create error. */
const char* gwg_last_error(const gwg_ctx* ctx);
/* ABI version (GWG_ABI_VERSION). */
int32_t gwg_abi_version(void);
/* Hash of the sources this library was built from: 16 hex digits of the
 * SHA-256 over its kernel, host and header files and compile flags (fixed
 * order), so that a caller can check that the library matches the sources
 * beside it.  Static string, never NULL. */
const char* gwg_source_hash(void);

/* ------------------------------------------------------------ thin film */
/* One coating stack in incidence order. */
typedef struct {
    int32_t n_layers;           /* 0 <= n_layers <= 4096 */
    const double* thk_nm;       /* device [n_layers], >= 0 */
    const uint8_t* mat;         /* host [n_layers], indices into the material table */
    int32_t mat_in, mat_out;    /* incident (lossless) and exit media */
} gwg_stack;

/* Effective coefficients of one stack for n_q queries (Methods, thin-film
 * solver; Eq. 3 amplitude convention).  Query q uses wavelength index
 * d_lambda_idx[q] (device int32, < n_lambda) and angle of incidence
 * d_theta[q] (device f64, radians, in [0, pi/2)) in the incident medium.
 * d_out (device f64 [n_q][8]) receives r_s, r_p, t_s, t_p as (re, im).
 * precision: GWG_FP64 or GWG_FP32 (GWG_FP32_MIXED applies the tracer's
 * re-solve rule).  Out-of-range indices in device arrays give NaN outputs. */
int gwg_tmm_rt(gwg_ctx* ctx, const gwg_stack* stack, const gwg_materials* mats,
               int64_t n_q, const int32_t* d_lambda_idx, const double* d_theta,
               int32_t precision, double* d_out, void* stream);

/* ---------------------------------------------------------------- trace */
/* Slab: glass 0 <= z <= T_mm, 0 <= x <= L_mm, unbounded in y; rays enter
 * through the top-face window [pupil_x0, pupil_x0 + pupil_w] x
 * [-pupil_h/2, pupil_h/2]; they are binned on the plane z = T + eye_relief
 * over the rectangle [eye_x0, eye_x0 + eye_w) x [eye_y0, eye_y0 + eye_h).
 *
 * Eye pupils (Results, "System Architecture": a grid of pupil positions in
 * the eyebox, whose images are the objective): with n_eye_pupils > 0 the
 * eyebox plane holds that many circular pupils of radius
 * eye_pupil_radius_mm centred at eye_pupil_xy_mm[2 p], [2 p + 1] (host,
 * mm), and the "bins" are the pupils instead of the grid: a ray crossing the
 * plane at (x, y) lands in pupil p when (x - cx)^2 + (y - cy)^2 < r^2, and
 * every eyebox output holds one value per pupil (bins_x must equal
 * n_eye_pupils and bins_y 1; the eye_x0..eye_h rectangle is then unused).
 * Pupils must not overlap (centre distances >= 2 r), so a ray lands in at
 * most one.  With n_eye_pupils = 0 the other two fields are ignored. */
typedef struct {
    double T_mm, L_mm, eye_relief_mm;
    int32_t mat_glass, mat_air;
    double pupil_x0_mm, pupil_w_mm, pupil_h_mm;
    double eye_x0_mm, eye_y0_mm, eye_w_mm, eye_h_mm;
    int32_t bins_x, bins_y;     /* 1..4096 each */
    int32_t n_eye_pupils;       /* 0 (eyebox grid) or 1..64 */
    double eye_pupil_radius_mm; /* > 0 with pupils */
    const double* eye_pupil_xy_mm;  /* host [n_eye_pupils][2] */
} gwg_slab;

/* Partially reflective mirror array: n_mirrors (1..16) parallel planes with
 * normal (-sin tilt, 0, cos tilt) through (center_x + (m - (M-1)/2) pitch, ., T/2),
 * spanning the slab thickness.  omega[m] in (0, 1) is the probability of
 * sampling the reflected branch at mirror m (Eq. 6). */
typedef struct {
    int32_t n_mirrors;
    double tilt_deg, pitch_mm, center_x_mm;
    const double* omega;        /* host [n_mirrors] */
} gwg_prma;

/* Coating stacks of n_designs candidate designs.  Layer 0 faces the +normal
 * side of its mirror; a hit from the -normal side sees the reverse order.
 * Slots j >= n_layers[d][m] are padding and ignored. */
typedef struct {
    int32_t n_designs, n_mirrors, max_layers;   /* max_layers 1..1024 */
    const double* thk_nm;       /* device [D][M][Lmax] f64, >= 0 */
    const uint8_t* mat;         /* host [D][M][Lmax] material indices */
    const int32_t* n_layers;    /* host [D][M], 0..max_layers */
} gwg_stacks;

/* Ray batch: every (design, selected wavelength, FoV point) gets
 * rays_per_point rays.  fov_mode 0: fov_deg is [n_fov][2] (theta_x, theta_y)
 * field angles in degrees; fov_mode 1: one point whose rays draw field
 * angles uniformly in fov_deg = [[x_lo, x_hi], [y_lo, y_hi]] (n_fov = 1).
 * A field angle (tx, ty) is the direction normalize(tan tx, tan ty, 1) in
 * air at the eye. */
typedef struct {
    int32_t n_lambda_sel;
    const int32_t* lambda_sel;  /* host [n_lambda_sel] indices into the table */
    int32_t fov_mode;
    int32_t n_fov;
    const double* fov_deg;      /* host */
    int64_t rays_per_point;     /* 1 .. 2^40 */
    int32_t max_events;         /* 1..256 ray-surface interactions per ray */
    int32_t first_design;       /* >= 0: the call's designs are designs first_design,
                                   first_design + 1, ... of a larger batch, and draw that
                                   batch's random streams (a batch traced in chunks of
                                   designs gives the same results as in one call) */
} gwg_rays;

/* Eyebox outputs, device arrays of shape [D][n_lambda_sel][F][bins_y][bins_x]
 * (F = n_fov, or 1 in fov_mode 1).  q_bins accumulates round-half-even(w 2^fp_shift)
 * per ray (per-ray value clamped at 2^40), counts the number of rays
 * landing in the bin (geometry only).  irradiance (optional, may be NULL)
 * receives q_bins 2^-fp_shift / rays_per_point.  Every output is
 * overwritten. */
typedef struct {
    uint64_t* q_bins;
    uint32_t* counts;
    double* irradiance;
    int32_t fp_shift;           /* 0..40 */
} gwg_eyebox;

/* Per-ray record for sampled comparisons: written for ray ids
 * id = k * record_stride into records[k]. */
typedef struct {
    int32_t bin;        /* flat bin within its point, -1 if not binned */
    int32_t category;   /* GWG_CAT_* */
    int32_t n_events;   /* ray-surface interactions */
    int32_t n_prma;     /* mirror hits */
    double w;           /* final |E|^2 */
} gwg_ray_record;

enum { GWG_CAT_EYEBOX = 0, GWG_CAT_MISS = 1, GWG_CAT_LEAK = 2, GWG_CAT_END = 3,
       GWG_CAT_TRUNC = 4, GWG_CAT_LOST = 5, GWG_CAT_FACE_R = 6, GWG_NCAT = 8 };

/* Counters of one call.  Forward: rays traced, ray-surface interactions,
 * mirror hits, layer steps (sum over hits of the stack's layer count),
 * hits solved in double precision, saturated bin contributions, terminations
 * and final power per category.  Backward: the same for the regenerated
 * paths (only rays that end in a bin with nonzero dL/dI are regenerated past
 * their geometry), plus rays / hits / layer steps that went through the
 * adjoint, and of those layer steps the ones whose exit-to-incident sweep
 * the forward had stored (ck_entries_per_ray). */
typedef struct {
    int64_t rays, interactions, prma_hits, layer_steps, fp64_hits, saturated;
    int64_t adjoint_rays, adjoint_hits, adjoint_layer_steps;
    int64_t n_cat[GWG_NCAT];
    double power[GWG_NCAT];     /* summed final |E|^2 per category (fixed-point, 2^-24) */
    int64_t adjoint_stored_layer_steps;
} gwg_stats;

/* Forward Monte Carlo trace of the whole batch (Methods; Eq. 5, Eq. 6).
 * Ray id = (((first_design + d) * n_lambda_sel + l) * F + f) * rays_per_point + i
 * draws its random numbers from Philox4x32-10 with key (seed_lo, seed_hi ^ step_lo),
 * counter (id_lo, id_hi, block, tag): tag 0 block 0 gives the birth words,
 * tag 1 block h/4 the word of the h-th mirror hit.  step < 2^32.
 * flags: 0 or GWG_FWD_GRAD with at most one of GWG_FWD_MEMO,
 * GWG_FWD_TABLE.  With GWG_FWD_GRAD
 * (a gwg_trace_backward will follow) the trace also runs the path part of the adjoint for every ray
 * that reaches the eyebox and keeps one entry per mirror hit in the context
 * (about 48 bytes per hit, within a fixed memory budget); the backward then
 * only runs the thin-film adjoints.  Without it (or beyond the budget) the
 * backward regenerates the paths.  Results are identical either way.
 * records: optional device array (NULL to skip) with record_stride >= 1.
 * stats: optional host struct; when given the call synchronizes the stream
 * and returns GWG_E_OVERFLOW if any bin contribution saturated.
 * The context remembers the scene, seed, step, precision and thk pointer
 * for gwg_trace_backward; thk must not change in between. */
#define GWG_FWD_GRAD 1u
/* GWG_FWD_MEMO: hit keys are memoized per work item (one design, wavelength
 * and FoV point; within it the collimated rays share a few keys).  The
 * forward solves each distinct (kappa, mirror, side) key once and reuses its
 * coefficients, which are those of the per-hit solve bit for bit, so the bins
 * are identical (fov_mode 0 only; with fov_mode 1, or where the key tables do
 * not fit in LDS, the forward solves per hit).  With GWG_FWD_GRAD the
 * backward solves one thin-film adjoint per distinct (kappa, mirror, side,
 * branch) key, with the key's summed cotangents, instead of one per mirror
 * hit (exact by linearity, up to summation order; the sums run in a fixed
 * order). */
#define GWG_FWD_MEMO 2u
/* GWG_FWD_TABLE: the thin-film response is precomputed per (design,
 * wavelength, mirror, side) at n = table_nodes incidence angles
 * theta_j = j (pi/2)/(n-1) in the glass, and every hit interpolates it with a
 * Catmull-Rom cubic in its angle (Methods, memory-saving strategies; the
 * response is even in theta below theta_0, the last segment is clamped).
 * The results are those of the interpolated model, not of the per-hit solve.
 * The table takes 64 * D * n_lambda_sel * M * 2 * n bytes of device memory
 * (GWG_E_INVAL if it does not fit in half of the free memory).  With
 * GWG_FWD_GRAD, gwg_trace_backward returns the exact gradient of the
 * interpolated model: the hits' cotangents are summed per table entry in
 * 64-bit fixed point (exact, order-independent), and one thin-film adjoint
 * runs per entry with a nonzero sum.  A table forward without GWG_FWD_GRAD
 * has no backward (GWG_E_STATE).  Excludes GWG_FWD_MEMO. */
#define GWG_FWD_TABLE 4u
int gwg_trace_forward(gwg_ctx* ctx, const gwg_slab* slab, const gwg_prma* prma,
                      const gwg_materials* mats, const gwg_stacks* stacks,
                      const gwg_rays* rays, uint64_t seed, uint64_t step,
                      int32_t precision, uint32_t flags, const gwg_eyebox* out,
                      gwg_ray_record* records, int64_t record_stride,
                      gwg_stats* stats, void* stream);

/* Learned reflection probabilities (Methods): gradient, with respect to
 * every mirror's reflection probability omega_m, of
 *     J = sum over (design, wavelength, FoV) points and bins of W * I
 * in the scalar-reflectance model (each coating idealised as reflecting the
 * fraction omega_m of the incident energy, geometry only, no polarization),
 * whose irradiance is I = counts / rays_per_point.  Score-function
 * estimator on the paths of the last gwg_trace_forward (same seed, step and
 * decisions; its thk must still be valid):
 *     dJ/domega_m = sum_points 1/N sum_rays (W_bin - beta) S_m,
 * S_m = sum over the ray's hits on mirror m of 1/omega_m (reflected) or
 * -1/(1 - omega_m) (transmitted), beta = the point's J (an unbiased
 * baseline since E[S_m] = 0), omega_m = the sampling probability
 * floor(omega 2^32) / 2^32; a ray outside the eyebox has W = 0.
 * d_W: device f64 [D][n_lambda_sel][F][bins_y][bins_x] (1 for throughput, or
 * dL/dI of any loss of I); d_counts: device u32 counts of that forward;
 * d_grad: device f64 [M].  Deterministic (fixed-order sums). */
int gwg_omega_gradient(gwg_ctx* ctx, const double* d_W, const uint32_t* d_counts, double* d_grad,
                       void* stream);

/* *kept = 1 if the last gwg_trace_forward (or the one recorded by a stream
 * capture) stored adjoint entries, so that gwg_trace_backward runs the
 * thin-film adjoints only; 0 if the backward will regenerate the paths. */
int gwg_forward_kept_entries(const gwg_ctx* ctx, int32_t* kept);

/* Gradient of a loss with respect to every layer thickness, given
 * d_dL_dI (device f64, the eyebox shape of the last forward).  The sampled
 * paths of the last forward are used: when that forward ran with
 * GWG_FWD_GRAD, the backward reads the adjoint entries it stored (and their
 * stored sweep checkpoints) and runs only the thin-film adjoints; items whose
 * entries did not fit, or a forward without GWG_FWD_GRAD, have their paths
 * regenerated from the same seed and step.  Either way the result is the
 * pathwise derivative of the unquantized estimator I = sum w /
 * rays_per_point.  d_grad: device f64 [D][M][max_layers],
 * overwritten (padding slots get 0).  sample_stride >= 1: only rays with
 * id % sample_stride == 0 contribute (1 = all rays).  Deterministic: the
 * same inputs give bit-identical gradients.  stats: optional host struct
 * (synchronizes the stream). */
int gwg_trace_backward(gwg_ctx* ctx, const double* d_dL_dI, double* d_grad,
                       int64_t sample_stride, gwg_stats* stats, void* stream);

/* Eyebox loss (Eq. 1) and dL/dI for irradiance d_irr (device f64,
 * [D][n_l][F][B]), summed over designs.  kind 0: -mean(eta) + w_e Var_b(E_b)
 * + w_f Var_f(phi_f); kind 1: -mean(eta) + w_f CV_f + w_e CV_b, with
 * eta = sum_b I (per wavelength and FoV point), E_b the mean of I over
 * wavelengths and FoV points, phi_f the mean of eta over wavelengths,
 * population moments; kind 2 (pupil images, B = pupils): kind 1 with the
 * brightness term -mean(eta) / B, the mean of I over wavelengths, FoV
 * points and pupils (with the same number of wavelengths per colour
 * channel, also the mean over colour channels).  d_loss: device f64 [1]; d_dL_dI: device f64, same
 * shape as d_irr (may be NULL).  Fixed-order reductions: deterministic. */
int gwg_loss(gwg_ctx* ctx, const double* d_irr, int32_t D, int32_t n_l, int32_t F,
             int32_t B, int32_t kind, double w_f, double w_e, double* d_loss,
             double* d_dL_dI, void* stream);

/* gwg_loss without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and results (bit for bit) as
 * gwg_loss; its work buffer is a fixed 4 MiB device array inside the library
 * (one per GPU, held until the process ends, its address looked up when a
 * context is created on that GPU) instead of context memory.  The shape must
 * satisfy D * (n_l * F + B + F + 8) <= 524288, else GWG_E_INVAL (nothing is
 * launched; gwg_loss has no such limit).  Every call on one GPU shares that
 * array, whichever context or stream it comes from: calls that overlap in
 * time on one GPU (different streams, or different host threads) race and
 * give wrong results; serialize them.  The caller still provides d_irr,
 * d_loss and d_dL_dI. */
int gwg_loss_noalloc(gwg_ctx* ctx, const double* d_irr, int32_t D, int32_t n_l, int32_t F,
                     int32_t B, int32_t kind, double w_f, double w_e, double* d_loss,
                     double* d_dL_dI, void* stream);

/* ---------------------------------------------------------------- tuning */
/* Launch parameters of the trace kernels (0 = automatic).  rays_per_block
 * is the tile of rays of one (design, wavelength, FoV) point handled by a
 * workgroup; block_threads is 64, 128 or 256 (adjoint: 64 or 128).
 * adj_entries_per_ray (0..64, 0 = 8) sizes the adjoint entry regions of
 * GWG_FWD_GRAD: a region holding more entries than this times its rays is
 * regenerated by the backward instead.  memo_keys (0..128, 0 = 128) is the
 * capacity of each wave's key table in the memoized forward (GWG_FWD_MEMO):
 * a wave meeting more keys in one work item solves the rest of it per hit.
 * table_nodes (0 = 8192, else 4..2^20) is the number of incidence angles of
 * the angle table (GWG_FWD_TABLE).  ck_entries_per_ray (0 = 4, -1 = none,
 * else 1..64): with GWG_FWD_GRAD at FP64 on lossless stacks, the forward
 * solve keeps the adjoint's sweep checkpoints (8 doubles every 32 layers
 * of a hit whose layers all propagate, every 16 of one that meets an
 * evanescent layer) for up to this many entries per ray of each entry
 * region, within a memory budget (the smaller of 128 GiB and half the free
 * memory), so the backward skips that sweep for them; the gradient is the
 * same bit for bit. */
typedef struct {
    int32_t block_threads;
    int64_t rays_per_block;
    int32_t bwd_block_threads;
    int64_t bwd_rays_per_block;
    int32_t adj_entries_per_ray;
    int32_t memo_keys;
    int32_t table_nodes;
    int32_t ck_entries_per_ray;
} gwg_tuning;

int gwg_set_tuning(gwg_ctx* ctx, const gwg_tuning* tuning);
int gwg_get_tuning(const gwg_ctx* ctx, gwg_tuning* tuning);

/* Device step counter for captured graphs.  With d_step != NULL (device
 * uint32, owned by the caller) the trace kernels draw their Philox key from
 * (seed_lo, seed_hi ^ (step + *d_step)), reading *d_step when they start, so
 * a graph that captured forward, loss and backward with a fixed `step` draws
 * fresh paths on every replay if it also advances *d_step after the
 * backward.  Forward and backward of one step must see the same value.
 * NULL restores the plain step argument.  During stream capture the trace,
 * loss and backward calls allocate nothing and synchronize nothing: every
 * buffer must have been sized by the same call made once before capturing
 * (else GWG_E_STATE), and stats cannot be requested. */
int gwg_set_step_source(gwg_ctx* ctx, const uint32_t* d_step);

/* Autotuner.  Times the forward trace of this scene (same arguments as
 * gwg_trace_forward, step 0) for workgroup sizes 256/128 and ray tiles of
 * 1/4 to 4 times the automatic tile (with GWG_FWD_GRAD: forward plus
 * adjoint with dL/dI = 1, since the adjoint runs on the forward's tiles),
 * checks that the eyebox bins are bit-identical across them (scenes of up
 * to 2^24 bins), then times the adjoint for adjoint workgroup sizes 128/64,
 * and keeps the
 * fastest as the context's tuning (*out).  Results are cached in the
 * context by scene signature (scene tables, precision, flags, device) and,
 * with cache_path != NULL, read from and appended to that text file.  Runs
 * several full traces and synchronizes the stream.  Leaves no forward for
 * gwg_trace_backward. */
int gwg_autotune(gwg_ctx* ctx, const gwg_slab* slab, const gwg_prma* prma,
                 const gwg_materials* mats, const gwg_stacks* stacks,
                 const gwg_rays* rays, uint64_t seed, int32_t precision,
                 uint32_t flags, const char* cache_path, gwg_tuning* out,
                 void* stream);

/* ---------------------------------------------------------------- timing */
/* Kernel timing for measurement.  While enabled, the library records a HIP
 * event on the caller's stream right before and right after each launch of
 * the forward trace kernel and of the adjoint trace kernel, in a ring of
 * GWG_TIMING_RING launches per kernel.  Enabling (again) clears the rings.
 * gwg_kernel_times writes the durations in milliseconds of the last n
 * launches of `kernel` (GWG_KERNEL_FORWARD or GWG_KERNEL_ADJOINT), oldest
 * first; it waits for those events.  Errors: GWG_E_INVAL for a bad kernel id,
 * n < 1, n > GWG_TIMING_RING, or n larger than the launches recorded since
 * timing was enabled; GWG_E_STATE when timing is off. */
enum { GWG_KERNEL_FORWARD = 0, GWG_KERNEL_ADJOINT = 1, GWG_TIMING_RING = 64 };
int gwg_set_timing(gwg_ctx* ctx, int32_t enable);
int gwg_kernel_times(gwg_ctx* ctx, int32_t kernel, int32_t n, double* ms_out);

#ifdef __cplusplus
}
#endif
#endif /* GWG_H */
