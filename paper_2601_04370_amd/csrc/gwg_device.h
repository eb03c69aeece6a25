// Device building blocks for gfx950: complex arithmetic, Philox4x32-10,
// sine/cosine, and the per-hit characteristic-matrix thin-film solve with its
// adjoint.  Included by the kernel translation unit only.
//
// Thin-film solve (Methods, "Multilayer thin-film solver"): for a stack of
// layers j = 0..L-1 in incidence order between an incident medium 0 and an
// exit medium, with invariant kappa = n_0 sin(theta_0) and
// z_j = N_j^2 - kappa^2, each layer is the 2x2 characteristic matrix
//     M_j = [[cos d_j, -i sin d_j / eta_j], [-i eta_j sin d_j, cos d_j]],
//     d_j = k0 q_j t_j,  q_j = sqrt(z_j) (Im >= 0),
//     eta_j = q_j (s) or N_j^2 / q_j (p)       [exp(-i w t) convention],
// and [B; C] = M_0 M_1 ... M_{L-1} [1; eta_exit].  The Eq. 3-convention
// coefficients are r_s = (eta_0 B - C)/(eta_0 B + C), t_s = 2 eta_0/(eta_0 B + C),
// r_p = -(same with p admittances), t_p = (2 eta_0/(...)) cos(theta_0)/cos(theta_exit).
//
// For a lossless layer the matrix entries are real multiples of 1 and -i
// whether the layer is propagating (z > 0: circular functions) or evanescent
// (z < 0: hyperbolic functions), so the chain runs on real coefficients
// [[C, -i X], [-i Y, C]] with per-polarization real X, Y.  Absorbing layers
// take a general complex path.
//
// Derivative (adjoint): dM_j/dt_j = M_j D_j with the constant generator
//     D_s = -i k0 [[0, 1], [z_j, 0]],   D_p = -i k0 [[0, z_j/N_j^2], [N_j^2, 0]],
// so for a coefficient c with cotangent row rho = dc/d[B; C],
//     dc/dt_j = u_{j-1}^T D_j w_j,  u_{j-1}^T = rho^T M_0..M_{j-1},  w_j = M_j..M_{L-1}[1; eta_exit].
// The covector u runs from the incident side, the vector w from the exit
// side; w is recomputed segment by segment from checkpoints stored during a
// first exit-to-incident sweep, which keeps both recurrences in their
// numerically stable direction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gwg_trig_poly.h"

namespace gwg {

// ---------------------------------------------------------------- complex
struct cd { double re, im; };
__device__ __host__ inline cd mk(double r, double i) { cd z; z.re = r; z.im = i; return z; }
__device__ inline cd cadd(cd a, cd b) { return mk(a.re + b.re, a.im + b.im); }
__device__ inline cd csub(cd a, cd b) { return mk(a.re - b.re, a.im - b.im); }
__device__ inline cd cmul(cd a, cd b) { return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
__device__ inline cd cscale(cd a, double s) { return mk(a.re * s, a.im * s); }
__device__ inline cd cconj(cd a) { return mk(a.re, -a.im); }
__device__ inline cd cdiv(cd a, cd b)
{
    // Smith's algorithm
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, den = b.re + b.im * r;
        return mk((a.re + a.im * r) / den, (a.im - a.re * r) / den);
    }
    double r = b.re / b.im, den = b.im + b.re * r;
    return mk((a.re * r + a.im) / den, (a.im * r - a.re) / den);
}
__device__ inline cd csqrt_up(cd z)
{
    // principal root rotated to Im >= 0 (and Re >= 0 on the real axis)
    double m = sqrt(z.re * z.re + z.im * z.im);
    double a = sqrt(0.5 * (m + fabs(z.re)));
    cd r;
    if (a == 0.0) return mk(0.0, 0.0);
    if (z.re >= 0.0) r = mk(a, 0.5 * z.im / a);
    else r = mk(0.5 * fabs(z.im) / a, z.im >= 0.0 ? a : -a);
    if (r.im < 0.0 || (r.im == 0.0 && r.re < 0.0)) r = mk(-r.re, -r.im);
    return r;
}

// ------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw, SC'11: ten rounds of the 4x32 Philox S-box,
// multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85.
struct u32x4 { uint32_t x, y, z, w; };
__device__ inline u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                 uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    u32x4 r; r.x = c0; r.y = c1; r.z = c2; r.w = c3;
    return r;
}
__device__ inline double u24(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

// ------------------------------------------------------------ sin / cos
// Phases here are finite and moderate (|x| < 1e4).  Reduction by multiples
// of pi/2 with a two-term Cody-Waite split (each product subtracted with one
// FMA), then Taylor polynomials of sin and cos on [-pi/4, pi/4]: truncation
// below 1e-16 (f64, degree 15/16) or 2e-9 (f32, degree 9/8).
constexpr double inv_fact(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= (double)i; return 1.0 / f; }

__device__ inline void sincos_cw(double x, double* s, double* c)
{
#pragma clang fp contract(fast)
    const double two_over_pi = 0.63661977236758134308;
    const double pio2_hi = 1.5707963267948966;          // nearest double to pi/2
    const double pio2_lo = 6.123233995736766e-17;       // pi/2 - pio2_hi
    double n = rint(x * two_over_pi);
    double r = fma(-n, pio2_hi, x);
    r = fma(-n, pio2_lo, r);
    double r2 = r * r;
    double ps = inv_fact(15);
    ps = fma(ps, -r2, inv_fact(13));
    ps = fma(ps, -r2, inv_fact(11));
    ps = fma(ps, -r2, inv_fact(9));
    ps = fma(ps, -r2, inv_fact(7));
    ps = fma(ps, -r2, inv_fact(5));
    ps = fma(ps, -r2, inv_fact(3));
    double sn = fma(-r * r2, ps, r);                    // r - r^3/3! + ...
    double pc = inv_fact(16);
    pc = fma(pc, -r2, inv_fact(14));
    pc = fma(pc, -r2, inv_fact(12));
    pc = fma(pc, -r2, inv_fact(10));
    pc = fma(pc, -r2, inv_fact(8));
    pc = fma(pc, -r2, inv_fact(6));
    pc = fma(pc, -r2, inv_fact(4));
    pc = fma(pc, -r2, inv_fact(2));
    double cs = fma(-r2, pc, 1.0);                      // 1 - r^2/2! + ...
    int q = (int)n & 3;
    double so = (q & 1) ? cs : sn;
    double co = (q & 1) ? sn : cs;
    *s = (q & 2) ? -so : so;
    *c = ((q + 1) & 2) ? -co : co;
}

__device__ inline void sincos_cw(float x, float* s, float* c)
{
#pragma clang fp contract(fast)
    const float two_over_pi = 0.636619772f;
    const float pio2_hi = 1.57079637f;                  // nearest float to pi/2
    const float pio2_lo = -4.37113883e-8f;              // pi/2 - pio2_hi
    float n = rintf(x * two_over_pi);
    float r = fmaf(-n, pio2_hi, x);
    r = fmaf(-n, pio2_lo, r);
    float r2 = r * r;
    float ps = (float)inv_fact(9);
    ps = fmaf(ps, -r2, (float)inv_fact(7));
    ps = fmaf(ps, -r2, (float)inv_fact(5));
    ps = fmaf(ps, -r2, (float)inv_fact(3));
    float sn = fmaf(-r * r2, ps, r);
    float pc = (float)inv_fact(10);
    pc = fmaf(pc, -r2, (float)inv_fact(8));
    pc = fmaf(pc, -r2, (float)inv_fact(6));
    pc = fmaf(pc, -r2, (float)inv_fact(4));
    pc = fmaf(pc, -r2, (float)inv_fact(2));
    float cs = fmaf(-r2, pc, 1.0f);
    int q = (int)n & 3;
    float so = (q & 1) ? cs : sn;
    float co = (q & 1) ? sn : cs;
    *s = (q & 2) ? -so : so;
    *c = ((q + 1) & 2) ? -co : co;
}

// Circular or hyperbolic cosine and sine of a >= 0 with one shared
// polynomial evaluation.  With u = -r^2 (circular) or +r^2 (hyperbolic),
//     sin r or sinh r = r (1 + u P_F(u)),
//     cos r or cosh r = 1 + u P_G(u),
// where P_F and P_G are minimax fits (Remez exchange, degrees 5 and 6 in u)
// of the entire functions the two share, on u in [-(pi/4)^2, (pi/8)^2]
// (gwg_trig_poly.h, written by gen_trig_poly.py; max errors 8e-17 and 1e-18
// before rounding, one term fewer each than truncated Taylor series of the
// same accuracy).  So the dominant Horner evaluation is common to lanes of
// either kind and a wave that mixes propagating and evanescent layers
// executes it once.
// Circular: r = a - n pi/2 (two-term Cody-Waite), then a quadrant rotation.
// Hyperbolic: r = a / 2^k <= pi/8, then k doublings
// (sinh 2r = 2 sinh r cosh r, cosh 2r = cosh^2 r + sinh^2 r).
// The single-precision variant keeps Taylor coefficients 1/n! (degrees 9/10).
__constant__ float kInvFactF[11] = {
    (float)inv_fact(0), (float)inv_fact(1), (float)inv_fact(2), (float)inv_fact(3), (float)inv_fact(4),
    (float)inv_fact(5), (float)inv_fact(6), (float)inv_fact(7), (float)inv_fact(8), (float)inv_fact(9),
    (float)inv_fact(10) };

// HC = false compiles the circular case alone (hyper must then be false):
// the same operations, so the same results, without the hyperbolic branch.
template <bool HC = true>
__device__ inline void gtrig(double a, bool hyper_in, double* C, double* S)
{
#pragma clang fp contract(fast)
    const bool hyper = HC && hyper_in;
    const double two_over_pi = 0.63661977236758134308;
    const double pio2_hi = 1.5707963267948966;
    const double pio2_lo = 6.123233995736766e-17;
    double n = rint(a * two_over_pi);
    int k = 0;
    if (hyper) {
        // smallest k with a / 2^k <= pi/8 (a is finite and moderate)
        int e;
        frexp(a * 2.5464790894703255, &e);      // a / (pi/8) = m 2^e, m in [0.5, 1)
        k = e > 0 ? e : 0;
        n = 0.0;                                 // the quadrant rotation below is then the identity
    }
    // r = a - n pi/2; exactly a on hyperbolic lanes (n = 0), which then
    // scale it by 2^-k (k = 0 leaves circular lanes unchanged)
    double r = fma(-n, pio2_hi, a);
    r = fma(-n, pio2_lo, r);
    if (HC) r = ldexp(r, -k);
    double u = hyper ? r * r : -(r * r);
    double ps = kTrigPolyF[5];
    ps = fma(ps, u, kTrigPolyF[4]);
    ps = fma(ps, u, kTrigPolyF[3]);
    ps = fma(ps, u, kTrigPolyF[2]);
    ps = fma(ps, u, kTrigPolyF[1]);
    ps = fma(ps, u, kTrigPolyF[0]);
    double sn = fma(r * u, ps, r);
    double pc = kTrigPolyG[6];
    pc = fma(pc, u, kTrigPolyG[5]);
    pc = fma(pc, u, kTrigPolyG[4]);
    pc = fma(pc, u, kTrigPolyG[3]);
    pc = fma(pc, u, kTrigPolyG[2]);
    pc = fma(pc, u, kTrigPolyG[1]);
    pc = fma(pc, u, 0.5);
    double cs = fma(u, pc, 1.0);
    // Both kinds run the same straight-line code (no divergent branch): the
    // quadrant rotation (the identity for hyperbolic lanes, whose n is 0),
    // then the doublings (none for circular lanes, whose k is 0).
    // Quadrant q = n mod 4: swap for odd q, then flip signs through the sign
    // bit (S negative for q = 2, 3; C negative for q = 1, 2).
    const unsigned q = (unsigned)(int)n;
    const double so = (q & 1u) ? cs : sn;
    const double co = (q & 1u) ? sn : cs;
    const unsigned fs = (q & 2u) << 30, fc = ((q + 1u) & 2u) << 30;
    sn = __hiloint2double(__double2hiint(so) ^ (int)fs, __double2loint(so));
    cs = __hiloint2double(__double2hiint(co) ^ (int)fc, __double2loint(co));
    for (int i = 0; i < k; ++i) {
        double s2 = 2.0 * sn * cs;
        cs = fma(cs, cs, sn * sn);
        sn = s2;
    }
    *S = sn;
    *C = cs;
}

template <bool HC = true>
__device__ inline void gtrig(float a, bool hyper_in, float* C, float* S)
{
#pragma clang fp contract(fast)
    const bool hyper = HC && hyper_in;
    const float two_over_pi = 0.636619772f;
    const float pio2_hi = 1.57079637f;
    const float pio2_lo = -4.37113883e-8f;
    float n = rintf(a * two_over_pi);
    int k = 0;
    if (hyper) {
        int e;
        frexpf(a * 1.27323954f, &e);
        k = e > 0 ? e : 0;
        n = 0.0f;
    }
    float r = fmaf(-n, pio2_hi, a);
    r = fmaf(-n, pio2_lo, r);
    if (HC) r = ldexpf(r, -k);
    float u = hyper ? r * r : -(r * r);
    float ps = kInvFactF[9];
    ps = fmaf(ps, u, kInvFactF[7]);
    ps = fmaf(ps, u, kInvFactF[5]);
    ps = fmaf(ps, u, kInvFactF[3]);
    float sn = fmaf(r * u, ps, r);
    float pc = kInvFactF[10];
    pc = fmaf(pc, u, kInvFactF[8]);
    pc = fmaf(pc, u, kInvFactF[6]);
    pc = fmaf(pc, u, kInvFactF[4]);
    pc = fmaf(pc, u, kInvFactF[2]);
    float cs = fmaf(u, pc, 1.0f);
    const unsigned q = (unsigned)(int)n;
    const float so = (q & 1u) ? cs : sn;
    const float co = (q & 1u) ? sn : cs;
    sn = __uint_as_float(__float_as_uint(so) ^ ((q & 2u) << 30));
    cs = __uint_as_float(__float_as_uint(co) ^ (((q + 1u) & 2u) << 30));
    for (int i = 0; i < k; ++i) {
        float s2 = 2.0f * sn * cs;
        cs = fmaf(cs, cs, sn * sn);
        sn = s2;
    }
    *S = sn;
    *C = cs;
}

// gtrig with a half-period reduction and the sign left to the caller.
// Circular: a = n pi + r, |r| <= pi/2 (two-term Cody-Waite), and cos a,
// sin a are (-1)^n cos r, (-1)^n sin r; this returns C = cos r, S = sin r
// and adds n to *nsum.  A product of layer matrices [[C, .], [., C]] with
// entries linear in (C, S) then differs from the exact one by (-1)^sum n
// only, which the caller applies once.  No quadrant rotation is needed, at
// the price of longer polynomials (degrees 7 and 7 on u in [-(pi/2)^2,
// (pi/8)^2], max errors 5e-19 and 1e-17 before rounding).  Hyperbolic lanes
// (n = 0) are as in gtrig.
// The work is split in two: trig_reduce takes the argument to (r, u, n, k)
// and trig_eval evaluates the polynomials and the doublings, so a sweep can
// reduce the next layer's argument while it evaluates the current one's
// (the two are independent; the FP64 pipeline then has two chains to
// interleave).  gtrig_half is the two in a row.
struct TrigArg { double r, u, n; int k; };

template <bool HC = true>
__device__ inline TrigArg trig_reduce(double a, bool hyper_in)
{
#pragma clang fp contract(fast)
    const bool hyper = HC && hyper_in;
    const double one_over_pi = 0.31830988618379067154;
    const double pi_hi = 3.141592653589793116;
    const double pi_lo = 1.2246467991473532072e-16;
    double n = rint(a * one_over_pi);
    int k = 0;
    if (hyper) {
        int e;
        frexp(a * 2.5464790894703255, &e);      // a / (pi/8) = m 2^e, m in [0.5, 1)
        k = e > 0 ? e : 0;
        n = 0.0;
    }
    double r = fma(-n, pi_hi, a);
    r = fma(-n, pi_lo, r);
    if (HC) r = ldexp(r, -k);
    TrigArg t;
    t.r = r;
    t.u = hyper ? r * r : -(r * r);
    t.n = n;
    t.k = k;
    return t;
}

template <bool HC = true>
__device__ inline void trig_eval(const TrigArg& t, double* C, double* S, double* nsum)
{
#pragma clang fp contract(fast)
    const double r = t.r, u = t.u;
    // the two Horner chains step in turn: each FP64 step waits on the one
    // before it, so the other chain's step fills the gap
    double ps = kTrigHalfPolyF[7], pc = kTrigHalfPolyG[7];
    ps = fma(ps, u, kTrigHalfPolyF[6]); pc = fma(pc, u, kTrigHalfPolyG[6]);
    ps = fma(ps, u, kTrigHalfPolyF[5]); pc = fma(pc, u, kTrigHalfPolyG[5]);
    ps = fma(ps, u, kTrigHalfPolyF[4]); pc = fma(pc, u, kTrigHalfPolyG[4]);
    ps = fma(ps, u, kTrigHalfPolyF[3]); pc = fma(pc, u, kTrigHalfPolyG[3]);
    ps = fma(ps, u, kTrigHalfPolyF[2]); pc = fma(pc, u, kTrigHalfPolyG[2]);
    ps = fma(ps, u, kTrigHalfPolyF[1]); pc = fma(pc, u, kTrigHalfPolyG[1]);
    ps = fma(ps, u, kTrigHalfPolyF[0]); pc = fma(pc, u, 0.5);
    double sn = fma(r * u, ps, r);
    double cs = fma(u, pc, 1.0);
    if (HC)
        for (int i = 0; i < t.k; ++i) {
            double s2 = 2.0 * sn * cs;
            cs = fma(cs, cs, sn * sn);
            sn = s2;
        }
    *nsum += t.n;
    *S = sn;
    *C = cs;
}

template <bool HC = true>
__device__ inline void gtrig_half(double a, bool hyper_in, double* C, double* S, double* nsum)
{
    trig_eval<HC>(trig_reduce<HC>(a, hyper_in), C, S, nsum);
}

// cosh and sinh of x >= 0 from expm1 (no cancellation for small x)
__device__ inline void coshsinh(double x, double* ch, double* sh)
{
    double em = expm1(x);
    double ep = em + 1.0;
    *sh = 0.5 * em * (em + 2.0) / ep;
    *ch = 1.0 + 0.5 * em * em / ep;
}
__device__ inline void coshsinh(float x, float* ch, float* sh)
{
    float em = expm1f(x);
    float ep = em + 1.0f;
    *sh = 0.5f * em * (em + 2.0f) / ep;
    *ch = 1.0f + 0.5f * em * em / ep;
}

// ------------------------------------------------------ per-hit slot params
// Per lane and per material slot, NPF values:
//   lossless:  P0 kq (signed: >= 0 circular with d = kq t; < 0 hyperbolic with
//              d = -kq t), P1 xs, P2 ys, P3 xp, P4 yp  (X = S x, Y = S y for s / p)
//   absorbing: P0, P1 = q (re, im); P2, P3 = N^2 (re, im); P4 unused.
// The table of a lane stores element (s, p) at sp[(s * NPF + p) * ls].
constexpr int NPF = 5;
constexpr double kTinyZ = 1e-24;   // |z| floor: keeps q != 0 exactly at the critical angle

__device__ inline void slot_params(double nre, double nim, double kappa, double k0, double* P)
{
    if (nim == 0.0) {
        double n2 = nre * nre;
        double z = n2 - kappa * kappa;
        if (fabs(z) < kTinyZ) z = kTinyZ;
        if (z > 0.0) {
            double q = sqrt(z);
            P[0] = k0 * q; P[1] = 1.0 / q; P[2] = q;
            P[3] = q / n2; P[4] = n2 / q;
        } else {
            double Q = sqrt(-z);
            P[0] = -k0 * Q; P[1] = 1.0 / Q; P[2] = -Q;
            P[3] = -Q / n2; P[4] = n2 / Q;
        }
    } else {
        cd N = mk(nre, nim);
        cd N2 = cmul(N, N);
        cd z = csub(N2, mk(kappa * kappa, 0.0));
        cd q = csqrt_up(z);
        P[0] = q.re; P[1] = q.im; P[2] = N2.re; P[3] = N2.im; P[4] = 0.0;
    }
}

// Per-lane slot tables.  slot_params gives P[5] for one slot; a table keeps
// what the layer loops read and returns, for slot s,
//   lossless(s, kq, xs, ys, xp, yp)   P0..P4 of a lossless slot,
//   absorbing(s, Pl)                  Pl = q (re, im), N^2 (re, im).
// Slot tables are laid out per wave: value p of slot s of lane l of wave w
// at base[((w n_slots + s) kPer + p) 64 + l].  The lane stride is the
// compile-time 64, so the reads of one slot's values take immediate offsets
// from one address; consecutive lanes read consecutive doubles.
constexpr int kSlotLanes = 64;
__device__ inline double* slot_lane_base(double* base, int n_slots, int per, int tid)
{
    return base + (tid / kSlotLanes) * n_slots * per * kSlotLanes + (tid % kSlotLanes);
}

// One layer of a stack as the thin-film solves read it from LDS: the
// thickness, the slot's byte offset in a lane's slot table (slot x values
// per slot x kSlotLanes x 8) and the slot.  Each stack of Lmax layers sits
// between kRecPad pad records (zero thickness, slot 0) at either end, so
// the reads that run ahead of a sweep stay inside the stack's records and
// a layer is one 16-byte read.
struct __align__(16) LayerRec {
    double t;
    uint32_t soff;
    uint32_t slot;
};
constexpr int kRecPad = 3;
__host__ __device__ inline int rec_stride(int Lmax) { return Lmax + 2 * kRecPad; }

// Layer sources of the thin-film solves.  A cursor yields one stack's
// layers in incidence order; reads past the stack's end are harmless:
// records have pads there, arrays clamp the index to the last layer.
struct RecCursor {
    const LayerRec* p;
    int dir;
    __device__ LayerRec get() const { return *p; }
    __device__ void next() { p += dir; }
};
struct ArrCursor {
    const double* thk;
    const uint8_t* slot;
    int idx, dir, last;
    uint32_t unit;                       // bytes per slot in a lane's slot table
    __device__ LayerRec get() const
    {
        const uint32_t s = slot[idx];
        LayerRec r;
        r.t = thk[idx]; r.soff = s * unit; r.slot = s;
        return r;
    }
    __device__ void next() { idx = idx == last ? idx : idx + dir; }
};
// One stack as records (rec: its layer 0) or as thickness and slot arrays.
struct RecStack {
    const LayerRec* rec;
    __device__ RecCursor cursor(int L, bool front) const
    {
        RecCursor c = { rec + (front ? L - 1 : 0), front ? -1 : 1 };
        return c;
    }
};
struct ArrStack {
    const double* thk;
    const uint8_t* slot;
    uint32_t unit;
    __device__ ArrCursor cursor(int L, bool front) const
    {
        ArrCursor c = { thk, slot, front ? L - 1 : 0, front ? -1 : 1, front ? 0 : L - 1, unit };
        return c;
    }
};
// A design's stacks (one per mirror) in either form.
struct RecStacks {
    const LayerRec* base;                // [M][rec_stride(Lmax)]
    int Lmax;
    __device__ RecStack mirror(int m) const
    {
        RecStack s = { base + m * rec_stride(Lmax) + kRecPad };
        return s;
    }
};
struct ArrStacks {
    const double* thk;                   // [M][Lmax]
    const uint8_t* slot;
    int Lmax;
    uint32_t unit;
    __device__ ArrStack mirror(int m) const
    {
        ArrStack s = { thk + m * Lmax, slot + m * Lmax, unit };
        return s;
    }
};

// Records of n_stacks stacks (thk, slot: [n_stacks][Lmax]) into dst
// ([n_stacks][rec_stride(Lmax)]), for slot tables of `per` values per slot.
// Called by the whole block.
__device__ inline void stage_recs(LayerRec* dst, const double* thk, const uint8_t* slot, int n_stacks, int Lmax,
                                  int per)
{
    const int stride = rec_stride(Lmax), n = n_stacks * stride;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int m = i / stride, j = i - m * stride - kRecPad;
        LayerRec r = { 0.0, 0u, 0u };
        if (j >= 0 && j < Lmax) {
            const uint32_t sl = slot[m * Lmax + j];
            r.t = thk[m * Lmax + j];
            r.slot = sl;
            r.soff = sl * (uint32_t)(per * kSlotLanes * 8);
        }
        dst[i] = r;
    }
}

// LaneSlots5 keeps all five values per lane (lanes may differ in
// wavelength).  LaneSlots3 keeps kq, x_s, y_s per lane and takes N^2 of the
// slot from arrays shared by the workgroup (one wavelength per workgroup):
// x_p = y_s / N^2 and y_p = N^2 x_s for both lossless kinds.
struct LaneSlots5 {
    static constexpr int kPer = 5;
    double* sp;                 // this lane's value 0 of slot 0 (slot_lane_base)
    static constexpr int ls = kSlotLanes;
    __device__ void put(int s, const double* P) const
    {
#pragma unroll
        for (int p = 0; p < 5; ++p) sp[(s * 5 + p) * ls] = P[p];
    }
    __device__ void lossless(int s, double& kq, double& xs, double& ys, double& xp, double& yp) const
    {
        const double* P = sp + s * 5 * ls;
        kq = P[0]; xs = P[ls]; ys = P[2 * ls]; xp = P[3 * ls]; yp = P[4 * ls];
    }
    __device__ void absorbing(int s, double* Pl) const
    {
        const double* P = sp + s * 5 * ls;
        Pl[0] = P[0]; Pl[1] = P[ls]; Pl[2] = P[2 * ls]; Pl[3] = P[3 * ls];
    }
    __device__ void lossless_r(const LayerRec& r, double& kq, double& xs, double& ys, double& xp,
                               double& yp) const
    {
        const double* P = (const double*)((const unsigned char*)sp + r.soff);
        kq = P[0]; xs = P[ls]; ys = P[2 * ls]; xp = P[3 * ls]; yp = P[4 * ls];
    }
};
struct LaneSlots3 {
    static constexpr int kPer = 3;
    double* sp;                 // this lane's value 0 of slot 0 (slot_lane_base)
    static constexpr int ls = kSlotLanes;
    const double* nsq;          // N^2 (re, im) per slot
    const double* pxy;          // per slot (1 / Re N^2 if lossless, Re N^2), 16-byte aligned pairs
    __device__ void put(int s, const double* P) const
    {
        sp[(s * 3) * ls] = P[0]; sp[(s * 3 + 1) * ls] = P[1]; sp[(s * 3 + 2) * ls] = P[2];
    }
    __device__ void lossless(int s, double& kq, double& xs, double& ys, double& xp, double& yp) const
    {
        const double* P = sp + s * 3 * ls;
        kq = P[0]; xs = P[ls]; ys = P[2 * ls];
        const double2 c = reinterpret_cast<const double2*>(pxy)[s];   // one paired LDS read
        xp = ys * c.x; yp = xs * c.y;
    }
    __device__ void lossless_r(const LayerRec& r, double& kq, double& xs, double& ys, double& xp,
                               double& yp) const
    {
        const double* P = (const double*)((const unsigned char*)sp + r.soff);
        kq = P[0]; xs = P[ls]; ys = P[2 * ls];
        const double2 c = reinterpret_cast<const double2*>(pxy)[r.slot];
        xp = ys * c.x; yp = xs * c.y;
    }
    __device__ void absorbing(int s, double* Pl) const
    {
        const double* P = sp + s * 3 * ls;
        Pl[0] = P[0]; Pl[1] = P[ls]; Pl[2] = nsq[2 * s]; Pl[3] = nsq[2 * s + 1];
    }
};

// LaneSlots3x: the values LaneSlots3 returns, all five kept per lane (x_p
// and y_p formed once, by the same products, when the slot is put), so a
// layer reads them instead of multiplying again.  Same results as LaneSlots3.
struct LaneSlots3x {
    static constexpr int kPer = 5;
    double* sp;                 // this lane's value 0 of slot 0 (slot_lane_base)
    static constexpr int ls = kSlotLanes;
    const double* nsq;          // N^2 (re, im) per slot
    const double* pxy;          // per slot (1 / Re N^2 if lossless, Re N^2), 16-byte aligned pairs
    __device__ void put(int s, const double* P) const
    {
        double* Q = sp + s * 5 * ls;
        Q[0] = P[0]; Q[ls] = P[1]; Q[2 * ls] = P[2];
        const double2 c = reinterpret_cast<const double2*>(pxy)[s];
        Q[3 * ls] = P[2] * c.x; Q[4 * ls] = P[1] * c.y;
    }
    __device__ void lossless(int s, double& kq, double& xs, double& ys, double& xp, double& yp) const
    {
        const double* P = sp + s * 5 * ls;
        kq = P[0]; xs = P[ls]; ys = P[2 * ls]; xp = P[3 * ls]; yp = P[4 * ls];
    }
    __device__ void absorbing(int s, double* Pl) const
    {
        const double* P = sp + s * 5 * ls;
        Pl[0] = P[0]; Pl[1] = P[ls]; Pl[2] = nsq[2 * s]; Pl[3] = nsq[2 * s + 1];
    }
    __device__ void lossless_r(const LayerRec& r, double& kq, double& xs, double& ys, double& xp,
                               double& yp) const
    {
        const double* P = (const double*)((const unsigned char*)sp + r.soff);
        kq = P[0]; xs = P[ls]; ys = P[2 * ls]; xp = P[3 * ls]; yp = P[4 * ls];
    }
};

// ------------------------------------------------------------ chain steps
template <typename T> struct V2 { T br, bi, cr, ci; };   // [B; C] of one polarization
template <typename T> struct CTv { T re, im; };

// [B; C] <- [[C, -i X], [-i Y, C]] [B; C] with real C, X, Y
template <typename T>
__device__ inline void step_real(V2<T>& v, T C, T X, T Y)
{
    // explicit fused operations: the rounding does not depend on how the
    // compiler contracts each inlined copy
    T br = fma(C, v.br, X * v.ci);
    T bi = fma(C, v.bi, -(X * v.cr));
    T cr = fma(C, v.cr, Y * v.bi);
    T ci = fma(C, v.ci, -(Y * v.br));
    v.br = br; v.bi = bi; v.cr = cr; v.ci = ci;
}

template <typename T>
__device__ inline CTv<T> tmul(CTv<T> a, CTv<T> b)
{
#pragma clang fp contract(fast)
    CTv<T> r; r.re = a.re * b.re - a.im * b.im; r.im = a.re * b.im + a.im * b.re; return r;
}
template <typename T>
__device__ inline CTv<T> tdiv(CTv<T> a, CTv<T> b)
{
    T den = b.re * b.re + b.im * b.im;
    CTv<T> r; r.re = (a.re * b.re + a.im * b.im) / den; r.im = (a.im * b.re - a.re * b.im) / den; return r;
}

// general complex step: [B; C] <- [[C, -iX], [-iY, C]] [B; C]
template <typename T>
__device__ inline void step_cplx(V2<T>& v, CTv<T> C, CTv<T> X, CTv<T> Y)
{
    CTv<T> B = { v.br, v.bi }, Cv = { v.cr, v.ci };
    CTv<T> mX = { X.im, -X.re }, mY = { Y.im, -Y.re };   // -i X, -i Y
    CTv<T> b1 = tmul(C, B), b2 = tmul(mX, Cv), c1 = tmul(mY, B), c2 = tmul(C, Cv);
    v.br = b1.re + b2.re; v.bi = b1.im + b2.im;
    v.cr = c1.re + c2.re; v.ci = c1.im + c2.im;
}

// Trig part of a lossless layer: circular or hyperbolic by the sign of kq
// (HC = false: the caller knows every layer is circular).
template <typename T, bool HC = true>
__device__ inline void layer_cs(T kq, T t, T* C, T* S)
{
    const bool hyper = HC && kq < (T)0;
    gtrig<HC>(hyper ? -kq * t : kq * t, hyper, C, S);
}

// layer_cs up to a sign: in double precision the half-period form (C, S
// are (-1)^n times the layer's cosine and sine, n added to *nsum); the
// single-precision chain keeps the exact sign and leaves *nsum alone.
template <typename T, bool HC = true>
__device__ inline void layer_cs_half(T kq, T t, T* C, T* S, double* nsum)
{
    const bool hyper = HC && kq < (T)0;
    if constexpr (sizeof(T) == 8)
        gtrig_half<HC>(hyper ? -kq * t : kq * t, hyper, C, S, nsum);
    else
        gtrig<HC>(hyper ? -kq * t : kq * t, hyper, C, S);
}

// layer_cs_half in two parts (see trig_reduce): LayerTrig<T, HC>::reduce
// for a layer's (kq, t), then eval.  The single-precision chain keeps the
// whole routine in eval.
template <typename T, bool HC> struct LayerTrig;
template <bool HC> struct LayerTrig<double, HC> {
    using Arg = TrigArg;
    __device__ static Arg reduce(double kq, double t)
    {
        const bool hyper = HC && kq < 0.0;
        return trig_reduce<HC>(hyper ? -kq * t : kq * t, hyper);
    }
    __device__ static void eval(const Arg& a, double* C, double* S, double* nsum) { trig_eval<HC>(a, C, S, nsum); }
};
template <bool HC> struct LayerTrig<float, HC> {
    struct Arg { float kq, t; };
    __device__ static Arg reduce(float kq, float t) { return Arg{ kq, t }; }
    __device__ static void eval(const Arg& a, float* C, float* S, double* nsum)
    {
        layer_cs_half<float, HC>(a.kq, a.t, C, S, nsum);
    }
};

// Entries of an absorbing layer: returns C, X_s, Y_s, X_p, Y_p.
template <typename T>
__device__ inline void layer_cplx(const T* P, T k0, T t, CTv<T>* C, CTv<T>* Xs, CTv<T>* Ys,
                                  CTv<T>* Xp, CTv<T>* Yp)
{
    CTv<T> q = { P[0], P[1] }, N2 = { P[2], P[3] };
    T a = k0 * q.re * t, b = k0 * q.im * t;
    T sa, ca, ch, sh;
    sincos_cw(a, &sa, &ca);
    coshsinh(b, &ch, &sh);
    CTv<T> cosd = { ca * ch, -sa * sh }, sind = { sa * ch, ca * sh };
    *C = cosd;
    *Xs = tdiv(sind, q);
    *Ys = tmul(q, sind);
    *Xp = tdiv(tmul(sind, q), N2);
    *Yp = tdiv(tmul(N2, sind), q);
}

// Renormalize a single-precision chain vector (exact power-of-two scaling).
template <typename T>
__device__ inline void renorm(V2<T>& v, int& e)
{
    T m = fmax(fmax(fabs(v.br), fabs(v.bi)), fmax(fabs(v.cr), fabs(v.ci)));
    if (m > (T)1e18) {
        int ex;
        frexp(m, &ex);
        v.br = ldexp(v.br, -ex); v.bi = ldexp(v.bi, -ex);
        v.cr = ldexp(v.cr, -ex); v.ci = ldexp(v.ci, -ex);
        e += ex;
    }
}

// Coefficients (Eq. 3 convention) from the chain result.
struct Coef4 { cd rs, rp, ts, tp; };

template <typename T>
__device__ inline Coef4 finish_coeffs(const V2<T>& vs, const V2<T>& vp, int es, int ep,
                                      double eta0s, double eta0p, cd tp_factor)
{
    cd Bs = mk((double)vs.br, (double)vs.bi), Cs = mk((double)vs.cr, (double)vs.ci);
    cd Bp = mk((double)vp.br, (double)vp.bi), Cp = mk((double)vp.cr, (double)vp.ci);
    cd dens = cadd(cscale(Bs, eta0s), Cs), denp = cadd(cscale(Bp, eta0p), Cp);
    Coef4 o;
    o.rs = cdiv(csub(cscale(Bs, eta0s), Cs), dens);
    cd rpm = cdiv(csub(cscale(Bp, eta0p), Cp), denp);
    o.rp = mk(-rpm.re, -rpm.im);
    o.ts = cscale(cdiv(mk(2.0 * eta0s, 0.0), dens), ldexp(1.0, -es));
    o.tp = cscale(cmul(cdiv(mk(2.0 * eta0p, 0.0), denp), tp_factor), ldexp(1.0, -ep));
    return o;
}

// Sign flip of x when sb is 1 << 31 (an exact negation), identity for 0.
__device__ inline double flip_sign(double x, uint32_t sb)
{
    return __hiloint2double(__double2hiint(x) ^ (int)sb, __double2loint(x));
}

// Lossless stack: one loop body for every layer.  The LDS reads run ahead of
// the arithmetic: the layer record two layers ahead, the slot's parameters
// one layer ahead.  HC = false: no layer of any lane is evanescent.
// In double precision the layers' cosines and sines come from the
// half-period reduction with the sign (-1)^n of each left out, so the chain
// vector is (-1)^(sum n) times the exact one; that sign is put back on the
// stored checkpoints and on the result (exact negations).
template <typename T, bool HC, class SL, class Cur>
__device__ __attribute__((always_inline)) inline void lossless_sweep(Cur cur, int L, const SL& sl, V2<T>& vs,
                                                                     V2<T>& vp, int& es, int& ep, double* ck,
                                                                     int64_t ckb, int kseg = kSegL)
{
    double nsum = 0.0;                                  // sum of the layers' n (exact: small integers)
    auto sign_bit = [&]() { return (uint32_t)((int)nsum & 1) << 31; };
    // ck (T = double only): the adjoint's sweep checkpoints v_{g kseg}
    // (incidence-order layer g kseg and below) go to the 64-byte block g at
    // ck + g ckb, whole; v_0 goes to block 0 after the loop.
    auto store = [&](int g) {
        const uint32_t sb = sign_bit();
        double2* c = (double2*)(ck + (int64_t)g * ckb);
        c[0] = make_double2(flip_sign((double)vs.br, sb), flip_sign((double)vs.bi, sb));
        c[1] = make_double2(flip_sign((double)vs.cr, sb), flip_sign((double)vs.ci, sb));
        c[2] = make_double2(flip_sign((double)vp.br, sb), flip_sign((double)vp.bi, sb));
        c[3] = make_double2(flip_sign((double)vp.cr, sb), flip_sign((double)vp.ci, sb));
    };
    // Software pipeline over the layers: while layer j is evaluated and
    // applied, layer j+1's argument is reduced (from slot parameters read
    // one iteration earlier), layer j+2's slot parameters are read, and
    // layer j+3's record; no value is used in the iteration that loads it.
    using LT = LayerTrig<T, HC>;
    const LayerRec r0 = cur.get();
    double kq, xs, ys, xp, yp;
    sl.lossless_r(r0, kq, xs, ys, xp, yp);
    typename LT::Arg ta = LT::reduce((T)kq, (T)r0.t);      // t = 0 gives the identity exactly
    cur.next();
    const LayerRec r1 = cur.get();
    double kq1, xs1, ys1, xp1, yp1;
    sl.lossless_r(r1, kq1, xs1, ys1, xp1, yp1);
    double t1 = r1.t;
    cur.next();
    LayerRec r2 = cur.get();
    // loop index j of the next checkpoint (incidence-order layer L-1-j a
    // positive multiple of kseg, a power of two), or L when none is left.
    // Checkpoint layers have j = L-1 (mod 4): after the first L mod 4
    // layers the loop takes four layers at a time and looks for a
    // checkpoint after the fourth only.
    const int ksh = 31 - __builtin_clz((unsigned)kseg);
    int jck = (L - 1) & (kseg - 1);
    if (jck >= L - 1) jck = L;
    auto layer = [&](int j) {
        cur.next();
        const LayerRec r3 = cur.get();                               // past the stack: pad records
        double kq2, xs2, ys2, xp2, yp2;
        sl.lossless_r(r2, kq2, xs2, ys2, xp2, yp2);
        const typename LT::Arg ta1 = LT::reduce((T)kq1, (T)t1);     // the next layer's (past the stack: unused)
        T C, S;
        LT::eval(ta, &C, &S, &nsum);
        step_real(vs, C, S * (T)xs, S * (T)ys);
        step_real(vp, C, S * (T)xp, S * (T)yp);
        if (sizeof(T) == 4 && (j & 7) == 7) { renorm(vs, es); renorm(vp, ep); }
        ta = ta1; xs = xs1; ys = ys1; xp = xp1; yp = yp1;
        kq1 = kq2; xs1 = xs2; ys1 = ys2; xp1 = xp2; yp1 = yp2; t1 = r2.t;
        r2 = r3;
    };
    auto checkpoint = [&](int j) {
        if (sizeof(T) == 8 && ck && j == jck) {
            store((L - 1 - j) >> ksh);
            jck = jck + (1 << ksh) < L - 1 ? jck + (1 << ksh) : L;
        }
    };
    const int pre = L & 3;
    int j = 0;
    for (; j < pre; ++j) layer(j);
    if (pre > 0) checkpoint(pre - 1);
#pragma unroll 1
    for (; j < L; j += 4) {
        layer(j);
        layer(j + 1);
        layer(j + 2);
        layer(j + 3);
        checkpoint(j + 3);
    }
    if constexpr (sizeof(T) == 8) {
        if (ck) store(0);
        const uint32_t sb = sign_bit();
        vs.br = flip_sign(vs.br, sb); vs.bi = flip_sign(vs.bi, sb);
        vs.cr = flip_sign(vs.cr, sb); vs.ci = flip_sign(vs.ci, sb);
        vp.br = flip_sign(vp.br, sb); vp.bi = flip_sign(vp.bi, sb);
        vp.cr = flip_sign(vp.cr, sb); vp.ci = flip_sign(vp.ci, sb);
    }
}

// Forward solve of one hit.  stk: this mirror's layers in stack order
// (LDS, RecStack or ArrStack); `front` selects incidence order 0..L-1
// (else reversed).  sl: this lane's slot table.  Exit
// medium admittances (es, ep) are complex in general.
// The stack thicknesses and slot parameters are read in double precision
// and rounded to the chain precision T once per layer.  circ: no lane of the
// calling wave has an evanescent lossless slot (the sweep then skips the
// hyperbolic case; the results are the same).  ck (lossless FP64 stacks):
// the entry's checkpoint blocks for the adjoint's sweep (block g at ck + g
// ckb, one every kseg layers), or null.
template <typename T, class SL, class Stk>
__device__ __attribute__((always_inline)) inline Coef4 tmm_solve(const Stk& stk, int L,
                                  bool front, const SL& sl, uint32_t cplx_mask, double k0d, double eta0s,
                                  double eta0p, cd etaEs, cd etaEp, cd tp_factor, bool circ = false,
                                  double* ck = nullptr, int64_t ckb = 8, int kseg = kSegL)
{
    const T k0 = (T)k0d;
    V2<T> vs = { (T)1, (T)0, (T)etaEs.re, (T)etaEs.im };
    V2<T> vp = { (T)1, (T)0, (T)etaEp.re, (T)etaEp.im };
    int es = 0, ep = 0;
    if (L <= 0) return finish_coeffs(vs, vp, es, ep, eta0s, eta0p, tp_factor);
    if (cplx_mask == 0u) {
        if (circ)
            lossless_sweep<T, false>(stk.cursor(L, front), L, sl, vs, vp, es, ep, ck, ckb, kseg);
        else
            lossless_sweep<T, true>(stk.cursor(L, front), L, sl, vs, vp, es, ep, ck, ckb, kseg);
        return finish_coeffs(vs, vp, es, ep, eta0s, eta0p, tp_factor);
    }
    auto cur = stk.cursor(L, front);
    for (int j = 0; j < L; ++j, cur.next()) {
        const LayerRec r = cur.get();
        T t = (T)r.t;                       // t = 0 gives the identity exactly
        const int s = (int)r.slot;
        if (!((cplx_mask >> s) & 1u)) {
            double kq, xs, ys, xp, yp;
            sl.lossless_r(r, kq, xs, ys, xp, yp);
            T C, S;
            layer_cs((T)kq, t, &C, &S);
            step_real(vs, C, S * (T)xs, S * (T)ys);
            step_real(vp, C, S * (T)xp, S * (T)yp);
        } else {
            double Pd[4];
            sl.absorbing(s, Pd);
            T Pl[4] = { (T)Pd[0], (T)Pd[1], (T)Pd[2], (T)Pd[3] };
            CTv<T> C, Xs, Ys, Xp, Yp;
            layer_cplx(Pl, k0, t, &C, &Xs, &Ys, &Xp, &Yp);
            step_cplx(vs, C, Xs, Ys);
            step_cplx(vp, C, Xp, Yp);
        }
        if (sizeof(T) == 4 && (j & 7) == 7) { renorm(vs, es); renorm(vp, ep); }
    }
    return finish_coeffs(vs, vp, es, ep, eta0s, eta0p, tp_factor);
}

}  // namespace gwg
