// Per-ray geometry and polarization steps of the Monte Carlo trace, shared by
// the forward and adjoint kernels.
//
// Geometry (synthetic waveguide): glass slab 0 <= z <= T, 0 <= x <= Lx,
// unbounded in y; M parallel mirror planes with normal n = (nx, 0, nz)
// across the full thickness divide it into M + 1 convex cells; a ray leaves
// its cell through the nearest of the cell's four bounding planes (top,
// bottom, left boundary, right boundary), never the plane it stands on.
// The path-determining operations (distances, position updates, mirror
// reflection, face tests, exit refraction, binning) are individually
// rounded double operations in a fixed order with FMA contraction disabled,
// so a CPU implementation with the same operation sequence reproduces every
// path decision bit for bit (integer bin counts are compared exactly).
#pragma once
#include <stddef.h>
#include "gwg_internal.h"
#include "gwg_device.h"

namespace gwg {

struct Ray {
    double px, py, pz, dx, dy, dz;
    cd e[3];
    int cell, last, nev, nprma;
    uint32_t w4[4];
    int64_t id;
    uint32_t key1;                    // Philox key word 1 of this launch
};

// Block-uniform data of one (design, wavelength, FoV) point, in LDS.
struct PointLds {
    double k0, ng, na;
    double dir[3];
    double slotN[2 * kMaxSlots];     // (re, im) per slot
    double nsq[2 * kMaxSlots];       // N^2 (re, im) per slot
    double pxy[2 * kMaxSlots];       // per slot: 1 / Re N^2 (lossless slot, else 0), Re N^2
    double crit[2 * kMaxSlots];      // near-critical kappa interval per slot
    double h[kMaxMirrors], sc_r[kMaxMirrors], sc_t[kMaxMirrors];
    uint32_t thr[kMaxMirrors];
    int32_t nlay[kMaxMirrors];
    // the walk's scene constants, read from LDS where they are used rather
    // than held in scalar registers across the walk
    double T, Lx, nx, nz, ER, ex0, ew, ey0, eh;
    int32_t M, Kmax, bins_x, bins_y;
    // smallest Re N^2 of a lossless slot: a hit whose kappa^2 exceeds it may
    // meet an evanescent layer (+huge without lossless slots)
    double kap2_evan;
};
// the slot tables read pxy in pairs (16-byte loads)
static_assert(offsetof(PointLds, pxy) % 16 == 0, "pxy pairs must be 16-byte aligned");

__device__ inline void cross3(double ax, double ay, double az, double bx, double by, double bz,
                              double* o)
{
    o[0] = ay * bz - az * by;
    o[1] = az * bx - ax * bz;
    o[2] = ax * by - ay * bx;
}

// The field's arithmetic (polarization bases, projections, Eq. 5, the face
// coefficients and weights) uses fused multiply-adds, written out because
// the library builds without contraction; the geometry (positions, surfaces,
// directions, kappa, bins) keeps the oracle's plain products so that paths
// and bins agree bit for bit.
__device__ inline void cross3_f(double ax, double ay, double az, double bx, double by, double bz, double* o)
{
    o[0] = fma(ay, bz, -(az * by));
    o[1] = fma(az, bx, -(ax * bz));
    o[2] = fma(ax, by, -(ay * bx));
}
__device__ inline cd cmul_f(cd a, cd b) { return mk(fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)); }
__device__ inline double dot3_f(const double* a) { return fma(a[2], a[2], fma(a[1], a[1], a[0] * a[0])); }

// s unit vector for direction d on a surface of normal n; when d is nearly
// parallel to n (s and p equivalent) the y axis projected orthogonal to d.
__device__ inline void s_basis(double dx, double dy, double dz, double nx, double ny, double nz, double* s)
{
    double c[3];
    cross3_f(dx, dy, dz, nx, ny, nz, c);
    double l = sqrt(dot3_f(c));
    if (l < 1e-6) {
        double yd = dy;
        c[0] = -yd * dx; c[1] = fma(-yd, dy, 1.0); c[2] = -yd * dz;
        l = sqrt(dot3_f(c));
    }
    double il = 1.0 / l;
    s[0] = c[0] * il; s[1] = c[1] * il; s[2] = c[2] * il;
}

// Components of a complex field along a real unit vector: sum_c e_c v_c.
__device__ inline cd dot_re(const cd* e, const double* v)
{
    return mk(fma(e[2].re, v[2], fma(e[1].re, v[1], e[0].re * v[0])),
              fma(e[2].im, v[2], fma(e[1].im, v[1], e[0].im * v[0])));
}

// Eq. 5 given the incoming field's components es = s.E and ep = p_in.E.
__device__ inline void apply_sp_proj(cd* e, const double* s, const double* pout, cd cs, cd cp, double scale,
                                     cd es, cd ep)
{
    cd as = cscale(cmul_f(cs, es), scale), ap = cscale(cmul_f(cp, ep), scale);
    for (int k = 0; k < 3; ++k)
        e[k] = mk(fma(as.re, s[k], ap.re * pout[k]), fma(as.im, s[k], ap.im * pout[k]));
}

// Eq. 5 on the local basis: E <- scale (cs (E.s) s + cp (E.p_in) p_out)
__device__ inline void apply_sp(cd* e, const double* s, const double* pin, const double* pout,
                                cd cs, cd cp, double scale)
{
    apply_sp_proj(e, s, pout, cs, cp, scale, dot_re(e, s), dot_re(e, pin));
}

__device__ inline double norm2(const cd* e)
{
    double ax = fma(e[0].re, e[0].re, e[0].im * e[0].im);
    double ay = fma(e[1].re, e[1].re, e[1].im * e[1].im);
    double az = fma(e[2].re, e[2].re, e[2].im * e[2].im);
    return (ax + ay) + az;
}

// Guided direction for field angles (thx, thy) in degrees: direction at the
// eye, refracted into the glass through the top face, mirrored by an
// in-coupler parallel to the mirrors.
__device__ inline void field_direction(double thx, double thy, double ng, double nx, double nz, double* d)
{
    double tx = tan(thx * (3.14159265358979323846 / 180.0));
    double ty = tan(thy * (3.14159265358979323846 / 180.0));
    double inv = 1.0 / sqrt(tx * tx + ty * ty + 1.0);
    double ax = tx * inv, ay = ty * inv;
    double gx = ax / ng, gy = ay / ng, gz = sqrt(1.0 - (ax * ax + ay * ay) / (ng * ng));
    double gn = nx * gx + nz * gz;
    double t2 = 2.0 * gn;
    d[0] = gx - t2 * nx;
    d[1] = gy;
    d[2] = gz - t2 * nz;
}

__device__ inline uint32_t philox_key1(const SceneDev& sc)
{
    return sc.step_dev ? (sc.seed_hi ^ (sc.step_host + *sc.step_dev)) : sc.key1;
}

__device__ inline void ray_birth(const SceneDev& sc, const PointLds& pl, int64_t id, Ray& r)
{
    r.key1 = philox_key1(sc);
    const int64_t gid = id + sc.id_base;      // the ray's id in the whole batch
    u32x4 w = philox10((uint32_t)(uint64_t)gid, (uint32_t)((uint64_t)gid >> 32), 0u, 0u, sc.key0, r.key1);
    r.id = gid;
    r.px = sc.px0 + u24(w.x) * sc.pw;
    r.py = u24(w.y) * sc.ph - 0.5 * sc.ph;
    r.pz = sc.T;
    if (sc.fov_mode == 1) {
        double thx = sc.fov_x0 + u24(w.z) * (sc.fov_x1 - sc.fov_x0);
        double thy = sc.fov_y0 + u24(w.w) * (sc.fov_y1 - sc.fov_y0);
        double d[3];
        field_direction(thx, thy, pl.ng, sc.nx, sc.nz, d);
        r.dx = d[0]; r.dy = d[1]; r.dz = d[2];
    } else {
        r.dx = pl.dir[0]; r.dy = pl.dir[1]; r.dz = pl.dir[2];
    }
    double s0[3], p0[3];
    s_basis(r.dx, r.dy, r.dz, 0.0, 0.0, 1.0, s0);
    cross3_f(r.dx, r.dy, r.dz, s0[0], s0[1], s0[2], p0);
    const double* e = (w.x & 1u) ? p0 : s0;
    for (int k = 0; k < 3; ++k) r.e[k] = mk(e[k], 0.0);
    r.cell = 0;
    r.last = SURF_TOP;
    r.nev = 0;
    r.nprma = 0;
}

// Nearest bounding plane of the current cell; moves the ray onto it.
__device__ inline int next_surface(const SceneDev& sc, const PointLds& pl, Ray& r)
{
    // One division per kind of surface, whatever the lanes of a wave face:
    // the face ahead (top or bottom, by the sign of dz), the mirror ahead
    // (the cell's left or right one, by the sign of dn) and, in an end cell,
    // the end face.  Each lane's quotient is the same as its own surface's;
    // the candidates are compared face first, then the left side (end 0 or
    // mirror cell-1), then the right side (end 1 or mirror cell), an earlier
    // candidate keeping a tie.
    double best = 0.0;
    int hit = -1;
    const bool up = r.dz > 0.0;
    if ((up && r.last != SURF_TOP) || (r.dz < 0.0 && r.last != SURF_BOTTOM)) {
        best = ((up ? pl.T : 0.0) - r.pz) / r.dz;
        hit = up ? SURF_TOP : SURF_BOTTOM;
    }
    const double dn = pl.nx * r.dx + pl.nz * r.dz;
    const double pn = pl.nx * r.px + pl.nz * r.pz;
    const bool ml = r.cell != 0 && dn > 0.0 && r.last != r.cell - 1;
    const bool mr = r.cell != pl.M && dn < 0.0 && r.last != r.cell;
    double tm = 0.0;
    const int mm = ml ? r.cell - 1 : r.cell;
    if (ml || mr) tm = (pl.h[mm] - pn) / dn;
    const bool e0 = r.cell == 0 && r.dx < 0.0 && r.last != SURF_END0;
    const bool e1 = r.cell == pl.M && r.dx > 0.0 && r.last != SURF_END1;
    double te = 0.0;
    if (e0 || e1) te = ((e0 ? 0.0 : pl.Lx) - r.px) / r.dx;
    if (e0) {
        if (hit < 0 || te < best) { best = te; hit = SURF_END0; }
    } else if (ml) {
        if (hit < 0 || tm < best) { best = tm; hit = mm; }
    }
    if (e1) {
        if (hit < 0 || te < best) { best = te; hit = SURF_END1; }
    } else if (mr) {
        if (hit < 0 || tm < best) { best = tm; hit = mm; }
    }
    if (hit < 0) return -1;
    r.px = r.px + best * r.dx;
    r.py = r.py + best * r.dy;
    r.pz = r.pz + best * r.dz;
    if (hit == SURF_TOP) r.pz = pl.T;
    if (hit == SURF_BOTTOM) r.pz = 0.0;
    if (hit == SURF_END0) r.px = 0.0;
    if (hit == SURF_END1) r.px = pl.Lx;
    return hit;
}

// Bare glass/air face (Eq. 3).  Returns 1 on total internal reflection.
struct FaceCoef { cd rs, rp, ts, tp; double flux, st2; int tir; };

__device__ inline FaceCoef face_coeffs(double ng, double na, double dx, double dy, double dz)
{
    FaceCoef f;
    double ng2 = ng * ng, na2 = na * na;
    f.st2 = ng2 * (dx * dx + dy * dy);
    double qi = ng * fabs(dz);
    f.tir = f.st2 > na2;
    cd qt = f.tir ? mk(0.0, sqrt(f.st2 - na2)) : mk(sqrt(na2 - f.st2), 0.0);
    // r and t of each polarization share their denominator: one reciprocal
    // 1/den = conj(den) / |den|^2 each (|den| is of order one here)
    const cd den_s = cadd(mk(qi, 0.0), qt);
    const double is = 1.0 / (den_s.re * den_s.re + den_s.im * den_s.im);
    const cd inv_s = mk(den_s.re * is, -den_s.im * is);
    f.rs = cmul_f(csub(mk(qi, 0.0), qt), inv_s);
    f.ts = cscale(inv_s, 2.0 * qi);
    const cd a = mk(na2 * qi, 0.0), b = cscale(qt, ng2);
    const cd den_p = cadd(a, b);
    const double ip = 1.0 / (den_p.re * den_p.re + den_p.im * den_p.im);
    const cd inv_p = mk(den_p.re * ip, -den_p.im * ip);
    f.rp = cmul_f(csub(a, b), inv_p);
    f.tp = cscale(inv_p, 2.0 * ng * na * qi);
    f.flux = f.tir ? 0.0 : sqrt(qt.re / qi);
    return f;
}

// Eyebox bin of a ray leaving the top face at (px, py) along air direction
// a: the grid cell of its crossing of the eyebox plane, or, with eye pupils,
// the pupil whose circle holds the crossing (pupils do not overlap).
__device__ inline int eyebox_bin(const SceneDev& sc, const PointLds& pl, double px, double py, const double* a)
{
    double xe = px + pl.ER * (a[0] / a[2]);
    double ye = py + pl.ER * (a[1] / a[2]);
    if (sc.n_pupils > 0) {
        for (int q = 0; q < sc.n_pupils; ++q) {
            const double dx = xe - sc.pupil_xy[2 * q];
            const double dy = ye - sc.pupil_xy[2 * q + 1];
            if (dx * dx + dy * dy < sc.pupil_r2) return q;
        }
        return -1;
    }
    double fx = ((xe - pl.ex0) / pl.ew) * (double)pl.bins_x;
    double fy = ((ye - pl.ey0) / pl.eh) * (double)pl.bins_y;
    if (!(fx >= 0.0 && fx < (double)pl.bins_x && fy >= 0.0 && fy < (double)pl.bins_y)) return -1;
    int bx = (int)fx, by = (int)fy;
    return by * pl.bins_x + bx;
}

__device__ inline void exit_direction(double ng, double na, const Ray& r, double st2, double* a)
{
    double rn = ng / na;
    a[0] = rn * r.dx;
    a[1] = rn * r.dy;
    a[2] = sqrt(1.0 - st2 / (na * na));
}

__device__ inline void mirror_reflect(double nx, double nz, double dx, double dz, double* ox, double* oz)
{
    double dn = nx * dx + nz * dz;
    double t2 = 2.0 * dn;
    *ox = dx - t2 * nx;
    *oz = dz - t2 * nz;
}

// Near-critical flag of the mixed-precision rule: kappa within any slot's interval.
__device__ inline bool near_critical(const PointLds& pl, int n_slots, double kappa)
{
    bool f = false;
    for (int s = 0; s < n_slots; ++s) f |= (kappa > pl.crit[2 * s] && kappa < pl.crit[2 * s + 1]);
    return f;
}

// ------------------------------------------------------- wave utilities
__device__ inline int wave_lane() { return (int)(threadIdx.x & 63); }

// Exclusive prefix sum over the 64 lanes of a wave; *total gets the sum.
__device__ inline int wave_excl_scan(int x, int* total)
{
    const int lane = wave_lane();
    int v = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    *total = __shfl(v, 63, 64);
    return v - x;
}

// Largest x over the 64 lanes (every lane must call).
__device__ inline int wave_max_int(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __shfl_xor(x, o, 64);
        x = y > x ? y : x;
    }
    return x;
}

// ------------------------------------------------------------ hit queue
// Mirror hits of one wave's current round of rays: entry p holds the hit's
// kappa and meta (mirror | front << 8), after the solve its four
// coefficients, and (field 10) the checkpoint slot of its adjoint entry or
// -1.  Field f of entry p at base[f * cap + p].
// A wave's hit queue holds up to Kmax hits per lane; hit h of lane l is in
// slot h * 64 + l, so the lanes' h-th hits share 512 contiguous bytes per
// field (the walks touch the lanes' hits in step).
__device__ inline int hq_slot(int lane, int h) { return h * 64 + lane; }

struct HitQueue {
    double* base;
    int cap;
    __device__ double kappa(int p) const { return base[p]; }
    __device__ int meta(int p) const { return (int)base[cap + p]; }
    __device__ void put(int p, double kappa, int meta) const
    {
        base[p] = kappa;
        base[cap + p] = (double)meta;
    }
    __device__ void put_coef(int p, const Coef4& c) const
    {
        double* b = base + 2 * cap + p;
        b[0] = c.rs.re; b[cap] = c.rs.im; b[2 * cap] = c.rp.re; b[3 * cap] = c.rp.im;
        b[4 * cap] = c.ts.re; b[5 * cap] = c.ts.im; b[6 * cap] = c.tp.re; b[7 * cap] = c.tp.im;
    }
    __device__ Coef4 coef(int p) const
    {
        const double* b = base + 2 * cap + p;
        Coef4 c;
        c.rs = mk(b[0], b[cap]); c.rp = mk(b[2 * cap], b[3 * cap]);
        c.ts = mk(b[4 * cap], b[5 * cap]); c.tp = mk(b[6 * cap], b[7 * cap]);
        return c;
    }
};
// Field 11 (non-memoized forward): the solve order, the slot of the wave's
// p-th solved hit at position p.
constexpr int kHitFields = 12;

// ------------------------------------------------------------ tape
// Field-changing events of one ray, for the reverse field sweep.  Event k
// takes four 16-byte words: the direction before the event (dx, dy), (dz,
// meta) with meta = type | mirror << 4 | front << 12 | reflected << 13, and
// two coefficient words (mirror hit and total internal reflection: c_s,
// c_p; exit: t_s, t_p and the flux factor, the transmission coefficients
// being real below the critical angle).  A mirror hit adds a record of two
// words, the incoming field's components s.E and p_in.E.  The 64 lanes of a
// wave keep word q of their event k side by side: 1 KB at ev + (k W + w) 512
// + 128 q doubles (W waves in the grid, w this wave), the mirror record at
// mr + (k W + w) 256 + 128 q.  In the field walk every walking lane records
// one event per iteration, so a wave's lanes store the same k together and
// each store instruction fills 16 whole cache lines; the reverse sweep reads
// the same way (reverse_sweep).
struct TapeRef { double* ev; double* mr; int64_t ks; };   // ks: doubles from event k to k + 1 (event words)

// The tape of lane `lane` of wave gwave of n_waves in a region of kmax *
// kTapeStride * 64 * n_waves doubles (event words first, then mirror records).
__device__ inline TapeRef tape_lane(double* region, int64_t kmax, int64_t n_waves, int64_t gwave, int lane)
{
    return { region + gwave * (64 * kTapeLine) + 2 * lane,
             region + kmax * n_waves * (64 * kTapeLine) + gwave * (64 * kTapeMir) + 2 * lane,
             n_waves * (64 * kTapeLine) };
}

__device__ inline void tape_put(const TapeRef& t, int k, double dx, double dy, double dz, int meta,
                                double c0, double c1, double c2, double c3)
{
    double2* b = (double2*)(t.ev + (int64_t)k * t.ks);
    b[0] = make_double2(dx, dy);
    b[64] = make_double2(dz, (double)meta);
    b[128] = make_double2(c0, c1);
    b[192] = make_double2(c2, c3);
}

__device__ inline void tape_put_mirror(const TapeRef& t, int k, cd es, cd ep)
{
    double2* b = (double2*)(t.mr + (int64_t)k * (t.ks / 2));
    b[0] = make_double2(es.re, es.im);
    b[64] = make_double2(ep.re, ep.im);
}

// Outcome of a terminated ray.
struct Outcome { int cat; int bin; double w; double w_in; };

// Walk one ray (already born) from its current state to termination.
// FIELD = false: geometry and branch decisions only; every mirror hit h calls
//   on_hit(h, kappa, meta) once its branch is drawn (meta = mirror | front
//   << 8 | reflected << 9) and on_hit.branch(m, refl).
// FIELD = true: also the polarization field (Eq. 5 at every event, Eq. 6 at
//   mirrors); mirror hit h takes its coefficients from
//   get_coef(h, direction, mirror, front) and, where GetCoef::kStoredBranch,
//   its branch from get_coef.refl(h) (the decision the geometry walk drew and
//   stored) instead of drawing it again; with TAPE and a non-null tape,
//   field-changing events are recorded for the adjoint.
// Both modes perform the same geometric operations, so they visit the same
// surfaces and take the same branches.  A total internal reflection and a
// mirror hit update the field with the same code (basis about the surface
// normal, Eq. 5 with the event's coefficients), so a wave whose lanes meet
// both runs it once.
template <bool FIELD, bool TAPE, class OnHit, class GetCoef>
__device__ inline void walk_ray(const SceneDev& sc, const PointLds& pl, Ray& r, Outcome& o,
                                OnHit on_hit, GetCoef get_coef, TapeRef tape, int* ntape)
{
    const double nx = pl.nx, nz = pl.nz;
    for (;;) {
        if (r.nev >= pl.Kmax) {
            o.cat = CAT_TRUNC; o.bin = -1; o.w = FIELD ? norm2(r.e) : 0.0; o.w_in = o.w;
            return;
        }
        int s = next_surface(sc, pl, r);
        if (s < 0) {
            o.cat = CAT_LOST; o.bin = -1; o.w = FIELD ? norm2(r.e) : 0.0; o.w_in = o.w;
            return;
        }
        r.nev++;
        // the event's field update: coefficients, scale, surface normal
        // (bnx, 0, bnz) and the direction after it
        cd cs = mk(0.0, 0.0), cp = mk(0.0, 0.0);
        double scale = 1.0, bnx = 0.0, bnz = 1.0;
        double ndx = r.dx, ndz = r.dz;
        int ev = EV_TIR, m = 0, front = 0, refl = 0;
        if (s == SURF_TOP || s == SURF_BOTTOM) {
            FaceCoef fc = face_coeffs(pl.ng, pl.na, r.dx, r.dy, r.dz);
            if (!fc.tir) {
                if (s == SURF_TOP) {
                    double sv[3], pin[3], pout[3];
                    double a[3];
                    exit_direction(pl.ng, pl.na, r, fc.st2, a);
                    o.w_in = 0.0;
                    o.w = 0.0;
                    if (FIELD) {
                        s_basis(r.dx, r.dy, r.dz, 0.0, 0.0, 1.0, sv);
                        cross3_f(r.dx, r.dy, r.dz, sv[0], sv[1], sv[2], pin);
                        cross3_f(a[0], a[1], a[2], sv[0], sv[1], sv[2], pout);
                        o.w_in = norm2(r.e);
                        if (TAPE && tape.ev) tape_put(tape, (*ntape)++, r.dx, r.dy, r.dz, EV_EXIT, fc.ts.re, fc.tp.re, fc.flux, 0.0);
                        apply_sp(r.e, sv, pin, pout, fc.ts, fc.tp, fc.flux);
                        o.w = norm2(r.e);
                    }
                    r.dx = a[0]; r.dy = a[1]; r.dz = a[2];
                    o.bin = eyebox_bin(sc, pl, r.px, r.py, a);
                    o.cat = o.bin >= 0 ? CAT_EYEBOX : CAT_MISS;
                    return;
                }
                o.cat = CAT_LEAK; o.bin = -1; o.w = FIELD ? norm2(r.e) : 0.0; o.w_in = o.w;
                return;
            }
            // total internal reflection at a face
            cs = fc.rs; cp = fc.rp;
            ndz = -r.dz;
        } else if (s == SURF_END0 || s == SURF_END1) {
            o.cat = CAT_END; o.bin = -1; o.w = FIELD ? norm2(r.e) : 0.0; o.w_in = o.w;
            return;
        } else {
            // mirror hit
            m = s;
            const double dn = nx * r.dx + nz * r.dz;
            front = dn < 0.0 ? 1 : 0;
            const int h = r.nprma;
            bool rf;
            if constexpr (FIELD && GetCoef::kStoredBranch) {
                rf = get_coef.refl(h);
            } else {
                if ((h & 3) == 0) {
                    u32x4 w = philox10((uint32_t)(uint64_t)r.id, (uint32_t)((uint64_t)r.id >> 32), (uint32_t)(h >> 2),
                                       1u, sc.key0, r.key1);
                    r.w4[0] = w.x; r.w4[1] = w.y; r.w4[2] = w.z; r.w4[3] = w.w;
                }
                const int hw = h & 3;
                const uint32_t word = hw == 0 ? r.w4[0] : hw == 1 ? r.w4[1] : hw == 2 ? r.w4[2] : r.w4[3];
                rf = word < pl.thr[m];
            }
            refl = rf ? 1 : 0;
            if (!FIELD) {
                double c[3];
                cross3(r.dx, r.dy, r.dz, nx, 0.0, nz, c);
                double kappa = pl.ng * sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
                on_hit(h, kappa, m | (front << 8) | (refl << 9));
                on_hit.branch(m, rf);
            }
            if (rf) mirror_reflect(nx, nz, r.dx, r.dz, &ndx, &ndz);
            if (FIELD) {
                const Coef4 co = get_coef(h, r.dx, r.dy, r.dz, m, front != 0);
                cs = rf ? co.rs : co.ts;
                cp = rf ? co.rp : co.tp;
                scale = rf ? pl.sc_r[m] : pl.sc_t[m];
            }
            bnx = nx; bnz = nz;
            ev = EV_MIRROR;
        }
        if (FIELD) {
            double sv[3], pin[3], pout[3];
            s_basis(r.dx, r.dy, r.dz, bnx, 0.0, bnz, sv);
            cross3_f(r.dx, r.dy, r.dz, sv[0], sv[1], sv[2], pin);
            cross3_f(ndx, r.dy, ndz, sv[0], sv[1], sv[2], pout);
            const cd es = dot_re(r.e, sv), ep = dot_re(r.e, pin);
            if (TAPE && tape.ev) {
                const int k = (*ntape)++;
                tape_put(tape, k, r.dx, r.dy, r.dz, ev | (m << 4) | (front << 12) | (refl << 13),
                         cs.re, cs.im, cp.re, cp.im);
                if (ev == EV_MIRROR) tape_put_mirror(tape, k, es, ep);
            }
            apply_sp_proj(r.e, sv, pout, cs, cp, scale, es, ep);
        }
        r.dx = ndx;
        r.dz = ndz;
        if (ev == EV_MIRROR) {
            if (!refl) r.cell += (m == r.cell) ? 1 : -1;
            r.last = m;
            r.nprma++;
        } else {
            r.last = s;
        }
    }
}

// One tape event as the reverse sweep reads it.
struct TapeLine { double dx, dy, dz, meta, c0, c1, c2, c3; };
__device__ inline TapeLine tape_line(const TapeRef& t, int k)
{
    const double2* b = (const double2*)(t.ev + (int64_t)k * t.ks);
    const double2 a0 = b[0], a1 = b[64], a2 = b[128], a3 = b[192];
    return { a0.x, a0.y, a1.x, a1.y, a2.x, a2.y, a3.x, a3.y };
}

// Reverse field sweep along one ray's fixed path (the adjoint of Eq. 5 and
// Eq. 6 for w = |E_K|^2): lambda_K = E_K, lambda_{k-1} = A_k^H lambda_k with
// A = scale (c_s s s^T + c_p p_out p_in^T).  For every mirror hit, last to
// first, calls emit(kappa, G_s, G_p, meta) with the holomorphic cotangents of
// the taken coefficients,
//     G_s = scale conj(lambda_k . s) (s . E_{k-1}),
//     G_p = scale conj(lambda_k . p_out) (p_in . E_{k-1}),
// and meta = mirror | front << 8 | reflected << 9.  nt events are on this
// lane's tape; ntw, the same on every calling lane, is the longest tape of
// the calling lanes.  The sweep steps a common event index i down from
// ntw - 1 and a lane takes event i once i < nt, so the lanes read the same
// event together.  A mirror hit's scale is the point's branch weight, that
// of a total internal reflection 1.
template <class Emit>
__device__ inline void reverse_sweep(const SceneDev& sc, const PointLds& pl, const cd* e_final, TapeRef tape,
                                     int nt, int ntw, Emit emit)
{
    cd lam[3] = { e_final[0], e_final[1], e_final[2] };
    // event words are requested two events ahead of their use, a mirror
    // record one event ahead (once that event's meta is in), so the memory
    // latency overlaps the arithmetic of the events in between
    const TapeLine zl = { 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0 };
    auto mirror_rec = [&](int k, double2& a, double2& b) {
        const double2* p = (const double2*)(tape.mr + (int64_t)k * (tape.ks / 2));
        a = p[0];
        b = p[64];
    };
    TapeLine n1 = zl, n2 = zl;
    if (ntw >= 1 && ntw - 1 < nt) n1 = tape_line(tape, ntw - 1);
    if (ntw >= 2 && ntw - 2 < nt) n2 = tape_line(tape, ntw - 2);
    double2 m0 = make_double2(0.0, 0.0), m1 = m0;
    if (ntw >= 1 && ntw - 1 < nt && ((int)n1.meta & 15) == EV_MIRROR) mirror_rec(ntw - 1, m0, m1);
    for (int i = ntw - 1; i >= 0; --i) {
        const TapeLine ev = n1;
        const double2 e0 = m0, e1 = m1;
        n1 = n2;
        if (i >= 2 && i - 2 < nt) n2 = tape_line(tape, i - 2);
        if (i >= 1 && i - 1 < nt && ((int)n1.meta & 15) == EV_MIRROR) mirror_rec(i - 1, m0, m1);
        if (i >= nt) continue;                          // this lane's tape is shorter
        const double dx = ev.dx, dy = ev.dy, dz = ev.dz;
        const int meta = (int)ev.meta;
        const int type = meta & 15, m = (meta >> 4) & 255;
        const int front = (meta >> 12) & 1, refl = (meta >> 13) & 1;
        cd cs = mk(ev.c0, ev.c1), cp = mk(ev.c2, ev.c3);
        double scale = 1.0;
        double sv[3], pin[3], pout[3];
        if (type == EV_MIRROR) {
            const cd es = mk(e0.x, e0.y), ep = mk(e1.x, e1.y);
            scale = refl ? pl.sc_r[m] : pl.sc_t[m];
            s_basis(dx, dy, dz, pl.nx, 0.0, pl.nz, sv);
            cross3_f(dx, dy, dz, sv[0], sv[1], sv[2], pin);
            double ndx = dx, ndz = dz;
            if (refl) mirror_reflect(pl.nx, pl.nz, dx, dz, &ndx, &ndz);
            cross3_f(ndx, dy, ndz, sv[0], sv[1], sv[2], pout);
            const cd ls = dot_re(lam, sv), lp = dot_re(lam, pout);
            const cd Gs = cscale(cmul_f(cconj(ls), es), scale);
            const cd Gp = cscale(cmul_f(cconj(lp), ep), scale);
            double c3[3];
            cross3(dx, dy, dz, pl.nx, 0.0, pl.nz, c3);
            const double kappa = pl.ng * sqrt(c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
            emit(kappa, Gs, Gp, m | (front << 8) | (refl << 9));
        } else {
            s_basis(dx, dy, dz, 0.0, 0.0, 1.0, sv);
            cross3_f(dx, dy, dz, sv[0], sv[1], sv[2], pin);
            if (type == EV_TIR) {
                cross3_f(dx, dy, -dz, sv[0], sv[1], sv[2], pout);
            } else {
                // exit: real t_s, t_p and the flux factor
                cs = mk(ev.c0, -0.0);
                cp = mk(ev.c1, -0.0);
                scale = ev.c2;
                Ray tmp;
                tmp.dx = dx; tmp.dy = dy; tmp.dz = dz;
                const double st2 = (pl.ng * pl.ng) * (dx * dx + dy * dy);
                double a[3];
                exit_direction(pl.ng, pl.na, tmp, st2, a);
                cross3_f(a[0], a[1], a[2], sv[0], sv[1], sv[2], pout);
            }
        }
        const cd ls = dot_re(lam, sv), lp = dot_re(lam, pout);
        const cd as = cscale(cmul_f(cconj(cs), ls), scale), ap = cscale(cmul_f(cconj(cp), lp), scale);
        for (int c = 0; c < 3; ++c) lam[c] = mk(fma(as.re, sv[c], ap.re * pin[c]), fma(as.im, sv[c], ap.im * pin[c]));
    }
}

}  // namespace gwg
