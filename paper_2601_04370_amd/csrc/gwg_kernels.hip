// HIP kernels for gfx950: batched thin-film solve, forward Monte Carlo trace
// with fixed-point eyebox scatter, adjoint trace, gradient reduction,
// irradiance and loss.  Launch wrappers at the end are the only entry points
// used by the host API (gwg_api.cpp).
#include "gwg_internal.h"
#include "gwg_device.h"
#include "gwg_adjoint.h"
#include "gwg_trace.h"
#include "gwg_launch.h"

namespace gwg {

// ------------------------------------------------------------------ fills
__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f64(double* p, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// --------------------------------------------------------- LDS arrangement
struct SmemLayout {
    int off_pl, off_thk, off_slot, off_sp, off_q, off_c, off_st, off_grad, total;
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline SmemLayout smem_layout(int M, int Lmax, int n_slots, int wg, int B,
                                                  bool lds_bins, int n_grad_regions)
{
    SmemLayout s;
    int o = 0;
    s.off_pl = o; o = align16(o + (int)sizeof(PointLds));
    s.off_thk = o; o = align16(o + 8 * M * Lmax);
    s.off_slot = o; o = align16(o + M * Lmax);
    s.off_sp = o; o = align16(o + 8 * n_slots * NPF * wg);
    s.off_q = o; o = align16(o + (lds_bins ? 8 * B : 0));
    s.off_c = o; o = align16(o + (lds_bins ? 4 * B : 0));
    s.off_st = o; o = align16(o + 8 * ST_WORDS);
    s.off_grad = o; o = align16(o + 8 * n_grad_regions * M * Lmax);
    s.total = o;
    return s;
}

// Stage one point's uniform data and its design's stacks into LDS.
__device__ inline void stage_point(const SceneDev& sc, int d, int l, int f, PointLds* pl,
                                   double* s_thk, uint8_t* s_slot)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const double* lt = sc.lam_tab + (int64_t)l * LT_STRIDE;
    if (tid == 0) {
        pl->k0 = lt[LT_K0];
        pl->ng = lt[LT_NG];
        pl->na = lt[LT_NA];
        if (sc.fov_mode == 0) {
            const double* dv = sc.dir_tab + ((int64_t)l * sc.F + f) * 4;
            pl->dir[0] = dv[0]; pl->dir[1] = dv[1]; pl->dir[2] = dv[2];
        }
        for (int s = 0; s < kMaxSlots; ++s) {
            double nr = lt[LT_SLOT + 2 * s], ni = lt[LT_SLOT + 2 * s + 1];
            pl->slotN[2 * s] = nr; pl->slotN[2 * s + 1] = ni;
            pl->nsq[2 * s] = nr * nr - ni * ni; pl->nsq[2 * s + 1] = 2.0 * nr * ni;
            pl->crit[2 * s] = lt[LT_CRIT + 2 * s]; pl->crit[2 * s + 1] = lt[LT_CRIT + 2 * s + 1];
        }
        for (int m = 0; m < sc.M; ++m) {
            pl->h[m] = sc.h[m]; pl->sc_r[m] = sc.sc_r[m]; pl->sc_t[m] = sc.sc_t[m];
            pl->thr[m] = sc.thr[m];
            pl->nlay[m] = sc.nlay[(int64_t)d * sc.M + m];
        }
    }
    const int n = sc.M * sc.Lmax;
    const double* gthk = sc.thk + (int64_t)d * n;
    const uint8_t* gslot = sc.slot + (int64_t)d * n;
    for (int i = tid; i < n; i += nt) { s_thk[i] = gthk[i]; s_slot[i] = gslot[i]; }
}

__device__ inline void decode_item(const SceneDev& sc, int64_t item, int64_t* point, int* d, int* l,
                                   int* f, int64_t* i0, int64_t* i1)
{
    int64_t pt = item / sc.tiles_per_point;
    int64_t tile = item - pt * sc.tiles_per_point;
    *point = pt;
    *f = (int)(pt % sc.F);
    int64_t rest = pt / sc.F;
    *l = (int)(rest % sc.n_lsel);
    *d = (int)(rest / sc.n_lsel);
    *i0 = tile * sc.rays_per_tile;
    int64_t e = *i0 + sc.rays_per_tile;
    *i1 = e < sc.N ? e : sc.N;
}

// Per-hit thin-film coefficients for this lane (fills the lane's slot table).
template <int MODE>
__device__ inline Coef4 hit_coeffs(const SceneDev& sc, const PointLds& pl, const double* s_thk,
                                   const uint8_t* s_slot, double* sp, int ls, int m, bool front,
                                   double kappa, bool* used_fp64)
{
    for (int s = 0; s < sc.n_slots; ++s) {
        double P[NPF];
        slot_params(pl.slotN[2 * s], pl.slotN[2 * s + 1], kappa, pl.k0, P);
#pragma unroll
        for (int p = 0; p < NPF; ++p) sp[(s * NPF + p) * ls] = P[p];
    }
    double z0 = pl.ng * pl.ng - kappa * kappa;
    double q0 = sqrt(z0 > kTinyZ ? z0 : kTinyZ);
    double eta0s = q0, eta0p = pl.ng * pl.ng / q0;
    const int L = pl.nlay[m];
    const double* thk = s_thk + m * sc.Lmax;
    const uint8_t* slot = s_slot + m * sc.Lmax;
    bool fp64 = (MODE == GWG_FP64) || (MODE == GWG_FP32_MIXED && near_critical(pl, sc.n_slots, kappa));
    *used_fp64 = fp64;
    if (MODE == GWG_FP64)
        return tmm_solve<double>(thk, slot, L, front, sp, ls, sc.slot_complex, pl.k0, eta0s, eta0p,
                                 mk(eta0s, 0.0), mk(eta0p, 0.0), mk(1.0, 0.0));
    if (fp64)
        return tmm_solve<double>(thk, slot, L, front, sp, ls, sc.slot_complex, pl.k0, eta0s, eta0p,
                                 mk(eta0s, 0.0), mk(eta0p, 0.0), mk(1.0, 0.0));
    return tmm_solve<float>(thk, slot, L, front, sp, ls, sc.slot_complex, pl.k0, eta0s, eta0p,
                            mk(eta0s, 0.0), mk(eta0p, 0.0), mk(1.0, 0.0));
}

// Tape of one event for the adjoint (double slots of this lane, stride ts).
struct TapeRef { double* base; int64_t ts; };

__device__ inline void tape_put(TapeRef t, int k, const Ray& r_before, cd cs, cd cp, double scale,
                                int type, int m, int front, int refl)
{
    double* b = t.base + (int64_t)k * kTapeStride * t.ts;
    b[0] = r_before.dx; b[t.ts] = r_before.dy; b[2 * t.ts] = r_before.dz;
    for (int c = 0; c < 3; ++c) { b[(3 + 2 * c) * t.ts] = r_before.e[c].re; b[(4 + 2 * c) * t.ts] = r_before.e[c].im; }
    b[9 * t.ts] = cs.re; b[10 * t.ts] = cs.im; b[11 * t.ts] = cp.re; b[12 * t.ts] = cp.im;
    b[13 * t.ts] = scale;
    b[14 * t.ts] = (double)(type | (m << 4) | (front << 12) | (refl << 13));
}

// Outcome of a terminated ray.
struct Outcome { int cat; int bin; double w; double w_in; };

// Advance one ray through face events until it hits a mirror (returns the
// mirror index, event already counted) or terminates (returns -1, fills o).
template <bool TAPE>
__device__ inline int advance(const SceneDev& sc, const PointLds& pl, Ray& r, Outcome& o,
                              TapeRef tape, int* ntape)
{
    for (;;) {
        if (r.nev >= sc.Kmax) { o.cat = CAT_TRUNC; o.bin = -1; o.w = norm2(r.e); o.w_in = o.w; return -1; }
        int s = next_surface(sc, pl, r);
        if (s < 0) { o.cat = CAT_LOST; o.bin = -1; o.w = norm2(r.e); o.w_in = o.w; return -1; }
        r.nev++;
        if (s == SURF_TOP || s == SURF_BOTTOM) {
            FaceCoef fc = face_coeffs(pl.ng, pl.na, r.dx, r.dy, r.dz);
            double sv[3], pin[3], pout[3];
            s_basis(r.dx, r.dy, r.dz, 0.0, 0.0, 1.0, sv);
            cross3(r.dx, r.dy, r.dz, sv[0], sv[1], sv[2], pin);
            if (fc.tir) {
                cross3(r.dx, r.dy, -r.dz, sv[0], sv[1], sv[2], pout);
                if (TAPE) tape_put(tape, (*ntape)++, r, fc.rs, fc.rp, 1.0, EV_TIR, 0, 0, 0);
                apply_sp(r.e, sv, pin, pout, fc.rs, fc.rp, 1.0);
                r.dz = -r.dz;
                r.last = s;
                continue;
            }
            if (s == SURF_TOP) {
                double a[3];
                exit_direction(pl.ng, pl.na, r, fc.st2, a);
                cross3(a[0], a[1], a[2], sv[0], sv[1], sv[2], pout);
                o.w_in = norm2(r.e);
                if (TAPE) tape_put(tape, (*ntape)++, r, fc.ts, fc.tp, fc.flux, EV_EXIT, 0, 0, 0);
                apply_sp(r.e, sv, pin, pout, fc.ts, fc.tp, fc.flux);
                r.dx = a[0]; r.dy = a[1]; r.dz = a[2];
                o.w = norm2(r.e);
                o.bin = eyebox_bin(sc, r.px, r.py, a);
                o.cat = o.bin >= 0 ? CAT_EYEBOX : CAT_MISS;
                return -1;
            }
            o.cat = CAT_LEAK; o.bin = -1; o.w = norm2(r.e); o.w_in = o.w;
            return -1;
        }
        if (s == SURF_END0 || s == SURF_END1) {
            o.cat = CAT_END; o.bin = -1; o.w = norm2(r.e); o.w_in = o.w;
            return -1;
        }
        return s;
    }
}

// Mirror event: branch (Eq. 6), Eq. 5 field update, cell bookkeeping.
template <int MODE, bool TAPE>
__device__ inline void mirror_event(const SceneDev& sc, const PointLds& pl, const double* s_thk,
                                    const uint8_t* s_slot, double* sp, int ls, Ray& r, int m,
                                    TapeRef tape, int* ntape, bool* used_fp64)
{
    const double nx = sc.nx, nz = sc.nz;
    double dn = nx * r.dx + nz * r.dz;
    bool front = dn < 0.0;
    double c[3];
    cross3(r.dx, r.dy, r.dz, nx, 0.0, nz, c);
    double kappa = pl.ng * sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    Coef4 co = hit_coeffs<MODE>(sc, pl, s_thk, s_slot, sp, ls, m, front, kappa, used_fp64);
    int h = r.nprma;
    if ((h & 3) == 0) {
        u32x4 w = philox10((uint32_t)(uint64_t)r.id, (uint32_t)((uint64_t)r.id >> 32), (uint32_t)(h >> 2), 1u,
                           sc.key0, sc.key1);
        r.w4[0] = w.x; r.w4[1] = w.y; r.w4[2] = w.z; r.w4[3] = w.w;
    }
    const int hw = h & 3;
    uint32_t word = hw == 0 ? r.w4[0] : hw == 1 ? r.w4[1] : hw == 2 ? r.w4[2] : r.w4[3];
    bool refl = word < pl.thr[m];
    double ndx = r.dx, ndz = r.dz;
    if (refl) mirror_reflect(nx, nz, r.dx, r.dz, &ndx, &ndz);
    double sv[3], pin[3], pout[3];
    s_basis(r.dx, r.dy, r.dz, nx, 0.0, nz, sv);
    cross3(r.dx, r.dy, r.dz, sv[0], sv[1], sv[2], pin);
    cross3(ndx, r.dy, ndz, sv[0], sv[1], sv[2], pout);
    cd cs = refl ? co.rs : co.ts;
    cd cp = refl ? co.rp : co.tp;
    double scale = refl ? pl.sc_r[m] : pl.sc_t[m];
    if (TAPE) tape_put(tape, (*ntape)++, r, cs, cp, scale, EV_MIRROR, m, front ? 1 : 0, refl ? 1 : 0);
    apply_sp(r.e, sv, pin, pout, cs, cp, scale);
    r.dx = ndx; r.dz = ndz;
    if (!refl) r.cell += (m == r.cell) ? 1 : -1;
    r.last = m;
    r.nprma++;
}

// ======================================================== forward kernel
// One workgroup per work item (design, wavelength, FoV point, ray tile).  Each
// lane traces rays tile_start + lane, + blockDim, ...; a lane whose ray
// terminates starts its next ray within the same step so that every mirror
// solve of the wave runs with as many lanes as possible.  Eyebox bins of the
// point accumulate in LDS (integer atomics) and are flushed with integer
// global atomics, so results do not depend on scheduling.
template <int MODE>
__global__ void __launch_bounds__(256) k_trace_fwd(SceneDev sc, uint64_t* __restrict__ q_out,
                                                   uint32_t* __restrict__ c_out,
                                                   unsigned long long* __restrict__ stats,
                                                   gwg_ray_record* __restrict__ rec, int64_t rec_stride,
                                                   int lds_bins)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int B = sc.bins_x * sc.bins_y;
    const SmemLayout lay = smem_layout(sc.M, sc.Lmax, sc.n_slots, blockDim.x, B, lds_bins != 0, 0);
    PointLds* pl = (PointLds*)(smem + lay.off_pl);
    double* s_thk = (double*)(smem + lay.off_thk);
    uint8_t* s_slot = (uint8_t*)(smem + lay.off_slot);
    double* s_sp = (double*)(smem + lay.off_sp);
    unsigned long long* s_q = (unsigned long long*)(smem + lay.off_q);
    uint32_t* s_c = (uint32_t*)(smem + lay.off_c);
    unsigned long long* s_st = (unsigned long long*)(smem + lay.off_st);

    int64_t point, i0, i1;
    int d, l, f;
    decode_item(sc, blockIdx.x, &point, &d, &l, &f, &i0, &i1);
    stage_point(sc, d, l, f, pl, s_thk, s_slot);
    const int tid = threadIdx.x, WG = blockDim.x;
    if (lds_bins)
        for (int i = tid; i < B; i += WG) { s_q[i] = 0ull; s_c[i] = 0u; }
    for (int i = tid; i < ST_WORDS; i += WG) s_st[i] = 0ull;
    __syncthreads();

    double* sp = s_sp + tid;
    const int64_t base = point * sc.N;
    uint64_t* gq = q_out + point * B;
    uint32_t* gc = c_out + point * B;
    const double wscale = ldexp(1.0, sc.fp_shift), wcap = ldexp(1.0, 40), pscale = 16777216.0;

    int64_t i = i0 + tid;
    bool have = i < i1;
    Ray r;
    if (have) ray_birth(sc, *pl, base + i, r);
    unsigned long long n_fp64 = 0, n_lay = 0;
    for (;;) {
        int m = -1;
        while (have) {
            Outcome o;
            TapeRef none = { nullptr, 0 };
            int nt = 0;
            m = advance<false>(sc, *pl, r, o, none, &nt);
            if (m >= 0) break;
            // terminated: scatter and bookkeeping
            atomicAdd(&s_st[ST_RAYS], 1ull);
            atomicAdd(&s_st[ST_EVENTS], (unsigned long long)r.nev);
            atomicAdd(&s_st[ST_PRMA], (unsigned long long)r.nprma);
            atomicAdd(&s_st[ST_CAT + o.cat], 1ull);
            double pw = o.w * pscale;
            atomicAdd(&s_st[ST_POW + o.cat], (unsigned long long)rint(pw < wcap ? pw : wcap));
            if (o.cat == CAT_EYEBOX || o.cat == CAT_MISS) {
                double pr = (o.w_in - o.w) * pscale;
                if (pr > 0.0) atomicAdd(&s_st[ST_POW + CAT_FACE_R], (unsigned long long)rint(pr < wcap ? pr : wcap));
            }
            if (o.cat == CAT_EYEBOX) {
                double u = o.w * wscale;
                if (u > wcap) { u = wcap; atomicAdd(&s_st[ST_SAT], 1ull); }
                unsigned long long qv = (unsigned long long)rint(u);
                if (lds_bins) { atomicAdd(&s_q[o.bin], qv); atomicAdd(&s_c[o.bin], 1u); }
                else { atomicAdd((unsigned long long*)&gq[o.bin], qv); atomicAdd(&gc[o.bin], 1u); }
            }
            if (rec && (r.id % rec_stride) == 0) {
                gwg_ray_record* q = rec + r.id / rec_stride;
                q->bin = o.cat == CAT_EYEBOX ? o.bin : -1;
                q->category = o.cat;
                q->n_events = r.nev;
                q->n_prma = r.nprma;
                q->w = o.w;
            }
            i += WG;
            have = i < i1;
            if (have) ray_birth(sc, *pl, base + i, r);
            m = -1;
        }
        if (!__any(m >= 0)) break;
        if (m >= 0) {
            TapeRef none = { nullptr, 0 };
            int nt = 0;
            bool u64 = false;
            mirror_event<MODE, false>(sc, *pl, s_thk, s_slot, sp, WG, r, m, none, &nt, &u64);
            n_fp64 += u64 ? 1ull : 0ull;
            n_lay += (unsigned long long)pl->nlay[m];
        }
    }
    if (n_fp64) atomicAdd(&s_st[ST_FP64], n_fp64);
    if (n_lay) atomicAdd(&s_st[ST_LAYERS], n_lay);
    __syncthreads();
    if (lds_bins) {
        for (int k = tid; k < B; k += WG) {
            if (s_c[k]) {
                atomicAdd((unsigned long long*)&gq[k], s_q[k]);
                atomicAdd(&gc[k], s_c[k]);
            }
        }
    }
    for (int k = tid; k < ST_WORDS; k += WG)
        if (s_st[k]) atomicAdd(&stats[k], s_st[k]);
}

#include "gwg_bwd_kernel.h"

// Sum per-item partial gradients in item order: grad[d][k] = sum_items(d) partial[item][k].
__global__ void k_grad_reduce(const double* __restrict__ partial, int64_t items_per_design, int ML,
                              int D, double* __restrict__ grad)
{
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)D * ML) return;
    int d = (int)(gid / ML), k = (int)(gid % ML);
    const double* p = partial + (int64_t)d * items_per_design * ML + k;
    double acc = 0.0;
    for (int64_t it = 0; it < items_per_design; ++it) acc += p[it * ML];
    grad[gid] = acc;
}

__global__ void k_mask_padding(double* grad, const int32_t* nlay, int D, int M, int Lmax)
{
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)D * M * Lmax) return;
    int j = (int)(gid % Lmax);
    int64_t dm = gid / Lmax;
    if (j >= nlay[dm]) grad[gid] = 0.0;
}

__global__ void k_irradiance(const uint64_t* __restrict__ q, int64_t n, double scale, double* __restrict__ irr)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        irr[i] = (double)q[i] * scale;
}

// ======================================================== thin-film queries
template <int MODE>
__global__ void __launch_bounds__(256) k_tmm_rt(const double* __restrict__ thk, const uint8_t* __restrict__ slot,
                                                int L, const double* __restrict__ lam_tab, int n_lambda,
                                                int n_slots, uint32_t cplx_mask,
                                                const int32_t* __restrict__ lidx,
                                                const double* __restrict__ theta, int64_t nq,
                                                double* __restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double* s_thk = (double*)smem;
    uint8_t* s_slot = (uint8_t*)(smem + align16(8 * L));
    double* s_sp = (double*)(smem + align16(8 * L) + align16(L > 0 ? L : 1));
    for (int i = threadIdx.x; i < L; i += blockDim.x) { s_thk[i] = thk[i]; s_slot[i] = slot[i]; }
    __syncthreads();
    double* sp = s_sp + threadIdx.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
        int li = lidx[q];
        double th = theta[q];
        double* o = out + q * 8;
        if (li < 0 || li >= n_lambda || !(th >= 0.0 && th < 1.5707963267948966)) {
            for (int k = 0; k < 8; ++k) o[k] = __builtin_nan("");
            continue;
        }
        const double* lt = lam_tab + (int64_t)li * LT_STRIDE;
        double k0 = lt[LT_K0], n0 = lt[LT_NG];
        cd NE = mk(lt[LT_NA], lt[LT_NA + 1]);
        double kappa = n0 * sin(th);
        for (int s = 0; s < n_slots; ++s) {
            double P[NPF];
            slot_params(lt[LT_SLOT + 2 * s], lt[LT_SLOT + 2 * s + 1], kappa, k0, P);
#pragma unroll
            for (int p = 0; p < NPF; ++p) sp[(s * NPF + p) * blockDim.x] = P[p];
        }
        double z0 = n0 * n0 - kappa * kappa;
        double q0 = sqrt(z0 > kTinyZ ? z0 : kTinyZ);
        cd NE2 = cmul(NE, NE);
        cd zE = csub(NE2, mk(kappa * kappa, 0.0));
        if (zE.im == 0.0 && fabs(zE.re) < kTinyZ) zE.re = kTinyZ;
        cd qE = csqrt_up(zE);
        cd etaEp = cdiv(NE2, qE);
        // t_p factor cos(theta_0) / cos(theta_exit) = (q0 / n0) / (qE / NE)
        cd tpf = cdiv(cscale(NE, q0 / n0), qE);
        bool fp64 = (MODE == GWG_FP64);
        if (MODE == GWG_FP32_MIXED) {
            for (int s = 0; s < n_slots; ++s)
                fp64 |= (kappa > lt[LT_CRIT + 2 * s] && kappa < lt[LT_CRIT + 2 * s + 1]);
        }
        Coef4 c = fp64 ? tmm_solve<double>(s_thk, s_slot, L, true, sp, blockDim.x, cplx_mask, k0, q0, n0 * n0 / q0, qE, etaEp, tpf)
                       : tmm_solve<float>(s_thk, s_slot, L, true, sp, blockDim.x, cplx_mask, k0, q0, n0 * n0 / q0, qE, etaEp, tpf);
        o[0] = c.rs.re; o[1] = c.rs.im; o[2] = c.rp.re; o[3] = c.rp.im;
        o[4] = c.ts.re; o[5] = c.ts.im; o[6] = c.tp.re; o[7] = c.tp.im;
    }
}

// ======================================================== loss (FP64)
// eta[d][l][f] = sum_b I  (one block per point, fixed-shape tree reduction)
__global__ void __launch_bounds__(256) k_loss_eta(const double* __restrict__ I, int B, double* __restrict__ eta)
{
    __shared__ double red[256];
    const double* row = I + (int64_t)blockIdx.x * B;
    double acc = 0.0;
    for (int b = threadIdx.x; b < B; b += blockDim.x) acc += row[b];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) eta[blockIdx.x] = red[0];
}

// E[d][b] = mean over (l, f) of I  (one thread per (d, b), fixed order)
__global__ void k_loss_eyeb(const double* __restrict__ I, int D, int nlf, int B, double* __restrict__ E)
{
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)D * B) return;
    int d = (int)(gid / B), b = (int)(gid % B);
    const double* p = I + (int64_t)d * nlf * B + b;
    double acc = 0.0;
    for (int k = 0; k < nlf; ++k) acc += p[(int64_t)k * B] / (double)nlf;
    E[gid] = acc;
}

// Per design: moments and the coefficients of dL/dI (one thread per design).
// coef[d] = { L_d, a_e, a_f, m_e, m_f, ebar, ibar } ; phi[d][f] written too.
__global__ void k_loss_scalar(const double* __restrict__ eta, const double* __restrict__ E, int D, int nl,
                              int F, int B, int kind, double w_f, double w_e, double* __restrict__ phi,
                              double* __restrict__ coef, double* __restrict__ loss)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double total = 0.0;
    for (int d = 0; d < D; ++d) {
        const double* et = eta + (int64_t)d * nl * F;
        double* ph = phi + (int64_t)d * F;
        double npts = (double)nl * (double)F;
        double ibar = 0.0;
        for (int f = 0; f < F; ++f) ph[f] = 0.0;
        for (int l = 0; l < nl; ++l)
            for (int f = 0; f < F; ++f) {
                double v = et[(int64_t)l * F + f];
                ph[f] += v / (double)nl;
                ibar += v / npts;
            }
        const double* Ed = E + (int64_t)d * B;
        double ebar = 0.0;
        for (int b = 0; b < B; ++b) ebar += Ed[b] / (double)B;
        double ve = 0.0, vf = 0.0;
        for (int b = 0; b < B; ++b) ve += (Ed[b] - ebar) * (Ed[b] - ebar) / (double)B;
        for (int f = 0; f < F; ++f) vf += (ph[f] - ibar) * (ph[f] - ibar) / (double)F;
        double L, ae, af, me, mf;
        if (kind == 0) {
            L = -ibar + w_e * ve + w_f * vf;
            ae = w_e; af = w_f; me = 0.0; mf = 0.0;
        } else {
            double se = sqrt(ve), sf = sqrt(vf);
            L = -ibar + w_f * (sf / ibar) + w_e * (se / ebar);
            ae = se > 0.0 ? w_e / (2.0 * se * ebar) : 0.0;
            af = sf > 0.0 ? w_f / (2.0 * sf * ibar) : 0.0;
            me = -w_e * se / (ebar * ebar);
            mf = -w_f * sf / (ibar * ibar);
        }
        double* c = coef + (int64_t)d * 8;
        c[0] = L; c[1] = ae; c[2] = af; c[3] = me; c[4] = mf; c[5] = ebar; c[6] = ibar;
        total += L;
    }
    loss[0] = total;
}

__global__ void k_loss_grad(const double* __restrict__ E, const double* __restrict__ phi,
                            const double* __restrict__ coef, int D, int nl, int F, int B,
                            double* __restrict__ G)
{
    int64_t n = (int64_t)D * nl * F * B;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int b = (int)(i % B);
        int64_t r = i / B;
        int f = (int)(r % F);
        r /= F;
        r /= nl;
        int d = (int)r;
        const double* c = coef + (int64_t)d * 8;
        double npts = (double)nl * (double)F;
        double ce = 2.0 * (E[(int64_t)d * B + b] - c[5]) / ((double)B * npts);
        double cf = 2.0 * (phi[(int64_t)d * F + f] - c[6]) / ((double)F * (double)nl);
        G[i] = -1.0 / npts + c[1] * ce + c[2] * cf + c[3] / ((double)B * npts) + c[4] / npts;
    }
}

// ======================================================== launch wrappers
static inline int grid_for(int64_t n, int bs, int cap = 65536)
{
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

size_t fwd_smem_bytes(const SceneDev& sc, int wg, bool lds_bins)
{
    return (size_t)smem_layout(sc.M, sc.Lmax, sc.n_slots, wg, sc.bins_x * sc.bins_y, lds_bins, 0).total;
}
size_t bwd_smem_bytes(const SceneDev& sc, int wg)
{
    return (size_t)smem_layout(sc.M, sc.Lmax, sc.n_slots, wg, sc.bins_x * sc.bins_y, false, (wg + 63) / 64).total;
}

hipError_t launch_trace_fwd(const SceneDev& sc, int wg, bool lds_bins, uint64_t* q, uint32_t* c,
                            unsigned long long* stats, gwg_ray_record* rec, int64_t rec_stride,
                            hipStream_t s)
{
    size_t sm = fwd_smem_bytes(sc, wg, lds_bins);
    dim3 grid((unsigned)sc.n_items), block(wg);
    switch (sc.precision) {
    case GWG_FP64:
        hipLaunchKernelGGL(k_trace_fwd<GWG_FP64>, grid, block, sm, s, sc, q, c, stats, rec, rec_stride, (int)lds_bins);
        break;
    case GWG_FP32_MIXED:
        hipLaunchKernelGGL(k_trace_fwd<GWG_FP32_MIXED>, grid, block, sm, s, sc, q, c, stats, rec, rec_stride, (int)lds_bins);
        break;
    default:
        hipLaunchKernelGGL(k_trace_fwd<GWG_FP32>, grid, block, sm, s, sc, q, c, stats, rec, rec_stride, (int)lds_bins);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_trace_bwd(const SceneDev& sc, int wg, int grid_blocks, const double* dLdI, unsigned long long* stats,
                            double* partial, double* scratch, int64_t sample_stride, hipStream_t s)
{
    size_t sm = bwd_smem_bytes(sc, wg);
    dim3 grid((unsigned)grid_blocks), block(wg);
    switch (sc.precision) {
    case GWG_FP64:
        hipLaunchKernelGGL(k_trace_bwd<GWG_FP64>, grid, block, sm, s, sc, dLdI, partial, scratch, sample_stride, stats);
        break;
    case GWG_FP32_MIXED:
        hipLaunchKernelGGL(k_trace_bwd<GWG_FP32_MIXED>, grid, block, sm, s, sc, dLdI, partial, scratch, sample_stride, stats);
        break;
    default:
        hipLaunchKernelGGL(k_trace_bwd<GWG_FP32>, grid, block, sm, s, sc, dLdI, partial, scratch, sample_stride, stats);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double* partial, int64_t items_per_design, int ML, int D,
                              double* grad, const int32_t* nlay, int M, int Lmax, hipStream_t s)
{
    int64_t n = (int64_t)D * ML;
    hipLaunchKernelGGL(k_grad_reduce, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, s, partial, items_per_design, ML, D, grad);
    hipLaunchKernelGGL(k_mask_padding, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, s, grad, nlay, D, M, Lmax);
    return hipGetLastError();
}

hipError_t launch_irradiance(const uint64_t* q, int64_t n, double scale, double* irr, hipStream_t s)
{
    hipLaunchKernelGGL(k_irradiance, dim3(grid_for(n, 256)), dim3(256), 0, s, q, n, scale, irr);
    return hipGetLastError();
}

size_t tmm_smem_bytes(int L, int n_slots, int wg)
{
    return (size_t)(align16(8 * L) + align16(L > 0 ? L : 1) + 8 * n_slots * NPF * wg);
}

hipError_t launch_tmm_rt(int precision, const double* thk, const uint8_t* slot, int L,
                         const double* lam_tab, int n_lambda, int n_slots, uint32_t cplx_mask,
                         const int32_t* lidx, const double* theta, int64_t nq, double* out, hipStream_t s)
{
    const int wg = 256;
    size_t sm = tmm_smem_bytes(L, n_slots, wg);
    dim3 grid(grid_for(nq, wg, 8192)), block(wg);
    switch (precision) {
    case GWG_FP64:
        hipLaunchKernelGGL(k_tmm_rt<GWG_FP64>, grid, block, sm, s, thk, slot, L, lam_tab, n_lambda, n_slots, cplx_mask, lidx, theta, nq, out);
        break;
    case GWG_FP32_MIXED:
        hipLaunchKernelGGL(k_tmm_rt<GWG_FP32_MIXED>, grid, block, sm, s, thk, slot, L, lam_tab, n_lambda, n_slots, cplx_mask, lidx, theta, nq, out);
        break;
    default:
        hipLaunchKernelGGL(k_tmm_rt<GWG_FP32>, grid, block, sm, s, thk, slot, L, lam_tab, n_lambda, n_slots, cplx_mask, lidx, theta, nq, out);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_loss(const double* I, int D, int nl, int F, int B, int kind, double w_f, double w_e,
                       double* work, double* loss, double* G, hipStream_t s)
{
    // work: eta [D nl F] | E [D B] | phi [D F] | coef [D 8]
    double* eta = work;
    double* E = eta + (int64_t)D * nl * F;
    double* phi = E + (int64_t)D * B;
    double* coef = phi + (int64_t)D * F;
    hipLaunchKernelGGL(k_loss_eta, dim3((unsigned)((int64_t)D * nl * F)), dim3(256), 0, s, I, B, eta);
    hipLaunchKernelGGL(k_loss_eyeb, dim3(grid_for((int64_t)D * B, 256, 1 << 30)), dim3(256), 0, s, I, D, nl * F, B, E);
    hipLaunchKernelGGL(k_loss_scalar, dim3(1), dim3(64), 0, s, eta, E, D, nl, F, B, kind, w_f, w_e, phi, coef, loss);
    if (G) hipLaunchKernelGGL(k_loss_grad, dim3(grid_for((int64_t)D * nl * F * B, 256)), dim3(256), 0, s, E, phi, coef, D, nl, F, B, G);
    return hipGetLastError();
}

}  // namespace gwg
