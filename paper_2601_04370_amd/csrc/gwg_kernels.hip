// HIP kernels for gfx950: batched thin-film solve, forward Monte Carlo trace
// with fixed-point eyebox scatter, adjoint trace, gradient reduction,
// irradiance and loss.  Launch wrappers at the end are the only entry points
// used by the host API (gwg_api.cpp).
#include <mutex>
#include <type_traits>

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

// recs: the stacks as layer records (LayerRec, off_thk; no slot array)
// rather than thickness and slot arrays.
__host__ __device__ inline SmemLayout smem_layout(int M, int Lmax, int n_slots, int wg, int B,
                                                  bool lds_bins, int n_grad_regions, int slot_per = LaneSlots3::kPer,
                                                  bool recs = false)
{
    SmemLayout s;
    int o = 0;
    s.off_pl = o; o = align16(o + (int)sizeof(PointLds));
    s.off_thk = o; o = align16(o + (recs ? (int)sizeof(LayerRec) * M * rec_stride(Lmax) : 8 * M * Lmax));
    s.off_slot = o; o = align16(o + (recs ? 0 : M * Lmax));
    s.off_sp = o; o = align16(o + 8 * n_slots * slot_per * ((wg + 63) / 64 * 64));   // whole waves
    s.off_q = o; o = align16(o + (lds_bins ? 8 * B : 0));
    s.off_c = o; o = align16(o + (lds_bins ? 4 * B : 0));
    s.off_st = o; o = align16(o + 8 * ST_WORDS);
    s.off_grad = o; o = align16(o + 8 * n_grad_regions * M * Lmax);
    s.total = o;
    return s;
}

// Stage one point's uniform data and its design's stacks into LDS: as
// thickness and slot arrays (s_thk, s_slot) or as layer records (s_rec, for
// slot tables of `per` values per slot).
__device__ inline void stage_point(const SceneDev& sc, int d, int l, int f, PointLds* pl,
                                   double* s_thk, uint8_t* s_slot, LayerRec* s_rec = nullptr, int per = 0)
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
        double k2e = 1e300;
        for (int s = 0; s < sc.n_slots; ++s)
            if (!((sc.slot_complex >> s) & 1u)) {
                const double nr = lt[LT_SLOT + 2 * s];
                k2e = fmin(k2e, nr * nr);
            }
        pl->kap2_evan = k2e;
        for (int s = 0; s < kMaxSlots; ++s) {
            double nr = lt[LT_SLOT + 2 * s], ni = lt[LT_SLOT + 2 * s + 1];
            pl->slotN[2 * s] = nr; pl->slotN[2 * s + 1] = ni;
            pl->nsq[2 * s] = nr * nr - ni * ni; pl->nsq[2 * s + 1] = 2.0 * nr * ni;
            pl->pxy[2 * s] = (ni == 0.0 && nr != 0.0) ? 1.0 / (nr * nr) : 0.0;
            pl->pxy[2 * s + 1] = nr * nr - ni * ni;
            pl->crit[2 * s] = lt[LT_CRIT + 2 * s]; pl->crit[2 * s + 1] = lt[LT_CRIT + 2 * s + 1];
        }
        for (int m = 0; m < sc.M; ++m) {
            pl->h[m] = sc.h[m]; pl->sc_r[m] = sc.sc_r[m]; pl->sc_t[m] = sc.sc_t[m];
            pl->thr[m] = sc.thr[m];
            pl->nlay[m] = sc.nlay[(int64_t)d * sc.M + m];
        }
        pl->T = sc.T; pl->Lx = sc.Lx; pl->nx = sc.nx; pl->nz = sc.nz; pl->ER = sc.ER;
        pl->ex0 = sc.ex0; pl->ew = sc.ew; pl->ey0 = sc.ey0; pl->eh = sc.eh;
        pl->M = sc.M; pl->Kmax = sc.Kmax; pl->bins_x = sc.bins_x; pl->bins_y = sc.bins_y;
    }
    const int n = sc.M * sc.Lmax;
    const double* gthk = sc.thk + (int64_t)d * n;
    const uint8_t* gslot = sc.slot + (int64_t)d * n;
    if (s_rec)
        stage_recs(s_rec, gthk, gslot, sc.M, sc.Lmax, per);
    else
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

// Work items are drawn from a launch-wide counter (a stats word cleared
// before the launch) rather than by a fixed stride over blocks: a block that
// drew cheap items goes on to the next one, so the launch ends within about
// one item of the mean.  Every output is indexed by item, never by block,
// so results do not depend on which block ran an item.  Called by the whole
// block.
__device__ inline int64_t draw_item(unsigned long long* ctr)
{
    __shared__ long long s_item;
    __syncthreads();                                   // the previous draw has been read
    if (threadIdx.x == 0) s_item = (long long)atomicAdd(ctr, 1ull);
    __syncthreads();
    return s_item;
}

#include "gwg_table.h"
#include "gwg_fwd_kernel.h"
#include "gwg_bwd_kernel.h"
#include "gwg_memo_kernel.h"
#include "gwg_table_kernel.h"
#include "gwg_omega_kernel.h"

// Sum per-item partial gradients in item order: grad[d][k] = sum_items(d) partial[item][k].
// Gradient reduction over the per-item partials, in two launches with a
// fixed order of additions (the gradient is the same bit for bit from run to
// run): range r of kGradRanges contiguous item ranges of a design is summed
// in item order, then the range sums in range order.
constexpr int kGradRanges = 64;

__global__ void k_grad_ranges(const double* __restrict__ partial, int64_t items_per_design, int ML,
                              double* __restrict__ tmp)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y, d = blockIdx.z;
    if (k >= ML) return;
    const int64_t a = items_per_design * r / kGradRanges, b = items_per_design * (r + 1) / kGradRanges;
    const double* p = partial + (int64_t)d * items_per_design * ML + k;
    double acc = 0.0;
    for (int64_t it = a; it < b; ++it) acc += p[it * ML];
    tmp[((int64_t)d * kGradRanges + r) * ML + k] = acc;
}

__global__ void k_grad_reduce(const double* __restrict__ tmp, int ML, int D, double* __restrict__ grad)
{
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)D * ML) return;
    int d = (int)(gid / ML), k = (int)(gid % ML);
    const double* p = tmp + (int64_t)d * kGradRanges * ML + k;
    double acc = 0.0;
    for (int r = 0; r < kGradRanges; ++r) acc += p[(int64_t)r * ML];
    grad[gid] = acc;
}

int64_t grad_reduce_tmp_doubles(int ML, int D) { return (int64_t)D * kGradRanges * ML; }

// Work items in decreasing order of a per-(item, wave) work count summed
// over the item's waves (adjoint entries; mirror hits of the last forward),
// by a counting sort over count >> shift in one workgroup.  Items in one
// bucket are placed in no particular order; the kernels' outputs are indexed
// by item, so their results do not depend on it.
constexpr int kOrderBuckets = 2048;

__global__ void __launch_bounds__(1024) k_item_order(const int32_t* __restrict__ cnt, int waves, int64_t n_items,
                                                     int shift, int32_t* __restrict__ order)
{
    __shared__ int hist[kOrderBuckets];
    __shared__ int part[1024];
    const int t = threadIdx.x;
    auto bucket = [&](int64_t it) {
        long long n = 0;
        for (int w = 0; w < waves; ++w) n += cnt[it * waves + w];
        const long long b = n > 0 ? n >> shift : 0;     // any count maps into the histogram
        return kOrderBuckets - 1 - (int)(b < kOrderBuckets ? b : kOrderBuckets - 1);   // largest first
    };
    for (int k = t; k < kOrderBuckets; k += 1024) hist[k] = 0;
    __syncthreads();
    for (int64_t it = t; it < n_items; it += 1024) atomicAdd(&hist[bucket(it)], 1);
    __syncthreads();
    // exclusive prefix sum over the buckets: two per thread, then a scan of
    // the 1024 pair sums
    const int a0 = hist[2 * t], a1 = hist[2 * t + 1];
    part[t] = a0 + a1;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const int base = part[t] - (a0 + a1);
    hist[2 * t] = base;
    hist[2 * t + 1] = base + a0;
    __syncthreads();
    for (int64_t it = t; it < n_items; it += 1024) order[atomicAdd(&hist[bucket(it)], 1)] = (int32_t)it;
}

hipError_t launch_item_order(const int32_t* cnt, int waves, int64_t n_items, int64_t max_count, int32_t* order,
                             hipStream_t s)
{
    int shift = 0;
    while ((max_count >> shift) >= kOrderBuckets) ++shift;
    hipLaunchKernelGGL(k_item_order, dim3(1), dim3(1024), 0, s, cnt, waves, n_items, shift, order);
    return hipGetLastError();
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
    LayerRec* s_rec = (LayerRec*)smem;
    double* s_sp = (double*)(smem + sizeof(LayerRec) * rec_stride(L));
    stage_recs(s_rec, thk, slot, 1, L, LaneSlots5::kPer);
    __syncthreads();
    const LaneSlots5 sl = { slot_lane_base(s_sp, n_slots, LaneSlots5::kPer, threadIdx.x) };
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
            sl.put(s, P);
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
        const RecStack stk = { s_rec + kRecPad };
        Coef4 c = fp64 ? tmm_solve<double>(stk, L, true, sl, cplx_mask, k0, q0, n0 * n0 / q0, qE, etaEp, tpf)
                       : tmm_solve<float>(stk, L, true, sl, cplx_mask, k0, q0, n0 * n0 / q0, qE, etaEp, tpf);
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

// E[d][b] = mean over (l, f) of I.  One block of 1024 threads per (design,
// 64 bins): wave w sums the rows k = w, w + 16, ... in order, then lane b's
// 16 wave sums are added in wave order (a fixed order).
__global__ void __launch_bounds__(1024) k_loss_eyeb(const double* __restrict__ I, int D, int nlf, int B,
                                                    double* __restrict__ E)
{
    __shared__ double part[16][64];
    const int tiles = (B + 63) / 64;
    const int d = blockIdx.x / tiles, b = (blockIdx.x % tiles) * 64 + (threadIdx.x & 63), w = threadIdx.x >> 6;
    double acc = 0.0;
    if (b < B) {
        const double* p = I + (int64_t)d * nlf * B + b;
        for (int k = w; k < nlf; k += 16) acc += p[(int64_t)k * B] / (double)nlf;
    }
    part[w][threadIdx.x & 63] = acc;
    __syncthreads();
    if (w == 0 && b < B) {
        double e = 0.0;
        for (int k = 0; k < 16; ++k) e += part[k][threadIdx.x];
        E[(int64_t)d * B + b] = e;
    }
}

// Sum over the block of each thread's v: a fixed tree over the 256 threads.
__device__ inline double block_sum256(double v, double* red)
{
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

// Per design (one block of 256 threads each): moments and the coefficients
// of dL/dI.  coef[d] = { L_d, a_e, a_f, m_e, m_f, ebar, ibar, bright };
// phi[d][f] written too.  bright weighs the throughput's mean in the
// brightness term: 1, or 1 / B for pupil images (kind 2), whose brightness is
// the mean over pupils rather than the sum over bins.  Sums are strided per thread, then a fixed tree.
__global__ void __launch_bounds__(256) k_loss_scalar(const double* __restrict__ eta, const double* __restrict__ E,
                                                     int nl, int F, int B, int kind, double w_f, double w_e,
                                                     double* __restrict__ phi, double* __restrict__ coef)
{
    __shared__ double red[256];
    const int d = blockIdx.x, t = threadIdx.x;
    const double* et = eta + (int64_t)d * nl * F;
    double* ph = phi + (int64_t)d * F;
    const double npts = (double)nl * (double)F;
    double part = 0.0;
    for (int f = t; f < F; f += 256) {
        double a = 0.0;
        for (int l = 0; l < nl; ++l) {
            const double v = et[(int64_t)l * F + f];
            a += v / (double)nl;
            part += v / npts;
        }
        ph[f] = a;
    }
    const double ibar = block_sum256(part, red);
    const double* Ed = E + (int64_t)d * B;
    part = 0.0;
    for (int b = t; b < B; b += 256) part += Ed[b] / (double)B;
    const double ebar = block_sum256(part, red);
    part = 0.0;
    for (int b = t; b < B; b += 256) part += (Ed[b] - ebar) * (Ed[b] - ebar) / (double)B;
    const double ve = block_sum256(part, red);
    part = 0.0;
    for (int f = t; f < F; f += 256) part += (ph[f] - ibar) * (ph[f] - ibar) / (double)F;   // this thread's own ph[f]
    const double vf = block_sum256(part, red);
    if (t != 0) return;
    double L, ae, af, me, mf;
    const double bright = kind == 2 ? 1.0 / (double)B : 1.0;
    if (kind == 0) {
        L = -ibar + w_e * ve + w_f * vf;
        ae = w_e; af = w_f; me = 0.0; mf = 0.0;
    } else {
        double se = sqrt(ve), sf = sqrt(vf);
        L = -ibar * bright + w_f * (sf / ibar) + w_e * (se / ebar);
        ae = se > 0.0 ? w_e / (2.0 * se * ebar) : 0.0;
        af = sf > 0.0 ? w_f / (2.0 * sf * ibar) : 0.0;
        me = -w_e * se / (ebar * ebar);
        mf = -w_f * sf / (ibar * ibar);
    }
    double* c = coef + (int64_t)d * 8;
    c[0] = L; c[1] = ae; c[2] = af; c[3] = me; c[4] = mf; c[5] = ebar; c[6] = ibar; c[7] = bright;
}

// Total loss: the designs' L_d in design order.
__global__ void k_loss_total(const double* __restrict__ coef, int D, double* __restrict__ loss)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double total = 0.0;
    for (int d = 0; d < D; ++d) total += coef[(int64_t)d * 8];
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
        G[i] = -c[7] / npts + c[1] * ce + c[2] * cf + c[3] / ((double)B * npts) + c[4] / npts;
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
    return (size_t)smem_layout(sc.M, sc.Lmax, sc.n_slots, wg, sc.bins_x * sc.bins_y, lds_bins, 0,
                               sc.memo ? LaneSlots3::kPer : LaneSlots3x::kPer, true).total
           + (sc.memo ? (size_t)(wg / 64) * fwd_memo_wave_bytes() : 0);
}
size_t bwd_smem_bytes(const SceneDev& sc, int wg)
{
    return (size_t)smem_layout(sc.M, sc.Lmax, sc.n_slots, wg, sc.bins_x * sc.bins_y, false, (wg + 63) / 64).total;
}

template <class K>
static int blocks_per_cu(K kernel, int wg, size_t smem)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, wg, smem) != hipSuccess || n < 1) n = 1;
    return n;
}

template <bool ADJ, bool TAB, bool MEMO = false>
static int fwd_blocks_per_cu(int precision, int wg, size_t smem)
{
    if (precision == GWG_FP64) return blocks_per_cu(k_trace_fwd<GWG_FP64, ADJ, TAB, MEMO>, wg, smem);
    if (precision == GWG_FP32_MIXED) return blocks_per_cu(k_trace_fwd<GWG_FP32_MIXED, ADJ, TAB, MEMO>, wg, smem);
    return blocks_per_cu(k_trace_fwd<GWG_FP32, ADJ, TAB, MEMO>, wg, smem);
}

template <bool TAB>
static int bwd_blocks_per_cu(int precision, int wg, size_t smem)
{
    if (precision == GWG_FP64) return blocks_per_cu(k_trace_bwd<GWG_FP64, TAB>, wg, smem);
    if (precision == GWG_FP32_MIXED) return blocks_per_cu(k_trace_bwd<GWG_FP32_MIXED, TAB>, wg, smem);
    return blocks_per_cu(k_trace_bwd<GWG_FP32, TAB>, wg, smem);
}

int trace_blocks_per_cu(int kind, int precision, int wg, size_t smem)
{
    switch (kind) {
    case KIND_FWD: return fwd_blocks_per_cu<false, false>(precision, wg, smem);
    case KIND_FWD_ADJ: return fwd_blocks_per_cu<true, false>(precision, wg, smem);
    case KIND_FWD_TAB: return fwd_blocks_per_cu<false, true>(precision, wg, smem);
    case KIND_FWD_ADJ_TAB: return fwd_blocks_per_cu<true, true>(precision, wg, smem);
    case KIND_FWD_MEMO: return fwd_blocks_per_cu<false, false, true>(precision, wg, smem);
    case KIND_FWD_ADJ_MEMO: return fwd_blocks_per_cu<true, false, true>(precision, wg, smem);
    case KIND_BWD_REGEN: return bwd_blocks_per_cu<false>(precision, wg, smem);
    case KIND_BWD_REGEN_TAB: return bwd_blocks_per_cu<true>(precision, wg, smem);
    case KIND_ADJ_LOSSLESS:
        return blocks_per_cu(k_adj_entries<true>, wg, smem);
    case KIND_ADJ_MEMO:
        return blocks_per_cu(k_adj_memo<false>, 64 * kMemoWaves, smem);
    case KIND_ADJ_MEMO_LOSSLESS:
        return blocks_per_cu(k_adj_memo<true>, 64 * kMemoWaves, smem);
    case KIND_TABLE_ACCUM:
        return blocks_per_cu(k_table_accum, 64 * kMemoWaves, smem);
    case KIND_OMEGA:
        return blocks_per_cu(k_omega_grad, wg, smem);
    default:
        return blocks_per_cu(k_adj_entries<false>, wg, smem);
    }
}

template <int MODE>
static void launch_fwd_mode(const SceneDev& sc, dim3 grid, dim3 block, size_t sm, bool lds_bins, uint64_t* q,
                            uint32_t* c, unsigned long long* stats, gwg_ray_record* rec, int64_t rec_stride,
                            double* scratch, const AdjStore* adj, double* tape, hipStream_t s)
{
    const bool tab = sc.table != nullptr, memo = sc.memo != 0;
    if (adj && tab)
        hipLaunchKernelGGL((k_trace_fwd<MODE, true, true, false>), grid, block, sm, s, sc, q, c, stats, rec, rec_stride,
                           (int)lds_bins, scratch, *adj, tape);
    else if (adj && memo)
        hipLaunchKernelGGL((k_trace_fwd<MODE, true, false, true>), grid, block, sm, s, sc, q, c, stats, rec, rec_stride,
                           (int)lds_bins, scratch, *adj, tape);
    else if (adj)
        hipLaunchKernelGGL((k_trace_fwd<MODE, true, false, false>), grid, block, sm, s, sc, q, c, stats, rec, rec_stride,
                           (int)lds_bins, scratch, *adj, tape);
    else if (tab)
        hipLaunchKernelGGL((k_trace_fwd<MODE, false, true, false>), grid, block, sm, s, sc, q, c, stats, rec, rec_stride,
                           (int)lds_bins, scratch, AdjStore{}, (double*)nullptr);
    else if (memo)
        hipLaunchKernelGGL((k_trace_fwd<MODE, false, false, true>), grid, block, sm, s, sc, q, c, stats, rec, rec_stride,
                           (int)lds_bins, scratch, AdjStore{}, (double*)nullptr);
    else
        hipLaunchKernelGGL((k_trace_fwd<MODE, false, false, false>), grid, block, sm, s, sc, q, c, stats, rec, rec_stride,
                           (int)lds_bins, scratch, AdjStore{}, (double*)nullptr);
}

hipError_t launch_trace_fwd(const SceneDev& sc, int wg, int grid_blocks, bool lds_bins, uint64_t* q, uint32_t* c,
                            unsigned long long* stats, gwg_ray_record* rec, int64_t rec_stride, double* scratch,
                            const AdjStore* adj, double* tape, hipStream_t s)
{
    size_t sm = fwd_smem_bytes(sc, wg, lds_bins);
    dim3 grid((unsigned)grid_blocks), block(wg);
    switch (sc.precision) {
    case GWG_FP64:
        launch_fwd_mode<GWG_FP64>(sc, grid, block, sm, lds_bins, q, c, stats, rec, rec_stride, scratch, adj, tape, s);
        break;
    case GWG_FP32_MIXED:
        launch_fwd_mode<GWG_FP32_MIXED>(sc, grid, block, sm, lds_bins, q, c, stats, rec, rec_stride, scratch, adj, tape, s);
        break;
    default:
        launch_fwd_mode<GWG_FP32>(sc, grid, block, sm, lds_bins, q, c, stats, rec, rec_stride, scratch, adj, tape, s);
        break;
    }
    return hipGetLastError();
}

template <bool TAB>
static void launch_bwd_mode(const SceneDev& sc, dim3 grid, dim3 block, size_t sm, const double* dLdI, double* partial,
                            double* scratch, int64_t sample_stride, const int32_t* regen, unsigned long long* stats,
                            hipStream_t s)
{
    switch (sc.precision) {
    case GWG_FP64:
        hipLaunchKernelGGL((k_trace_bwd<GWG_FP64, TAB>), grid, block, sm, s, sc, dLdI, partial, scratch, sample_stride,
                           regen, stats);
        break;
    case GWG_FP32_MIXED:
        hipLaunchKernelGGL((k_trace_bwd<GWG_FP32_MIXED, TAB>), grid, block, sm, s, sc, dLdI, partial, scratch,
                           sample_stride, regen, stats);
        break;
    default:
        hipLaunchKernelGGL((k_trace_bwd<GWG_FP32, TAB>), grid, block, sm, s, sc, dLdI, partial, scratch, sample_stride,
                           regen, stats);
        break;
    }
}

hipError_t launch_trace_bwd(const SceneDev& sc, int wg, int grid_blocks, const double* dLdI, unsigned long long* stats,
                            double* partial, double* scratch, int64_t sample_stride, const int32_t* regen,
                            hipStream_t s)
{
    size_t sm = bwd_smem_bytes(sc, wg);
    dim3 grid((unsigned)grid_blocks), block(wg);
    if (sc.table)
        launch_bwd_mode<true>(sc, grid, block, sm, dLdI, partial, scratch, sample_stride, regen, stats, s);
    else
        launch_bwd_mode<false>(sc, grid, block, sm, dLdI, partial, scratch, sample_stride, regen, stats, s);
    return hipGetLastError();
}

hipError_t launch_adj_entries(const SceneDev& sc, int wg, int grid_blocks, const double* dLdI,
                              unsigned long long* stats, double* partial, const AdjStore& st, double* scratch,
                              hipStream_t s)
{
    size_t sm = bwd_smem_bytes(sc, wg);
    if (sc.slot_complex == 0u)
        hipLaunchKernelGGL(k_adj_entries<true>, dim3((unsigned)grid_blocks), dim3(wg), sm, s, sc, dLdI, partial, st,
                           scratch, stats);
    else
        hipLaunchKernelGGL(k_adj_entries<false>, dim3((unsigned)grid_blocks), dim3(wg), sm, s, sc, dLdI, partial, st,
                           scratch, stats);
    return hipGetLastError();
}

hipError_t launch_adj_memo(const SceneDev& sc, int grid_blocks, const double* dLdI, unsigned long long* stats,
                           double* partial, const AdjStore& st, double* scratch, hipStream_t s)
{
    const size_t sm = memo_smem_bytes(sc);
    if (sc.slot_complex == 0u)
        hipLaunchKernelGGL(k_adj_memo<true>, dim3((unsigned)grid_blocks), dim3(64 * kMemoWaves), sm, s, sc, dLdI, partial, st,
                           scratch, stats);
    else
        hipLaunchKernelGGL(k_adj_memo<false>, dim3((unsigned)grid_blocks), dim3(64 * kMemoWaves), sm, s, sc, dLdI, partial, st,
                           scratch, stats);
    return hipGetLastError();
}

hipError_t launch_table_build(const SceneDev& sc, double* tab, int n_cu, unsigned long long* stats, hipStream_t s)
{
    const int wg = 256;
    const int64_t dls = (int64_t)sc.D * sc.n_lsel;
    const int64_t per = (int64_t)sc.M * 2 * sc.table_n;
    // enough workgroups to fill the device twice, each with at least one wave of entries
    int64_t chunks = std::max<int64_t>(1, (2 * (int64_t)n_cu + dls - 1) / dls);
    chunks = std::min<int64_t>(chunks, (per + wg - 1) / wg);
    const size_t sm = (size_t)smem_layout(sc.M, sc.Lmax, sc.n_slots, wg, sc.bins_x * sc.bins_y, false, 0,
                                          LaneSlots3::kPer, true).total;
    const dim3 grid((unsigned)(dls * chunks)), block(wg);
    switch (sc.precision) {
    case GWG_FP64:
        hipLaunchKernelGGL(k_table_build<GWG_FP64>, grid, block, sm, s, sc, tab, (int)chunks, stats);
        break;
    case GWG_FP32_MIXED:
        hipLaunchKernelGGL(k_table_build<GWG_FP32_MIXED>, grid, block, sm, s, sc, tab, (int)chunks, stats);
        break;
    default:
        hipLaunchKernelGGL(k_table_build<GWG_FP32>, grid, block, sm, s, sc, tab, (int)chunks, stats);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_absmax(const double* x, int64_t n, unsigned long long* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_absmax, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
}

hipError_t launch_table_accum(const SceneDev& sc, int grid_blocks, const double* dLdI, const AdjStore& st, hipStream_t s)
{
    hipLaunchKernelGGL(k_table_accum, dim3((unsigned)grid_blocks), dim3(64 * kMemoWaves), table_accum_smem_bytes(), s, sc,
                       dLdI, st);
    return hipGetLastError();
}

hipError_t launch_table_adj(const SceneDev& sc, double* partial, double* scratch, unsigned long long* stats,
                            hipStream_t s)
{
    const dim3 grid((unsigned)(table_adj_blocks(sc))), block(128);
    const size_t sm = table_adj_smem_bytes(sc);
    if (sc.slot_complex == 0u)
        hipLaunchKernelGGL(k_table_adj<true>, grid, block, sm, s, sc, partial, scratch, stats);
    else
        hipLaunchKernelGGL(k_table_adj<false>, grid, block, sm, s, sc, partial, scratch, stats);
    return hipGetLastError();
}

hipError_t launch_table_reduce(const double* partial, const SceneDev& sc, double* grad, hipStream_t s)
{
    const int64_t n = (int64_t)sc.D * sc.M * sc.Lmax;
    hipLaunchKernelGGL(k_table_reduce, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, s, partial, sc.D, sc.n_lsel, sc.M,
                       sc.Lmax, sc.nlay, grad);
    return hipGetLastError();
}

hipError_t launch_omega_grad(const SceneDev& sc, int grid_blocks, int wg, const double* W, const uint32_t* counts,
                             double* partial, double* grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_omega_grad, dim3((unsigned)grid_blocks), dim3(wg), omega_smem_bytes(sc, wg), s, sc, W, counts,
                       partial);
    hipLaunchKernelGGL(k_omega_reduce, dim3(1), dim3(64), 0, s, (const double*)partial, sc.n_items, sc.M, grad);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double* partial, int64_t items_per_design, int ML, int D, double* tmp,
                              double* grad, const int32_t* nlay, int M, int Lmax, hipStream_t s)
{
    int64_t n = (int64_t)D * ML;
    hipLaunchKernelGGL(k_grad_ranges, dim3((unsigned)((ML + 255) / 256), kGradRanges, (unsigned)D), dim3(256), 0, s,
                       partial, items_per_design, ML, tmp);
    hipLaunchKernelGGL(k_grad_reduce, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, s, (const double*)tmp, ML, D, grad);
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
    return (size_t)(sizeof(LayerRec) * rec_stride(L) + 8 * n_slots * LaneSlots5::kPer * ((wg + 63) / 64 * 64));
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
    hipLaunchKernelGGL(k_loss_eyeb, dim3((unsigned)((int64_t)D * ((B + 63) / 64))), dim3(1024), 0, s, I, D, nl * F, B, E);
    hipLaunchKernelGGL(k_loss_scalar, dim3((unsigned)D), dim3(256), 0, s, eta, E, nl, F, B, kind, w_f, w_e, phi, coef);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, s, (const double*)coef, D, loss);
    if (G) hipLaunchKernelGGL(k_loss_grad, dim3(grid_for((int64_t)D * nl * F * B, 256)), dim3(256), 0, s, E, phi, coef, D, nl, F, B, G);
    return hipGetLastError();
}

// ------------------------------------------ allocation-free loss scratch
// Work buffer of gwg_loss_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  On the host
// the array's name is not a device address: its address on each device is
// looked up once, with that device current, by hipGetSymbolAddress, and only
// that pointer is ever passed to kernels.
static __device__ __align__(256) double scratch[kLossScratchDoubles];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

hipError_t loss_scratch_setup(int device)
{
    if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = (double*)p;
    return hipSuccess;
}

double* loss_scratch(int device)
{
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace gwg
