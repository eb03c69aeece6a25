// Adjoint trace kernel.  Included by gwg_kernels.hip inside namespace gwg.
//
// Gradient checkpointing between the tracer and the thin-film solver
// (Methods, memory-saving strategies): the path part and the thin-film part
// of the adjoint run in two phases within each wave.
//
// Phase 1, per ray (one ray per lane per round): pass A regenerates the
// sampled path (same Philox words, same geometry, same coefficients) and
// writes a tape of its field-changing events; if the ray lands in a bin with
// nonzero dL/dI, pass B walks the tape backwards carrying the adjoint field
// lambda (lambda_K = E_K, lambda_{k-1} = A_k^H lambda_k) and, at every mirror
// hit, pushes the hit's kappa, mirror, side, branch and the holomorphic
// cotangents of its two coefficients
//     G_s = scale conj(lambda_k . s) (s . E_{k-1}),
//     G_p = scale conj(lambda_k . p_out) (p_in . E_{k-1})
// (times dL/dI / N) onto the wave's ring queue.  Positions come from a wave
// prefix sum over lanes, so the queue order is a fixed function of the ray
// order.
//
// Phase 2, whenever 64 entries are queued (and once more at the end of a work
// item): every lane takes one entry and runs the adjoint thin-film solve,
// adding dw/dt_j into the wave's private LDS row of that mirror.  All lanes
// run the same layer loop, independent of how long their rays were.
//
// Work items are assigned to persistent workgroups with a fixed stride, each
// wave owns its LDS accumulator, and the per-item partials are summed in item
// order afterwards, so the gradient is bit-identical from run to run.

constexpr int kQFields = 6;      // kappa, Gs.re, Gs.im, Gp.re, Gp.im, meta

struct Queue {
    double* base;      // this wave's queue, field f of slot p at base[f * cap + p]
    int cap;
};

__device__ inline void q_put(const Queue& q, int pos, double kappa, cd Gs, cd Gp, int meta)
{
    int p = pos % q.cap;
    q.base[0 * q.cap + p] = kappa;
    q.base[1 * q.cap + p] = Gs.re;
    q.base[2 * q.cap + p] = Gs.im;
    q.base[3 * q.cap + p] = Gp.re;
    q.base[4 * q.cap + p] = Gp.im;
    q.base[5 * q.cap + p] = (double)meta;
}

// Adjoint thin-film solve of queue entry `pos` (one per lane).
__device__ inline void adjoint_entry(const SceneDev& sc, const PointLds& pl, const double* s_thk,
                                     const uint8_t* s_slot, double* sp, int ls, double* gw, const Queue& q,
                                     int pos, double* chk, int64_t cstride)
{
    int p = pos % q.cap;
    double kappa = q.base[p];
    cd Gs = mk(q.base[1 * q.cap + p], q.base[2 * q.cap + p]);
    cd Gp = mk(q.base[3 * q.cap + p], q.base[4 * q.cap + p]);
    int meta = (int)q.base[5 * q.cap + p];
    int m = meta & 255;
    bool front = (meta >> 8) & 1, refl = (meta >> 9) & 1;
    for (int s = 0; s < sc.n_slots; ++s) {
        double P[NPF];
        slot_params(pl.slotN[2 * s], pl.slotN[2 * s + 1], kappa, pl.k0, P);
#pragma unroll
        for (int k = 0; k < NPF; ++k) sp[(s * NPF + k) * ls] = P[k];
    }
    double z0 = pl.ng * pl.ng - kappa * kappa;
    double q0 = sqrt(z0 > kTinyZ ? z0 : kTinyZ);
    tmm_adjoint(s_thk + m * sc.Lmax, s_slot + m * sc.Lmax, pl.nlay[m], front, sp, ls, sc.slot_complex,
                pl.k0, kappa * kappa, pl.nsq, q0, pl.ng * pl.ng / q0, refl, Gs, Gp, gw + m * sc.Lmax, chk,
                cstride);
}

template <int MODE>
__global__ void __launch_bounds__(128, 2) k_trace_bwd(SceneDev sc, const double* __restrict__ dLdI,
                                                   double* __restrict__ partial,
                                                   double* __restrict__ scratch, int64_t sample_stride,
                                                   unsigned long long* __restrict__ stats)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int WG = blockDim.x;
    const int n_waves = (WG + 63) / 64;
    const int B = sc.bins_x * sc.bins_y;
    const SmemLayout lay = smem_layout(sc.M, sc.Lmax, sc.n_slots, WG, B, false, n_waves);
    PointLds* pl = (PointLds*)(smem + lay.off_pl);
    double* s_thk = (double*)(smem + lay.off_thk);
    uint8_t* s_slot = (uint8_t*)(smem + lay.off_slot);
    double* s_sp = (double*)(smem + lay.off_sp);
    double* s_grad = (double*)(smem + lay.off_grad);
    unsigned long long* s_st = (unsigned long long*)(smem + lay.off_st);
    const int tid = threadIdx.x;
    const int wave = tid / 64;
    const int lane = wave_lane();
    const int ML = sc.M * sc.Lmax;
    double* gw = s_grad + (int64_t)wave * ML;
    double* sp = s_sp + tid;
    const int64_t nthreads = (int64_t)gridDim.x * WG;
    const int64_t gtid = (int64_t)blockIdx.x * WG + tid;
    const int64_t gwave = (int64_t)blockIdx.x * n_waves + wave;
    // scratch: [tape Kmax x 15][checkpoints n_chk x 8] per lane, then queues per wave
    TapeRef tape = { scratch + gtid, nthreads };
    const int64_t n_chk = sc.Lmax / kSeg + 1;
    double* chk = scratch + (int64_t)sc.Kmax * kTapeStride * nthreads + gtid;
    const int qcap = 64 * (sc.Kmax + 1);
    const int64_t n_waves_total = (int64_t)gridDim.x * n_waves;
    double* qbase = scratch + ((int64_t)sc.Kmax * kTapeStride + n_chk * 8) * nthreads;
    Queue q = { qbase + gwave * (int64_t)kQFields * qcap, qcap };
    const int hcap = 64 * sc.Kmax;
    const HitQueue hq = { qbase + n_waves_total * (int64_t)kQFields * qcap + gwave * (int64_t)kHitFields * hcap, hcap };
    for (int k = tid; k < ST_WORDS; k += WG) s_st[k] = 0ull;
    unsigned long long c_rays = 0, c_ev = 0, c_hits = 0, c_lay = 0, c_fp64 = 0;
    unsigned long long c_arays = 0, c_ahits = 0, c_alay = 0;

    for (int64_t item = blockIdx.x; item < sc.n_items; item += gridDim.x) {
        int64_t point, i0, i1;
        int d, l, f;
        decode_item(sc, item, &point, &d, &l, &f, &i0, &i1);
        __syncthreads();
        stage_point(sc, d, l, f, pl, s_thk, s_slot);
        for (int k = tid; k < n_waves * ML; k += WG) s_grad[k] = 0.0;
        __syncthreads();
        const int64_t base = point * sc.N;
        const double* g_bins = dLdI + point * B;
        int qhead = 0, qcount = 0;            // wave-uniform
        for (int64_t round = 0;; ++round) {
            const int64_t wave_first = i0 + (int64_t)wave * 64 + round * WG;
            if (wave_first >= i1) break;      // uniform across the wave
            const int64_t i = wave_first + lane;
            const int64_t id = base + i;
            bool active = i < i1 && (sample_stride <= 1 || (id % sample_stride) == 0);
            Ray r;
            Outcome o;
            o.cat = CAT_LOST;
            o.bin = -1;
            int nt = 0;
            TapeRef none = { nullptr, 0 };
            int nh = 0;
            if (active) {
                ray_birth(sc, *pl, id, r);
                walk_ray<false, false>(sc, *pl, r, o, NoHit{}, NoCoef{}, none, nullptr);
                nh = r.nprma;
            }
            int htotal;
            const int hoff = wave_excl_scan(nh, &htotal);
            if (active) {
                ray_birth(sc, *pl, id, r);
                walk_ray<false, false>(sc, *pl, r, o, PutHit{ hq, hoff }, NoCoef{}, none, nullptr);
            }
            __threadfence_block();
            solve_hits<MODE>(sc, *pl, s_thk, s_slot, sp, WG, hq, htotal, &c_fp64, &c_lay);
            __threadfence_block();
            if (active) {
                ray_birth(sc, *pl, id, r);
                walk_ray<true, true>(sc, *pl, r, o, NoHit{}, GetCoef{ hq, hoff }, tape, &nt);
                c_rays += 1;
                c_ev += (unsigned long long)r.nev;
                c_hits += (unsigned long long)r.nprma;
            }
            double gscale = 0.0;
            if (active && o.cat == CAT_EYEBOX) gscale = g_bins[o.bin] / (double)sc.N;
            const bool contrib = gscale != 0.0;
            int total;
            const int off = wave_excl_scan(contrib ? r.nprma : 0, &total);
            if (contrib) {
                c_arays += 1;
                int slotpos = qhead + qcount + off;
                cd lam[3] = { r.e[0], r.e[1], r.e[2] };
                for (int k = nt - 1; k >= 0; --k) {
                    const double* b = tape.base + (int64_t)k * kTapeStride * tape.ts;
                    const int64_t ts = tape.ts;
                    double dx = b[0], dy = b[ts], dz = b[2 * ts];
                    cd cs = mk(b[9 * ts], b[10 * ts]), cp = mk(b[11 * ts], b[12 * ts]);
                    double scale = b[13 * ts];
                    int meta = (int)b[14 * ts];
                    int type = meta & 15, m = (meta >> 4) & 255;
                    int front = (meta >> 12) & 1, refl = (meta >> 13) & 1;
                    double sv[3], pin[3], pout[3];
                    if (type == EV_MIRROR) {
                        s_basis(dx, dy, dz, sc.nx, 0.0, sc.nz, sv);
                        cross3(dx, dy, dz, sv[0], sv[1], sv[2], pin);
                        double ndx = dx, ndz = dz;
                        if (refl) mirror_reflect(sc.nx, sc.nz, dx, dz, &ndx, &ndz);
                        cross3(ndx, dy, ndz, sv[0], sv[1], sv[2], pout);
                        cd E[3];
                        for (int c = 0; c < 3; ++c) E[c] = mk(b[(3 + 2 * c) * ts], b[(4 + 2 * c) * ts]);
                        cd ls = cadd(cadd(cscale(lam[0], sv[0]), cscale(lam[1], sv[1])), cscale(lam[2], sv[2]));
                        cd lp = cadd(cadd(cscale(lam[0], pout[0]), cscale(lam[1], pout[1])), cscale(lam[2], pout[2]));
                        cd es = cadd(cadd(cscale(E[0], sv[0]), cscale(E[1], sv[1])), cscale(E[2], sv[2]));
                        cd ep = cadd(cadd(cscale(E[0], pin[0]), cscale(E[1], pin[1])), cscale(E[2], pin[2]));
                        cd Gs = cscale(cmul(cconj(ls), es), scale * gscale);
                        cd Gp = cscale(cmul(cconj(lp), ep), scale * gscale);
                        double c3[3];
                        cross3(dx, dy, dz, sc.nx, 0.0, sc.nz, c3);
                        double kappa = pl->ng * sqrt(c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
                        q_put(q, slotpos++, kappa, Gs, Gp, m | (front << 8) | (refl << 9));
                    } else {
                        s_basis(dx, dy, dz, 0.0, 0.0, 1.0, sv);
                        cross3(dx, dy, dz, sv[0], sv[1], sv[2], pin);
                        if (type == EV_TIR) {
                            cross3(dx, dy, -dz, sv[0], sv[1], sv[2], pout);
                        } else {
                            Ray tmp;
                            tmp.dx = dx; tmp.dy = dy; tmp.dz = dz;
                            double st2 = (pl->ng * pl->ng) * (dx * dx + dy * dy);
                            double a[3];
                            exit_direction(pl->ng, pl->na, tmp, st2, a);
                            cross3(a[0], a[1], a[2], sv[0], sv[1], sv[2], pout);
                        }
                    }
                    // lambda <- A^H lambda,  A = scale (cs s s^T + cp p_out p_in^T)
                    cd ls = cadd(cadd(cscale(lam[0], sv[0]), cscale(lam[1], sv[1])), cscale(lam[2], sv[2]));
                    cd lp = cadd(cadd(cscale(lam[0], pout[0]), cscale(lam[1], pout[1])), cscale(lam[2], pout[2]));
                    cd as = cscale(cmul(cconj(cs), ls), scale), ap = cscale(cmul(cconj(cp), lp), scale);
                    for (int c = 0; c < 3; ++c) lam[c] = cadd(cscale(as, sv[c]), cscale(ap, pin[c]));
                }
            }
            qcount += total;
            __threadfence_block();
            // phase 2: drain full batches
            while (qcount >= 64) {
                adjoint_entry(sc, *pl, s_thk, s_slot, sp, WG, gw, q, qhead + lane, chk, nthreads);
                const int m = ((int)q.base[5 * q.cap + (qhead + lane) % q.cap]) & 255;
                c_ahits += 1;
                c_alay += (unsigned long long)pl->nlay[m];
                qhead = (qhead + 64) % q.cap;
                qcount -= 64;
            }
        }
        if (qcount > 0) {
            if (lane < qcount) {
                adjoint_entry(sc, *pl, s_thk, s_slot, sp, WG, gw, q, qhead + lane, chk, nthreads);
                const int m = ((int)q.base[5 * q.cap + (qhead + lane) % q.cap]) & 255;
                c_ahits += 1;
                c_alay += (unsigned long long)pl->nlay[m];
            }
            qcount = 0;
        }
        __syncthreads();
        double* out = partial + item * (int64_t)ML;
        for (int k = tid; k < ML; k += WG) {
            double acc = 0.0;
            for (int w = 0; w < n_waves; ++w) acc += s_grad[(int64_t)w * ML + k];
            out[k] = acc;
        }
    }
    const unsigned long long cnt[9] = { c_rays, c_ev, c_hits, c_fp64, 0ull, c_lay, c_arays, c_ahits, c_alay };
    for (int k = 0; k < 9; ++k)
        if (cnt[k]) atomicAdd(&s_st[k], cnt[k]);
    __syncthreads();
    for (int k = tid; k < 9; k += WG)
        if (s_st[k]) atomicAdd(&stats[k], s_st[k]);
}

int64_t bwd_scratch_doubles(const SceneDev& sc, int64_t grid_blocks, int wg)
{
    const int64_t nthreads = grid_blocks * wg;
    const int64_t n_chk = sc.Lmax / kSeg + 1;
    const int64_t n_waves = grid_blocks * ((wg + 63) / 64);
    return ((int64_t)sc.Kmax * kTapeStride + n_chk * 8) * nthreads
           + n_waves * ((int64_t)kQFields * 64 * (sc.Kmax + 1) + (int64_t)kHitFields * 64 * sc.Kmax);
}
