// Adjoint trace kernels.  Included by gwg_kernels.hip inside namespace gwg.
//
// Gradient checkpointing between the tracer and the thin-film solver
// (Methods, memory-saving strategies): the path part and the thin-film part
// of the adjoint run separately.
//
// Path part.  For every ray ending in an eyebox bin, the reverse field sweep
// (reverse_sweep) gives each of its mirror hits the holomorphic cotangents
// G_s, G_p of the two coefficients the ray took.  When the forward trace was
// asked to prepare a gradient it ran this sweep itself and stored one entry
// per hit (AdjStore); otherwise, or for work items whose entry regions
// overflowed, k_trace_bwd regenerates the paths: a geometry-only walk finds
// each ray's bin and queues its hits, the hits of rays in a bin with nonzero
// dL/dI are solved, those rays are walked again with the field and a tape of
// their field-changing events, and the sweep runs on the tape.
//
// Thin-film part.  Entries are drained 64 at a time, one per lane, so every
// lane runs the same layer loop whatever the length of its ray: the adjoint
// thin-film solve of the hit adds (dL/dI[bin] / N) d(2 Re(G_s c_s + G_p c_p))/dt_j
// into the wave's private LDS row of that mirror.
//
// Work items go to persistent workgroups with a fixed stride, each wave owns
// its LDS accumulator, and the per-item partials are summed in item order
// afterwards, so the gradient is bit-identical from run to run.

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

// Adjoint thin-film solve of one mirror hit (one per lane): kappa, the
// scaled cotangents and meta = mirror | front << 8 | reflected << 9.
// LOSSLESS: the scene has no absorbing slot (compiled without the general path).
// stored: chk is the entry's checkpoint block written by the forward solve
// (lossless stacks; the sweep is not run again).
template <bool LOSSLESS = false>
__device__ inline void adjoint_hit(const SceneDev& sc, const PointLds& pl, const double* s_thk,
                                   const uint8_t* s_slot, const LaneSlots3& sl, double* gw, double kappa, cd Gs,
                                   cd Gp, int meta, double* chk, int64_t cstride, bool stored = false)
{
    const int m = meta & 255;
    const bool front = (meta >> 8) & 1, refl = (meta >> 9) & 1;
    bool hyp = false;                       // an evanescent lossless slot at this kappa
    for (int s = 0; s < sc.n_slots; ++s) {
        double P[NPF];
        slot_params(pl.slotN[2 * s], pl.slotN[2 * s + 1], kappa, pl.k0, P);
        sl.put(s, P);
        hyp |= !((sc.slot_complex >> s) & 1u) && P[0] < 0.0;
    }
    const double z0 = pl.ng * pl.ng - kappa * kappa;
    const double q0 = sqrt(z0 > kTinyZ ? z0 : kTinyZ);
    if (LOSSLESS || sc.slot_complex == 0u) {
        // waves whose lanes all see circular layers take the sweep without
        // the hyperbolic case (same results).  A sweep the forward stored
        // has its hit's checkpoint interval; a sweep run here takes one
        // interval for the whole wave (lanes of one interval walk their
        // segments together), the longer one only if no lane meets an
        // evanescent layer.
        const bool circ = __ballot(hyp) == 0ull;
        const int kseg = stored ? ck_interval(hyp) : ck_interval(!circ);
        if (circ)
            tmm_adjoint_lossless<false>(s_thk + m * sc.Lmax, s_slot + m * sc.Lmax, pl.nlay[m], front, sl, pl.k0, q0,
                                        pl.ng * pl.ng / q0, refl, Gs, Gp, gw + m * sc.Lmax, chk, cstride, stored,
                                        kseg);
        else
            tmm_adjoint_lossless<true>(s_thk + m * sc.Lmax, s_slot + m * sc.Lmax, pl.nlay[m], front, sl, pl.k0, q0,
                                       pl.ng * pl.ng / q0, refl, Gs, Gp, gw + m * sc.Lmax, chk, cstride, stored,
                                       kseg);
    }
    else if (!LOSSLESS)
        tmm_adjoint(s_thk + m * sc.Lmax, s_slot + m * sc.Lmax, pl.nlay[m], front, sl, sc.slot_complex,
                    pl.k0, kappa * kappa, q0, pl.ng * pl.ng / q0, refl, Gs, Gp, gw + m * sc.Lmax, chk,
                    cstride);
}

// Adjoint thin-film solve of ring-queue entry `pos`.
__device__ inline void adjoint_entry(const SceneDev& sc, const PointLds& pl, const double* s_thk,
                                     const uint8_t* s_slot, const LaneSlots3& sl, double* gw, const Queue& q,
                                     int pos, double* chk, int64_t cstride)
{
    const int p = pos % q.cap;
    adjoint_hit(sc, pl, s_thk, s_slot, sl, gw, q.base[p], mk(q.base[1 * q.cap + p], q.base[2 * q.cap + p]),
                mk(q.base[3 * q.cap + p], q.base[4 * q.cap + p]), (int)q.base[5 * q.cap + p], chk, cstride);
}

// Pushes the entries of one ray onto the ring queue with the dL/dI factor applied.
struct QueueEmit {
    Queue q;
    int* pos;
    double gscale;
    __device__ void operator()(double kappa, cd Gs, cd Gp, int meta) const
    {
        q_put(q, (*pos)++, kappa, cscale(Gs, gscale), cscale(Gp, gscale), meta);
    }
};

template <int MODE, bool TAB>
__global__ void __launch_bounds__(128, 2) k_trace_bwd(SceneDev sc, const double* __restrict__ dLdI,
                                                   double* __restrict__ partial,
                                                   double* __restrict__ scratch, int64_t sample_stride,
                                                   const int32_t* __restrict__ regen,
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
    const LaneSlots3 sl = { slot_lane_base(s_sp, sc.n_slots, LaneSlots3::kPer, tid), pl->nsq, pl->pxy };
    const int64_t nthreads = (int64_t)gridDim.x * WG;
    const int64_t gtid = (int64_t)blockIdx.x * WG + tid;
    const int64_t gwave = (int64_t)blockIdx.x * n_waves + wave;
    // scratch: the tape (Kmax event slots of every lane), then n_chk x 8
    // checkpoint doubles per lane, then queues per wave
    const TapeRef tape = tape_lane(scratch, sc.Kmax, (int64_t)gridDim.x * n_waves, gwave, lane);
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
    // angle table: coefficients are interpolated and the sweep's cotangents go
    // to the table accumulators instead of the thin-film adjoint
    constexpr bool tabm = TAB;
    const double fx = tabm ? table_fx_scale(sc) : 0.0;

    for (int64_t item = draw_item(stats + ST_NEXT1); item < sc.n_items; item = draw_item(stats + ST_NEXT1)) {
        // regen (optional): only items whose stored entries overflowed
        if (regen && regen[item] == 0) continue;
        int64_t point, i0, i1;
        int d, l, f;
        decode_item(sc, item, &point, &d, &l, &f, &i0, &i1);
        stage_point(sc, d, l, f, pl, s_thk, s_slot);
        for (int k = tid; k < n_waves * ML; k += WG) s_grad[k] = 0.0;
        __syncthreads();
        const int64_t base = point * sc.N;
        const double* g_bins = dLdI + point * B;
        const int64_t dl = (int64_t)d * sc.n_lsel + l;
        const double* tab_dl = tabm ? sc.table + dl * sc.M * 2 * sc.table_n * 8 : nullptr;
        long long* acc_dl = tabm ? sc.tab_acc + dl * sc.M * 4 * sc.table_n * 4 : nullptr;
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
            TapeRef none = { nullptr, nullptr, 0 };
            int nh = 0;
            double gscale = 0.0;
            const int own = lane;                // this lane's column of the hit queue
            if (active) {
                ray_birth(sc, *pl, id, r);
                if constexpr (TAB)
                    walk_ray<false, false>(sc, *pl, r, o, NoHit{}, NoCoef{}, none, nullptr);
                else
                    walk_ray<false, false>(sc, *pl, r, o, PutHit{ hq, own }, NoCoef{}, none, nullptr);
                // the bin is fixed by geometry alone: rays that end outside the
                // eyebox or in a bin with dL/dI = 0 carry no gradient and are
                // not regenerated further
                if (o.cat == CAT_EYEBOX) gscale = g_bins[o.bin] / (double)sc.N;
                active = gscale != 0.0;
                nh = active ? r.nprma : 0;
            }
            if (!tabm) {
                int htotal;
                const int hoff = wave_excl_scan(nh, &htotal);
                __threadfence_block();
                solve_hits<MODE>(sc, *pl, ArrStacks{ s_thk, s_slot, sc.Lmax, LaneSlots3::kPer * kSlotLanes * 8 }, sl,
                                 hq, htotal, hoff, &c_fp64, &c_lay);
                __threadfence_block();
            }
            if (active) {
                ray_birth(sc, *pl, id, r);
                if constexpr (TAB)
                    walk_ray<true, true>(sc, *pl, r, o, NoHit{}, TabCoef{ tab_dl, sc.table_n, pl->ng, sc.nx, sc.nz }, tape, &nt);
                else
                    walk_ray<true, true>(sc, *pl, r, o, NoHit{}, GetCoef{ hq, own, nullptr }, tape, &nt);
                c_rays += 1;
                c_ev += (unsigned long long)r.nev;
                c_hits += (unsigned long long)r.nprma;
            }
            const bool contrib = active;
            const int ntw = wave_max_int(contrib ? nt : 0);
            if constexpr (TAB) {
                if (contrib) {
                    c_arays += 1;
                    reverse_sweep(sc, *pl, r.e, tape, nt, ntw, TableEmit{ acc_dl, sc.table_n, pl->ng, gscale, fx });
                }
                continue;
            }
            int total;
            const int off = wave_excl_scan(contrib ? r.nprma : 0, &total);
            if (contrib) {
                c_arays += 1;
                int slotpos = qhead + qcount + off;
                reverse_sweep(sc, *pl, r.e, tape, nt, ntw, QueueEmit{ q, &slotpos, gscale });
            }
            qcount += total;
            __threadfence_block();
            // phase 2: drain full batches
            while (qcount >= 64) {
                adjoint_entry(sc, *pl, s_thk, s_slot, sl, gw, q, qhead + lane, chk, nthreads);
                const int m = ((int)q.base[5 * q.cap + (qhead + lane) % q.cap]) & 255;
                c_ahits += 1;
                c_alay += (unsigned long long)pl->nlay[m];
                qhead = (qhead + 64) % q.cap;
                qcount -= 64;
            }
        }
        if (qcount > 0) {
            if (lane < qcount) {
                adjoint_entry(sc, *pl, s_thk, s_slot, sl, gw, q, qhead + lane, chk, nthreads);
                const int m = ((int)q.base[5 * q.cap + (qhead + lane) % q.cap]) & 255;
                c_ahits += 1;
                c_alay += (unsigned long long)pl->nlay[m];
            }
            qcount = 0;
        }
        __syncthreads();
        if constexpr (TAB) continue;
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

// One kind's queue of entry indices in a wave: n (wave-uniform) entries at
// positions 0..n-1, position p in lane p of lo (p < 64) or of hi (p >= 64).
struct KindQueue {
    int lo = -1, hi = -1, n = 0;
    // file lane's entry c if `mine` (all lanes call; entries keep lane order)
    __device__ void add(bool mine, int c, int lane)
    {
        const unsigned long long m = __ballot(mine);
        const int below = __popcll(m & ((1ull << lane) - 1ull));
        const int cnt = __popcll(m);
        // a permutation of the lanes: the entries go to lanes (n + rank) mod
        // 64, the other lanes' pushes fill the remaining lanes (unread)
        const int dst = mine ? ((n + below) & 63) : ((n + cnt + (lane - below)) & 63);
        const int got = __builtin_amdgcn_ds_permute(dst << 2, c);
        if (lane >= n && lane < n + cnt) lo = got;               // positions n .. 63
        if (lane + 64 < n + cnt) hi = got;                       // positions 64 .. n + cnt - 1
        n += cnt;
    }
    // the first min(n, 64) entries, one per lane (-1 past n)
    __device__ int take()
    {
        const int lane = (int)(threadIdx.x & 63);
        const int v = lane < n ? lo : -1;
        lo = hi;
        hi = -1;
        n = n > 64 ? n - 64 : 0;
        return v;
    }
};

// Thin-film part of the adjoint over the entries stored by the forward trace.
// Items whose regions overflowed are left to k_trace_bwd.  LOSSLESS: the
// scene has no absorbing slot.
template <bool LOSSLESS>
__global__ void __launch_bounds__(128, 2) k_adj_entries(SceneDev sc, const double* __restrict__ dLdI,
                                                     double* __restrict__ partial, AdjStore st,
                                                     double* __restrict__ scratch,
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
    const LaneSlots3 sl = { slot_lane_base(s_sp, sc.n_slots, LaneSlots3::kPer, tid), pl->nsq, pl->pxy };
    const int64_t nthreads = (int64_t)gridDim.x * WG;
    double* chk = scratch + (int64_t)blockIdx.x * WG + tid;
    for (int k = tid; k < ST_WORDS; k += WG) s_st[k] = 0ull;
    unsigned long long c_ahits = 0, c_alay = 0, c_astored = 0;

    for (int64_t it = draw_item(stats + ST_NEXT0); it < sc.n_items; it = draw_item(stats + ST_NEXT0)) {
        const int64_t item = st.order ? (int64_t)st.order[it] : it;
        if (st.ovf[item] != 0) continue;
        int64_t point, i0, i1;
        int d, l, f;
        decode_item(sc, item, &point, &d, &l, &f, &i0, &i1);
        stage_point(sc, d, l, f, pl, s_thk, s_slot);
        for (int k = tid; k < n_waves * ML; k += WG) s_grad[k] = 0.0;
        __syncthreads();
        const double* g_bins = dLdI + point * B;
        const int32_t* cnt = st.cnt + item * st.waves;
        int total = 0;
        for (int w = 0; w < st.waves; ++w) total += cnt[w];
        // Batches of one kind: the wave scans its chunks of 64 entries (item
        // order) and files each entry under its kind, an entry whose kappa
        // may meet an evanescent layer or one that cannot; a batch of 64 is
        // taken from a kind's queue as soon as it holds that many, the rest
        // at the end.  Most batches then take the sweeps without the
        // hyperbolic case, and a batch's entries stay close together in item
        // order (their stored sweeps share lines).  Each kind's queue is two
        // registers per lane, positions 0-63 and 64-127; entries reach their
        // positions by a lane permutation.
        KindQueue qc, qh;
        int chunk = wave;
        for (;;) {
            int v = -1;
            for (;;) {                                    // wave-uniform: the next batch
                if (qc.n >= 64) { v = qc.take(); break; }
                if (qh.n >= 64) { v = qh.take(); break; }
                if (chunk * 64 >= total) {
                    if (qc.n > 0) { v = qc.take(); break; }
                    if (qh.n > 0) { v = qh.take(); break; }
                    break;
                }
                const int c = chunk * 64 + lane;
                bool ev = false;
                if (c < total) {
                    int rr = 0, k = c;
                    while (k >= cnt[rr]) { k -= cnt[rr]; ++rr; }
                    const double kap = st.ent[(item * st.waves + rr) * st.cap_w + k];
                    ev = kap * kap > pl->kap2_evan;
                }
                qc.add(c < total && !ev, c, lane);
                qh.add(c < total && ev, c, lane);
                chunk += n_waves;
            }
            if (__ballot(v >= 0) == 0ull) break;
            if (v >= 0) {
                int rr = 0, k = v;
                while (k >= cnt[rr]) { k -= cnt[rr]; ++rr; }
                const int64_t e = (item * st.waves + rr) * st.cap_w + k;
                const double kappa = st.ent[e];
                const int64_t meta = (int64_t)st.ent[5 * st.total + e];
                const int bin = (int)(meta >> 10);
                const double gscale = g_bins[bin] / (double)sc.N;
                if (gscale != 0.0) {
                    const cd Gs = cscale(mk(st.ent[1 * st.total + e], st.ent[2 * st.total + e]), gscale);
                    const cd Gp = cscale(mk(st.ent[3 * st.total + e], st.ent[4 * st.total + e]), gscale);
                    const int mm = (int)(meta & 1023);
                    // the forward stored this entry's sweep (lossless FP64 stacks)
                    const bool stored = LOSSLESS && st.ck && k < st.ck_cap;
                    double* c = stored ? st.ck + ((item * st.waves + rr) * st.ck_cap + k) * 8 : chk;
                    adjoint_hit<LOSSLESS>(sc, *pl, s_thk, s_slot, sl, gw, kappa, Gs, Gp, mm, c,
                                          stored ? 8 * st.ck_total : nthreads, stored);
                    c_ahits += 1;
                    c_alay += (unsigned long long)pl->nlay[mm & 255];
                    if (stored) c_astored += (unsigned long long)pl->nlay[mm & 255];
                }
            }
        }
        __syncthreads();
        double* out = partial + item * (int64_t)ML;
        for (int k = tid; k < ML; k += WG) {
            double acc = 0.0;
            for (int w = 0; w < n_waves; ++w) acc += s_grad[(int64_t)w * ML + k];
            out[k] = acc;
        }
    }
    if (c_ahits) atomicAdd(&s_st[ST_ADJ_HITS], c_ahits);
    if (c_alay) atomicAdd(&s_st[ST_ADJ_LAYERS], c_alay);
    if (c_astored) atomicAdd(&s_st[ST_ADJ_STORED], c_astored);
    __syncthreads();
    for (int k = tid; k < ST_WORDS; k += WG)
        if (s_st[k]) atomicAdd(&stats[k], s_st[k]);
}

int64_t adj_scratch_doubles(const SceneDev& sc, int64_t grid_blocks, int wg)
{
    return (sc.Lmax / kSeg + 1) * 8 * grid_blocks * wg;
}

int64_t bwd_scratch_doubles(const SceneDev& sc, int64_t grid_blocks, int wg)
{
    const int64_t nthreads = grid_blocks * wg;
    const int64_t n_chk = sc.Lmax / kSeg + 1;
    const int64_t n_waves = grid_blocks * ((wg + 63) / 64);
    return ((int64_t)sc.Kmax * kTapeStride + n_chk * 8) * nthreads
           + n_waves * ((int64_t)kQFields * 64 * (sc.Kmax + 1) + (int64_t)kHitFields * 64 * sc.Kmax);
}
