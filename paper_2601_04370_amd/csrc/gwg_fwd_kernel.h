// Forward trace kernel.  Included by gwg_kernels.hip inside namespace gwg.
//
// Two-pass intersection (Methods, memory-saving strategies): the path of a
// ray (surfaces, branch decisions) does not depend on the coatings, so each
// wave processes its rays in rounds of one ray per lane:
//   1. a geometry-only walk writes each hit's kappa, mirror and side to the
//      ray's lane's slots of the wave's hit queue and finds the ray's fate;
//   2. a wave prefix sum of the hit counts orders the wave's hits densely,
//      and they are solved in batches of 64, one per lane, so every lane of
//      the wave runs the same layer loop whatever the path lengths;
//   3. a second walk replays the path with the polarization field, taking
//      the coefficients from the ray's own slots, and scatters into the
//      eyebox bins;
//   4. with ADJ (a gradient will follow), the second walk also writes a tape
//      of the field-changing events and every ray that reached the eyebox
//      runs the reverse field sweep, storing one adjoint entry per mirror hit
//      (AdjStore) for the backward.
// Walks are cheap next to the thin-film solves (a few hundred operations per
// event against tens of thousands per hit).
//
// Memoized solves (GWG_FWD_MEMO, collimated beams): a hit's coefficients
// depend only on its kappa, mirror and side, and within one work item the
// rays share a handful of such keys (kappa comes from direction bits that
// every ray with the same event history shares exactly).  Each wave then
// keeps a table of the item's keys with their coefficients: step 2 resolves
// every queued hit to its key, solves only keys not seen before in the item,
// and step 3 reads the coefficients by key.  The coefficients are those of
// the per-hit solve bit for bit; an item with more than kFwdMemoKeys keys
// per wave goes on hit by hit.

// Thin-film coefficients of one hit for this lane (fills the lane's slot table).
template <int MODE, class SL, class Stks>
__device__ inline Coef4 hit_solve(const SceneDev& sc, const PointLds& pl, const Stks& stks,
                                  const SL& sl, int m, bool front, double kappa,
                                  bool* used_fp64, double* ck = nullptr, int64_t ckb = 8)
{
    bool hyp = false;                       // an evanescent lossless slot at this kappa
    for (int s = 0; s < sc.n_slots; ++s) {
        double P[NPF];
        slot_params(pl.slotN[2 * s], pl.slotN[2 * s + 1], kappa, pl.k0, P);
        sl.put(s, P);
        hyp |= !((sc.slot_complex >> s) & 1u) && P[0] < 0.0;
    }
    const bool circ = __ballot(hyp) == 0ull;
    const double z0 = pl.ng * pl.ng - kappa * kappa;
    const double q0 = sqrt(z0 > kTinyZ ? z0 : kTinyZ);
    const double eta0s = q0, eta0p = pl.ng * pl.ng / q0;
    const int L = pl.nlay[m];
    const auto stk = stks.mirror(m);
    const bool fp64 = (MODE == GWG_FP64) || (MODE == GWG_FP32_MIXED && near_critical(pl, sc.n_slots, kappa));
    *used_fp64 = fp64;
    if (fp64)
        return tmm_solve<double>(stk, L, front, sl, sc.slot_complex, pl.k0, eta0s, eta0p,
                                 mk(eta0s, 0.0), mk(eta0p, 0.0), mk(1.0, 0.0), circ, MODE == GWG_FP64 ? ck : nullptr,
                                 ckb);
    return tmm_solve<float>(stk, L, front, sl, sc.slot_complex, pl.k0, eta0s, eta0p,
                            mk(eta0s, 0.0), mk(eta0p, 0.0), mk(1.0, 0.0), circ);
}

// Dense hit p (the wave's hits in ray order) belongs to the largest lane
// whose exclusive prefix sum of hit counts (off) is <= p: lanes without hits
// share the next lane's offset and lose the search to it.  Returns its queue
// slot.  Called by all lanes of the wave (shuffles).
__device__ inline int dense_slot(int p, int off, int)
{
    int l = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int c = l + step;
        if (__shfl(off, c, 64) <= p) l = c;
    }
    return hq_slot(l, p - __shfl(off, l, 64));
}

// Solve the wave's `total` queued hits in batches of 64 (one per lane);
// off: this lane's exclusive prefix sum of hit counts.  perm: take the hits
// in the order queue field 11 lists (else lane by lane).
// ck (non-null): checkpoint store of the adjoint entries; a hit whose
// queue field 10 holds a slot c >= 0 stores its sweep checkpoints there.
template <int MODE, class SL, class Stks>
__device__ inline void solve_hits(const SceneDev& sc, const PointLds& pl, const Stks& stks,
                                  const SL& sl, const HitQueue& hq, int total,
                                  int off, unsigned long long* n_fp64, unsigned long long* n_lay,
                                  double* ck = nullptr, int64_t ck_total = 0, bool perm = false)
{
    const int lane = wave_lane();
    for (int b = 0; b < total; b += 64) {
        const int p = b + lane;
        const int pp = p < total ? p : total - 1;
        const int q = perm ? (int)hq.base[11 * (int64_t)hq.cap + pp] : dense_slot(pp, off, sc.Kmax);
        if (p < total) {
            const double kappa = hq.kappa(q);
            const int meta = hq.meta(q);
            const int m = meta & 255;
            bool u64 = false;
            double* ckp = nullptr;
            if (ck) {
                const double c = hq.base[10 * (int64_t)hq.cap + q];
                if (c >= 0.0) ckp = ck + (int64_t)c * 8;
            }
            const Coef4 c = hit_solve<MODE>(sc, pl, stks, sl, m, (meta >> 8) & 1, kappa, &u64, ckp,
                                            8 * ck_total);
            hq.put_coef(q, c);
            *n_fp64 += u64 ? 1ull : 0ull;
            *n_lay += (unsigned long long)pl.nlay[m];
        }
    }
}

// ------------------------------------------------------- memoized solves
constexpr int kFwdMemoHash = 256;   // open-addressing slots (at most half full)

// One wave's key table: keys and hash slots in LDS, coefficients in global
// scratch (field f of key u at coef[f * kFwdMemoKeys + u]).
struct FwdMemo {
    unsigned long long* kbits;   // [kFwdMemoKeys] bits of kappa
    int* kmeta;                  // [kFwdMemoKeys] mirror | front << 8
    int* ksrc;                   // [kFwdMemoKeys] queue entry of the key's first hit
    int* hslot;                  // [kFwdMemoHash] key index, -1 if empty
    double* coef;                // [8][kFwdMemoKeys]
};

__host__ __device__ inline int fwd_memo_wave_bytes() { return kFwdMemoKeys * (8 + 4 + 4) + kFwdMemoHash * 4; }

__device__ inline FwdMemo fwd_memo(unsigned char* base, int w, double* coef)
{
    unsigned char* mb = base + w * fwd_memo_wave_bytes();
    FwdMemo fm;
    fm.kbits = (unsigned long long*)mb;
    fm.kmeta = (int*)(mb + 8 * kFwdMemoKeys);
    fm.ksrc = (int*)(mb + 12 * kFwdMemoKeys);
    fm.hslot = (int*)(mb + 16 * kFwdMemoKeys);
    fm.coef = coef;
    return fm;
}

__device__ inline int fmemo_hash(unsigned long long kb, int km)
{
    uint32_t x = (uint32_t)kb ^ ((uint32_t)(kb >> 32) * 0x9E3779B1u) ^ ((uint32_t)km * 0x85EBCA77u);
    x ^= x >> 15;
    x *= 0x2C1B3C6Du;
    x ^= x >> 12;
    return (int)(x & (kFwdMemoHash - 1));
}

// Key index of (kb, km), or -1 - s with s the empty slot that ends its probe.
__device__ inline int fmemo_find(const FwdMemo& fm, unsigned long long kb, int km)
{
    int h = fmemo_hash(kb, km);
    for (;;) {
        const int u = fm.hslot[h];
        if (u < 0) return -1 - h;
        if (fm.kbits[u] == kb && fm.kmeta[u] == km) return u;
        h = (h + 1) & (kFwdMemoHash - 1);
    }
}

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);      // this wave's LDS operations have completed (lgkmcnt = 0)
    __builtin_amdgcn_wave_barrier();
}

// Resolve the wave's `total` queued hits to key indices, appending new keys
// to the table (*U keys so far); a hit's index goes to its first coefficient
// field.  Returns false if the table would hold more than cap keys.
__device__ inline bool fmemo_resolve(const HitQueue& hq, int total, int off, int kmax, const FwdMemo& fm, int cap,
                                     int* U)
{
    const int lane = wave_lane();
    for (int b = 0; b < total; b += 64) {
        const int p0 = b + lane;
        const bool act = p0 < total;
        const int p = dense_slot(act ? p0 : total - 1, off, kmax);
        unsigned long long kb = 0ull;
        int km = 0, idx = 0;
        if (act) {
            kb = (unsigned long long)__double_as_longlong(hq.kappa(p));
            km = hq.meta(p) & 511;
            idx = fmemo_find(fm, kb, km);
        }
        for (;;) {
            const unsigned long long open = __ballot(act && idx < 0);
            if (open == 0ull) break;
            if (*U == cap) return false;
            const int leader = __ffsll((long long)open) - 1;
            const int u = *U;
            if (lane == leader) {
                fm.kbits[u] = kb; fm.kmeta[u] = km; fm.ksrc[u] = p;
                fm.hslot[-1 - idx] = u;
            }
            *U = u + 1;
            wave_lds_sync();
            // the others probe again: the new key may be theirs, or may have
            // taken the slot their probe ended at
            if (act && idx < 0) idx = fmemo_find(fm, kb, km);
        }
        if (act) hq.base[2 * hq.cap + p] = (double)idx;
    }
    return true;
}

// Solve keys [u0, u1) (one per lane) from their first hits into the table.
template <int MODE, class SL, class Stks>
__device__ inline void fmemo_solve(const SceneDev& sc, const PointLds& pl, const Stks& stks,
                                   const SL& sl, const HitQueue& hq,
                                   const FwdMemo& fm, int u0, int u1, unsigned long long* n_fp64,
                                   unsigned long long* n_lay)
{
    const int lane = wave_lane();
    for (int b = u0; b < u1; b += 64) {
        const int u = b + lane;
        if (u < u1) {
            const int p = fm.ksrc[u];
            const double kappa = hq.kappa(p);
            const int meta = hq.meta(p);
            const int m = meta & 255;
            bool u64 = false;
            const Coef4 c = hit_solve<MODE>(sc, pl, stks, sl, m, (meta >> 8) & 1, kappa, &u64);
            double* o = fm.coef + u;
            o[0] = c.rs.re; o[kFwdMemoKeys] = c.rs.im; o[2 * kFwdMemoKeys] = c.rp.re; o[3 * kFwdMemoKeys] = c.rp.im;
            o[4 * kFwdMemoKeys] = c.ts.re; o[5 * kFwdMemoKeys] = c.ts.im;
            o[6 * kFwdMemoKeys] = c.tp.re; o[7 * kFwdMemoKeys] = c.tp.im;
            *n_fp64 += u64 ? 1ull : 0ull;
            *n_lay += (unsigned long long)pl.nlay[m];
        }
    }
}

struct NoHit {
    __device__ void operator()(int, double, int) const {}
    __device__ void branch(int, bool) const {}
};
struct NoCoef {
    static constexpr bool kStoredBranch = false;
    __device__ bool refl(int) const { return false; }
    __device__ Coef4 operator()(int, double, double, double, int, bool) const
    {
        Coef4 c;
        c.rs = c.rp = c.ts = c.tp = mk(0.0, 0.0);
        return c;
    }
};
struct PutHit {
    HitQueue q;
    int off;
    __device__ void operator()(int h, double kappa, int meta) const { q.put(hq_slot(off, h), kappa, meta); }
    __device__ void branch(int, bool) const {}
};
// Coefficients of the ray's hit h: from its queue entry, or (mc set) from
// the key table at the index its queue entry holds.
struct GetCoef {
    HitQueue q;
    int off;
    const double* mc;
    static constexpr bool kStoredBranch = true;   // the geometry walk stored the branch in the meta word
    __device__ bool refl(int h) const { return (((int)q.base[q.cap + hq_slot(off, h)]) >> 9) & 1; }
    __device__ Coef4 operator()(int h, double, double, double, int, bool) const
    {
        if (!mc) return q.coef(hq_slot(off, h));
        const double* b = mc + (int)q.base[2 * q.cap + hq_slot(off, h)];
        Coef4 c;
        c.rs = mk(b[0], b[kFwdMemoKeys]); c.rp = mk(b[2 * kFwdMemoKeys], b[3 * kFwdMemoKeys]);
        c.ts = mk(b[4 * kFwdMemoKeys], b[5 * kFwdMemoKeys]); c.tp = mk(b[6 * kFwdMemoKeys], b[7 * kFwdMemoKeys]);
        return c;
    }
};

// Persistent workgroups walk the work items with a fixed stride; each wave
// handles a strided share of the item's rays.  Eyebox bins of the current
// point accumulate in LDS (integer atomics) and are flushed per item with
// integer global atomics: the result does not depend on scheduling.
template <int MODE, bool ADJ, bool TAB, bool MEMO>
__global__ void __launch_bounds__(256, 2) k_trace_fwd(SceneDev sc, uint64_t* __restrict__ q_out,
                                                   uint32_t* __restrict__ c_out,
                                                   unsigned long long* __restrict__ stats,
                                                   gwg_ray_record* __restrict__ rec, int64_t rec_stride,
                                                   int lds_bins, double* __restrict__ scratch, AdjStore st,
                                                   double* __restrict__ tape_scratch)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int B = sc.bins_x * sc.bins_y;
    const int WG = blockDim.x;
    const int n_waves = WG / 64;
    // slot table: all five values per lane, except with the memoized solves,
    // whose key tables need the LDS (they solve few hits)
    using SlotTable = typename std::conditional<MEMO, LaneSlots3, LaneSlots3x>::type;
    const SmemLayout lay = smem_layout(sc.M, sc.Lmax, sc.n_slots, WG, B, lds_bins != 0, 0, SlotTable::kPer, true);
    PointLds* pl = (PointLds*)(smem + lay.off_pl);
    LayerRec* s_rec = (LayerRec*)(smem + lay.off_thk);
    const RecStacks stks = { s_rec, sc.Lmax };
    double* s_sp = (double*)(smem + lay.off_sp);
    unsigned long long* s_q = (unsigned long long*)(smem + lay.off_q);
    uint32_t* s_c = (uint32_t*)(smem + lay.off_c);
    unsigned long long* s_st = (unsigned long long*)(smem + lay.off_st);
    const int tid = threadIdx.x, wave = tid / 64, lane = wave_lane();
    const int64_t gwave = (int64_t)blockIdx.x * n_waves + wave;
    const int cap = 64 * sc.Kmax;
    const HitQueue hq = { scratch + gwave * (int64_t)kHitFields * cap, cap };
    const SlotTable sl = { slot_lane_base(s_sp, sc.n_slots, SlotTable::kPer, tid), pl->nsq, pl->pxy };
    const double wscale = ldexp(1.0, sc.fp_shift), wcap = ldexp(1.0, 40), pscale = 16777216.0;
    for (int k = tid; k < ST_WORDS; k += WG) s_st[k] = 0ull;
    unsigned long long n_fp64 = 0, n_lay = 0;
    const TapeRef tape = { tape_scratch + (int64_t)blockIdx.x * WG + tid, (int64_t)gridDim.x * WG };
    const FwdMemo fm = fwd_memo(smem + lay.total, wave,
                                scratch + (int64_t)gridDim.x * n_waves * kHitFields * cap + gwave * 8 * kFwdMemoKeys);
    constexpr bool tabm = TAB;                           // angle-table thin film: no hit queue
    double t_gmax = 0.0;                                 // largest cotangent component (angle table)
    unsigned long long t_ne = 0;                         // cotangent pairs emitted (angle table)

    for (int64_t it = draw_item(stats + ST_NEXT0); it < sc.n_items; it = draw_item(stats + ST_NEXT0)) {
        const int64_t item = sc.fwd_order ? (int64_t)sc.fwd_order[it] : it;
        int64_t point, i0, i1;
        int d, l, f;
        decode_item(sc, item, &point, &d, &l, &f, &i0, &i1);
        stage_point(sc, d, l, f, pl, nullptr, nullptr, s_rec, SlotTable::kPer);
        int64_t n_work = 0;                               // this wave's mirror hits in this item (uniform)
        if (lds_bins)
            for (int k = tid; k < B; k += WG) { s_q[k] = 0ull; s_c[k] = 0u; }
        __syncthreads();
        const int64_t base = point * sc.N;
        uint64_t* gq = q_out + point * B;
        uint32_t* gc = c_out + point * B;
        int64_t n_ent = 0;                                // this wave's entries in this item (uniform)
        bool memo = MEMO && sc.memo != 0;                 // this wave's key table is in use (uniform)
        int n_keys = 0;
        if (memo) {
            for (int k = lane; k < kFwdMemoHash; k += 64) fm.hslot[k] = -1;
            wave_lds_sync();
        }
        const int64_t ent0 = (item * st.waves + wave) * st.cap_w;
        const double* tab_dl = tabm ? sc.table + (int64_t)(d * sc.n_lsel + l) * sc.M * 2 * sc.table_n * 8 : nullptr;
        for (int64_t round = 0;; ++round) {
            const int64_t wave_first = i0 + (int64_t)wave * 64 + round * WG;
            if (wave_first >= i1) break;                  // uniform across the wave
            const int64_t i = wave_first + lane;
            const bool active = i < i1;
            const int64_t id = base + i;
            Ray r;
            Outcome o;
            TapeRef none = { nullptr, 0 };
            int nh = 0;
            bool to_eyebox = false;                        // fixed by geometry alone
            // geometry walk: the hits go to this lane's slots of the queue
            // (the angle table needs no queue: the walk only finds the rays
            // bound for the eyebox, whose fields the adjoint tapes)
            const int own = lane;                          // this lane's column of the hit queue
            if (active && (!tabm || ADJ)) {
                ray_birth(sc, *pl, id, r);
                if (tabm)
                    walk_ray<false, false>(sc, *pl, r, o, NoHit{}, NoCoef{}, none, nullptr);
                else
                    walk_ray<false, false>(sc, *pl, r, o, PutHit{ hq, own }, NoCoef{}, none, nullptr);
                nh = r.nprma;
                to_eyebox = o.cat == CAT_EYEBOX;
            }
            if (!tabm) {
                int total;
                const int off = wave_excl_scan(nh, &total);
                n_work += total;
                // FP64 with a checkpoint store: the hits of rays bound for the
                // eyebox learn the slots of their future adjoint entries (the
                // sweep emits a ray's hits last to first)
                const bool cks = ADJ && MODE == GWG_FP64 && st.ck != nullptr && !memo;
                if (cks) {
                    int etot;
                    const int eoff = wave_excl_scan(to_eyebox ? nh : 0, &etot);
                    for (int h = 0; h < nh; ++h) {
                        const int64_t k = n_ent + eoff + (nh - 1 - h);
                        double c = -1.0;
                        if (to_eyebox && k < st.ck_cap) c = (double)((item * st.waves + wave) * st.ck_cap + k);
                        hq.base[10 * (int64_t)cap + hq_slot(own, h)] = c;
                    }
                }
                // solve order: first the hits that may meet an evanescent
                // layer (kappa^2 above the smallest lossless Re N^2), then the
                // rest, so that most batches of 64 take the circular-only sweep
                // (a batch's kind is still decided from its hits' own layers)
                if (!MEMO) {
                    int ne = 0;
                    for (int h = 0; h < nh; ++h) {
                        const double k = hq.kappa(hq_slot(own, h));
                        ne += k * k > pl->kap2_evan ? 1 : 0;
                    }
                    int net;
                    const int eo = wave_excl_scan(ne, &net);
                    int pe = eo, pc = net + (off - eo);    // positions < total
                    for (int h = 0; h < nh; ++h) {
                        const int q = hq_slot(own, h);
                        const double k = hq.kappa(q);
                        const int pos = k * k > pl->kap2_evan ? pe++ : pc++;
                        hq.base[11 * (int64_t)cap + pos] = (double)q;
                    }
                }
                __threadfence_block();
                const int u0 = n_keys;
                if (MEMO && memo && !fmemo_resolve(hq, total, off, sc.Kmax, fm, sc.memo, &n_keys)) memo = false;
                if (MEMO && memo)
                    fmemo_solve<MODE>(sc, *pl, stks, sl, hq, fm, u0, n_keys, &n_fp64, &n_lay);
                else
                    solve_hits<MODE>(sc, *pl, stks, sl, hq, total, off, &n_fp64, &n_lay,
                                     cks ? st.ck : nullptr, st.ck_total, !MEMO);
                __threadfence_block();
            }
            int nt = 0;
            if (active) {
                ray_birth(sc, *pl, id, r);
                const TapeRef rt = { to_eyebox ? tape.base : nullptr, tape.ts };
                if constexpr (TAB)
                    walk_ray<true, ADJ>(sc, *pl, r, o, NoHit{}, TabCoef{ tab_dl, sc.table_n, pl->ng, sc.nx, sc.nz }, rt, &nt);
                else
                    walk_ray<true, ADJ>(sc, *pl, r, o, NoHit{}, GetCoef{ hq, own, MEMO && memo ? fm.coef : nullptr }, rt, &nt);
                atomicAdd(&s_st[ST_RAYS], 1ull);
                atomicAdd(&s_st[ST_EVENTS], (unsigned long long)r.nev);
                atomicAdd(&s_st[ST_PRMA], (unsigned long long)r.nprma);
                atomicAdd(&s_st[ST_CAT + o.cat], 1ull);
                const double pw = o.w * pscale;
                atomicAdd(&s_st[ST_POW + o.cat], (unsigned long long)rint(pw < wcap ? pw : wcap));
                if (o.cat == CAT_EYEBOX || o.cat == CAT_MISS) {
                    const double pr = (o.w_in - o.w) * pscale;
                    if (pr > 0.0) atomicAdd(&s_st[ST_POW + CAT_FACE_R], (unsigned long long)rint(pr < wcap ? pr : wcap));
                }
                if (o.cat == CAT_EYEBOX) {
                    double u = o.w * wscale;
                    if (!(u <= wcap)) { u = (u > wcap) ? wcap : 0.0; atomicAdd(&s_st[ST_SAT], 1ull); }
                    const unsigned long long qv = (unsigned long long)rint(u);
                    if (lds_bins) { atomicAdd(&s_q[o.bin], qv); atomicAdd(&s_c[o.bin], 1u); }
                    else { atomicAdd((unsigned long long*)&gq[o.bin], qv); atomicAdd(&gc[o.bin], 1u); }
                }
                if (rec && (id % rec_stride) == 0) {
                    gwg_ray_record* q = rec + id / rec_stride;
                    q->bin = o.cat == CAT_EYEBOX ? o.bin : -1;
                    q->category = o.cat;
                    q->n_events = r.nev;
                    q->n_prma = r.nprma;
                    q->w = o.w;
                }
            }
            if (ADJ) {
                const bool eb = active && o.cat == CAT_EYEBOX;
                int etotal;
                const int eoff = wave_excl_scan(eb ? r.nprma : 0, &etotal);
                if (eb) {
                    int64_t k = n_ent + eoff;
                    const int64_t cap = st.cap_w;
                    const int64_t meta_bin = (int64_t)o.bin << 10;
                    reverse_sweep(sc, *pl, r.e, tape, nt, [&](double kappa, cd Gs, cd Gp, int meta) {
                        if constexpr (TAB) {
                            const double a = fmax(fmax(fabs(Gs.re), fabs(Gs.im)), fmax(fabs(Gp.re), fabs(Gp.im)));
                            t_gmax = a > t_gmax ? a : t_gmax;
                            ++t_ne;
                        }
                        if (k < cap) {
                            const int64_t e = ent0 + k;
                            st.ent[e] = kappa;
                            st.ent[1 * st.total + e] = Gs.re;
                            st.ent[2 * st.total + e] = Gs.im;
                            st.ent[3 * st.total + e] = Gp.re;
                            st.ent[4 * st.total + e] = Gp.im;
                            st.ent[5 * st.total + e] = (double)(meta_bin | (int64_t)meta);
                        }
                        ++k;
                    });
                }
                n_ent += etotal;
            }
        }
        if (ADJ && lane == 0) {
            st.cnt[item * st.waves + wave] = (int32_t)(n_ent < st.cap_w ? n_ent : st.cap_w);
            if (n_ent > st.cap_w) st.ovf[item] = 1;
        }
        if (sc.item_work && lane == 0) sc.item_work[item * n_waves + wave] = (int32_t)n_work;
        __syncthreads();
        if (lds_bins) {
            for (int k = tid; k < B; k += WG) {
                if (s_c[k]) {
                    atomicAdd((unsigned long long*)&gq[k], s_q[k]);
                    atomicAdd(&gc[k], s_c[k]);
                }
            }
        }
    }
    if (n_fp64) atomicAdd(&s_st[ST_FP64], n_fp64);
    if (n_lay) atomicAdd(&s_st[ST_LAYERS], n_lay);
    if constexpr (ADJ && TAB) {
        // nonnegative doubles order like their bit patterns
        const double gm = wave_max(t_gmax);
        if (lane == 0 && gm > 0.0) atomicMax(&sc.tab_scale[0], (unsigned long long)__double_as_longlong(gm));
        if (t_ne) atomicAdd(&sc.tab_scale[1], t_ne);
    }
    __syncthreads();
    for (int k = tid; k < ST_WORDS; k += WG)
        if (s_st[k]) atomicAdd(&stats[k], s_st[k]);
}

int64_t fwd_scratch_doubles(const SceneDev& sc, int64_t grid_blocks, int wg)
{
    return grid_blocks * (wg / 64) * ((int64_t)kHitFields * 64 * sc.Kmax + (sc.memo ? 8 * kFwdMemoKeys : 0));
}
