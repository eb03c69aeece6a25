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
                                 ckb, ck_interval(hyp));
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

// ----------------------------------------------------- pooled rounds
// The per-hit forward handles a wave's rays in pools of up to sc.pool rounds
// (kPoolMax at most).  The queue holds the pool's hits: ncol = 64 sc.pool
// columns (one per ray) of Kmax slots, hit h of column col in slot
// h * ncol + col.  Inputs of the solves: fields 0 (kappa), 1 (meta), 10
// (checkpoint slot), 11 (solve order).  The solves write each hit's taken
// coefficients (c_s, c_p: fields 2-5) and its branch (field 6) in the slot
// of the ray's place in the field-pass order (column pos), so the lanes of a
// field pass read adjacent slots.
constexpr int kSortBins = 128;                      // walk-length classes of the field-pass order

// doubles of global scratch per wave: the hit queue (kHitFields fields of
// 64 sc.pool sc.Kmax slots), one 64-bit word per column (carried data), and
// two 32-bit words per column (place in the order, column at each place)
__host__ __device__ inline int64_t fwd_wave_doubles(const SceneDev& sc)
{
    return (int64_t)kHitFields * 64 * sc.pool * sc.Kmax + 2 * 64 * sc.pool;
}

// Also counts the ray's hits whose kappa^2 exceeds kap2 (they may meet an
// evanescent layer) in *ne and marks hits h < 64 of them in bit h of *evm.
struct PutHitP {
    HitQueue q;
    int col, ncol;
    double kap2;
    int* ne;
    unsigned long long* evm;
    __device__ void operator()(int h, double kappa, int meta) const
    {
        q.put(h * ncol + col, kappa, meta);
        if (kappa * kappa > kap2) {
            ++*ne;
            if (h < 64) *evm |= 1ull << h;
        }
    }
    __device__ void branch(int, bool) const {}
};
// The field pass's coefficients of the ray at place pos of the order: the
// taken pair (c_s, c_p) returned as both the reflected and the transmitted
// one, and the branch.
struct GetCoefP {
    HitQueue q;
    int pos, ncol;
    static constexpr bool kStoredBranch = true;
    __device__ bool refl(int h) const { return q.base[6 * (int64_t)q.cap + h * ncol + pos] != 0.0; }
    __device__ Coef4 operator()(int h, double, double, double, int, bool) const
    {
        const double* b = q.base + 2 * (int64_t)q.cap + h * ncol + pos;
        const int64_t c = q.cap;
        Coef4 o;
        o.rs = o.ts = mk(b[0], b[c]);
        o.rp = o.tp = mk(b[2 * c], b[3 * c]);
        return o;
    }
};

// Solve a pool's ne + nc queued hits in batches of 64 (one per lane): field
// 11 lists the possibly evanescent hits' slots from its front (positions
// 0 .. ne-1) and the others' from its back (cap-1 down to cap-nc), so the
// batches of the second kind take the circular-only sweep.  colpos[col]:
// the place of column col in the field-pass order, where the hit's taken
// coefficients go.  ck (non-null): the checkpoint store; a hit whose field
// 10 holds a slot c >= 0 stores its sweep checkpoints there.
template <int MODE, class SL, class Stks>
__device__ inline void solve_pool(const SceneDev& sc, const PointLds& pl, const Stks& stks, const SL& sl,
                                  const HitQueue& hq, int ncol, const int32_t* colpos, int ne, int nc,
                                  unsigned long long* n_fp64, unsigned long long* n_lay, double* ck, int64_t ck_total)
{
    const int lane = wave_lane();
    const int total = ne + nc;
    const double* ord = hq.base + 11 * (int64_t)hq.cap;
    for (int b = 0; b < total; b += 64) {
        const int p = b + lane;
        if (p < total) {
            const int q = (int)ord[p < ne ? p : hq.cap - 1 - (p - ne)];
            const double kappa = hq.kappa(q);
            const int meta = hq.meta(q);
            const int m = meta & 255;
            bool u64 = false;
            double* ckp = nullptr;
            if (ck) {
                const double c = hq.base[10 * (int64_t)hq.cap + q];
                if (c >= 0.0) ckp = ck + (int64_t)c * 8;
            }
            const Coef4 c = hit_solve<MODE>(sc, pl, stks, sl, m, (meta >> 8) & 1, kappa, &u64, ckp, 8 * ck_total);
            const int h = q / ncol, col = q - h * ncol;
            const bool rf = (meta >> 9) & 1;
            double* o = hq.base + 2 * (int64_t)hq.cap + h * ncol + colpos[col];
            const int64_t cc = hq.cap;
            const cd cs = rf ? c.rs : c.ts, cp = rf ? c.rp : c.tp;
            o[0] = cs.re; o[cc] = cs.im; o[2 * cc] = cp.re; o[3 * cc] = cp.im;
            o[4 * cc] = rf ? 1.0 : 0.0;
            *n_fp64 += u64 ? 1ull : 0ull;
            *n_lay += (unsigned long long)pl.nlay[m];
        }
    }
}

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
    const int cap = 64 * sc.pool * sc.Kmax;                // queue slots of a wave (a pool of rounds)
    constexpr bool POOL = !MEMO && !TAB;
    const HitQueue hq = { scratch + gwave * fwd_wave_doubles(sc), cap };
    const SlotTable sl = { slot_lane_base(s_sp, sc.n_slots, SlotTable::kPer, tid), pl->nsq, pl->pxy };
    const double wscale = ldexp(1.0, sc.fp_shift), wcap = ldexp(1.0, 40), pscale = 16777216.0;
    for (int k = tid; k < ST_WORDS; k += WG) s_st[k] = 0ull;
    unsigned long long n_fp64 = 0, n_lay = 0;
    const TapeRef tape = tape_lane(tape_scratch, sc.Kmax, (int64_t)gridDim.x * n_waves, gwave, lane);
    const FwdMemo fm = fwd_memo(smem + lay.total, wave,
                                scratch + (int64_t)gridDim.x * n_waves * fwd_wave_doubles(sc) + gwave * 8 * kFwdMemoKeys);
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
        // The field pass of one ray: the walk with the polarization field
        // (coefficients from gcoef), the tape of the rays bound for the
        // eyebox, the statistics and the eyebox scatter, then the reverse
        // field sweep, whose adjoint entries take positions kent, kent + 1,
        // ... of the wave's region (the ray's hits, last to first).
        auto field_pass = [&](bool active, int64_t id, bool to_eyebox, int64_t kent, const auto& gcoef) {
            Ray r;
            Outcome o;
            int nt = 0;
            if (active) {
                ray_birth(sc, *pl, id, r);
                const TapeRef rt = { to_eyebox ? tape.ev : nullptr, tape.mr, tape.ks };
                walk_ray<true, ADJ>(sc, *pl, r, o, NoHit{}, gcoef, rt, &nt);
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
            const int ntw = ADJ ? wave_max_int(active && o.cat == CAT_EYEBOX ? nt : 0) : 0;
            if (ADJ && active && o.cat == CAT_EYEBOX) {
                int64_t k = kent;
                const int64_t cap_w = st.cap_w;
                const int64_t meta_bin = (int64_t)o.bin << 10;
                reverse_sweep(sc, *pl, r.e, tape, nt, ntw, [&](double kappa, cd Gs, cd Gp, int meta) {
                    if constexpr (TAB) {
                        const double a = fmax(fmax(fabs(Gs.re), fabs(Gs.im)), fmax(fabs(Gp.re), fabs(Gp.im)));
                        t_gmax = a > t_gmax ? a : t_gmax;
                        ++t_ne;
                    }
                    if (k < cap_w) {
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
        };
        if constexpr (POOL) {
            // Pools of up to sc.pool rounds of this wave's rays (64 per
            // round, a stride of WG rays apart): one geometry walk per ray,
            // the pool's hits solved in batches of 64, then the field passes
            // with the rays ordered by walk length, longest first, so that
            // the lanes of a round walk about equally long.  A ray's column
            // in the pool's queue is rr * 64 + lane (round rr of the pool);
            // its hit h sits in slot h * ncol + col.
            const int ncol = 64 * sc.pool;
            const int64_t first = i0 + (int64_t)wave * 64;
            const int n_rounds = first < i1 ? (int)((i1 - first + WG - 1) / WG) : 0;     // uniform
            // the ordering's class counts sit in this wave's slot tables,
            // which only the solves use (each hit's solve fills its lane's
            // table first)
            uint32_t* s_hist = (uint32_t*)(s_sp + (int64_t)wave * sc.n_slots * SlotTable::kPer * kSlotLanes);
            int64_t* colinfo = (int64_t*)(hq.base + (int64_t)kHitFields * cap);         // [ncol] carried data
            int32_t* colpos = (int32_t*)(colinfo + ncol);                               // [ncol] place of a column
            int32_t* colord = colpos + ncol;                                            // [ncol] column at a place
            const bool cks = ADJ && MODE == GWG_FP64 && st.ck != nullptr;
            for (int r0 = 0; r0 < n_rounds; r0 += sc.pool) {
                const int nr = n_rounds - r0 < sc.pool ? n_rounds - r0 : sc.pool;
                int n_e = 0, n_c = 0;                     // the pool's possibly evanescent / other hits (uniform)
                for (int rr = 0; rr < nr; ++rr) {
                    const int col = rr * 64 + lane;
                    const int64_t i = first + (int64_t)(r0 + rr) * WG + lane;
                    const bool active = i < i1;
                    Ray r;
                    Outcome o;
                    TapeRef none = { nullptr, nullptr, 0 };
                    int nh = 0, nev = 0, ne = 0;
                    unsigned long long evm = 0ull;         // bit h: hit h may meet an evanescent layer
                    bool to_eyebox = false;                // fixed by geometry alone
                    if (active) {
                        ray_birth(sc, *pl, base + i, r);
                        walk_ray<false, false>(sc, *pl, r, o, PutHitP{ hq, col, ncol, pl->kap2_evan, &ne, &evm },
                                               NoCoef{}, none, nullptr);
                        nh = r.nprma;
                        nev = r.nev;
                        to_eyebox = o.cat == CAT_EYEBOX;
                    }
                    int total;
                    (void)wave_excl_scan(nh, &total);
                    n_work += total;
                    // the ray's adjoint entries (rays bound for the eyebox)
                    // start at kent of the wave's region; with a checkpoint
                    // store its hits learn their entries' checkpoint slots
                    int64_t kent = 0;
                    if (ADJ) {
                        int etot;
                        const int eoff = wave_excl_scan(to_eyebox ? nh : 0, &etot);
                        kent = n_ent + eoff;
                        if (cks)
                            for (int h = 0; h < nh; ++h) {
                                const int64_t k = kent + (nh - 1 - h);
                                double c = -1.0;
                                if (to_eyebox && k < st.ck_cap) c = (double)((item * st.waves + wave) * st.ck_cap + k);
                                hq.base[10 * (int64_t)cap + h * ncol + col] = c;
                            }
                        n_ent += etot;
                    }
                    // solve order: the hits that may meet an evanescent layer
                    // from the front of field 11, the others from its back
                    int te, tc;
                    const int eo = wave_excl_scan(ne, &te);
                    const int co = wave_excl_scan(nh - ne, &tc);
                    int pe = n_e + eo, pc = n_c + co;
                    for (int h = 0; h < nh; ++h) {
                        const int q = h * ncol + col;
                        bool ev;
                        if (h < 64) {
                            ev = (evm >> h) & 1ull;
                        } else {
                            const double k = hq.kappa(q);
                            ev = k * k > pl->kap2_evan;
                        }
                        const int pos = ev ? pe++ : cap - 1 - pc++;
                        hq.base[11 * (int64_t)cap + pos] = (double)q;
                    }
                    n_e += te;
                    n_c += tc;
                    // walk-length class (0: no ray), carried data
                    const int cost = nev + (to_eyebox ? nev : 0);
                    const int key = active ? 1 + (cost < kSortBins - 2 ? cost : kSortBins - 2) : 0;
                    colinfo[col] = (kent << 16) | (int64_t)(key << 1) | (to_eyebox ? 1 : 0);
                }
                __threadfence_block();
                // the field-pass order: the pool's columns by walk-length
                // class, longest first (a counting sort)
                for (int k = lane; k < kSortBins; k += 64) s_hist[k] = 0u;
                wave_lds_sync();
                for (int rr = 0; rr < nr; ++rr) {
                    const int key = (int)((colinfo[rr * 64 + lane] >> 1) & 255);
                    atomicAdd(&s_hist[key], 1u);
                }
                wave_lds_sync();
                {
                    // bin offsets in decreasing class order (two bins a lane)
                    const int b0 = kSortBins - 1 - 2 * lane, b1 = b0 - 1;
                    const int h0 = (int)s_hist[b0], h1 = (int)s_hist[b1];
                    int tot;
                    const int ex = wave_excl_scan(h0 + h1, &tot);
                    s_hist[b0] = (uint32_t)ex;
                    s_hist[b1] = (uint32_t)(ex + h0);
                }
                wave_lds_sync();
                for (int rr = 0; rr < nr; ++rr) {
                    const int col = rr * 64 + lane;
                    const int key = (int)((colinfo[col] >> 1) & 255);
                    const int pos = (int)atomicAdd(&s_hist[key], 1u);
                    colpos[col] = pos;
                    colord[pos] = col;
                }
                wave_lds_sync();                          // the slot tables are the solves' again
                __threadfence_block();
                solve_pool<MODE>(sc, *pl, stks, sl, hq, ncol, colpos, n_e, n_c, &n_fp64, &n_lay,
                                 cks ? st.ck : nullptr, st.ck_total);
                __threadfence_block();
                for (int s2 = 0; s2 < nr; ++s2) {
                    const int pos = s2 * 64 + lane;
                    const int col = colord[pos];
                    const int64_t info = colinfo[col];
                    const int64_t i = first + (int64_t)(r0 + col / 64) * WG + (col & 63);
                    field_pass(((info >> 1) & 255) != 0, base + i, (info & 1) != 0, info >> 16,
                               GetCoefP{ hq, pos, ncol });
                }
                __threadfence_block();                    // the next pool's solves rewrite the queue
            }
        } else {
        for (int64_t round = 0;; ++round) {
            const int64_t wave_first = i0 + (int64_t)wave * 64 + round * WG;
            if (wave_first >= i1) break;                  // uniform across the wave
            const int64_t i = wave_first + lane;
            const bool active = i < i1;
            const int64_t id = base + i;
            Ray r;
            Outcome o;
            TapeRef none = { nullptr, nullptr, 0 };
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
            // this round's adjoint entries: ray by ray from kent (eyebox rays)
            int64_t kent = 0, etot_r = 0;
            if (ADJ) {
                int etot;
                const int eoff = wave_excl_scan(to_eyebox ? nh : 0, &etot);
                kent = n_ent + eoff;
                etot_r = etot;
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
                    for (int h = 0; h < nh; ++h) {
                        const int64_t k = kent + (nh - 1 - h);
                        double c = -1.0;
                        if (to_eyebox && k < st.ck_cap) c = (double)((item * st.waves + wave) * st.ck_cap + k);
                        hq.base[10 * (int64_t)cap + hq_slot(own, h)] = c;
                    }
                }
                __threadfence_block();
                const int u0 = n_keys;
                if (MEMO && memo && !fmemo_resolve(hq, total, off, sc.Kmax, fm, sc.memo, &n_keys)) memo = false;
                if (MEMO && memo)
                    fmemo_solve<MODE>(sc, *pl, stks, sl, hq, fm, u0, n_keys, &n_fp64, &n_lay);
                else
                    solve_hits<MODE>(sc, *pl, stks, sl, hq, total, off, &n_fp64, &n_lay,
                                     cks ? st.ck : nullptr, st.ck_total, false);
                __threadfence_block();
            }
            if constexpr (TAB)
                field_pass(active, id, to_eyebox, kent, TabCoef{ tab_dl, sc.table_n, pl->ng, sc.nx, sc.nz });
            else
                field_pass(active, id, to_eyebox, kent, GetCoef{ hq, own, MEMO && memo ? fm.coef : nullptr });
            if (ADJ) n_ent += etot_r;
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
    return grid_blocks * (wg / 64) * (fwd_wave_doubles(sc) + (sc.memo ? 8 * kFwdMemoKeys : 0));
}
