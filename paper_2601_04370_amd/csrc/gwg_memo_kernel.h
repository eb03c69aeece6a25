// Memoized thin-film adjoint.  Included by gwg_kernels.hip inside namespace gwg.
//
// The FoV beams are collimated, so within one work item (one design,
// wavelength and FoV point) the mirror hits share a handful of distinct
// (kappa, mirror, side, branch) keys: kappa is computed from direction bits
// that every ray with the same event history shares exactly.  The thin-film
// part of the gradient is linear in the cotangents,
//     sum_h 2 Re(G_h dc(kappa_h)/dt) = 2 Re((sum_{h in key} G_h) dc(kappa_key)/dt),
// so the backward sums the (dL/dI-scaled) cotangents of each key in entry
// order and runs one thin-film adjoint per key.  One workgroup per item; the
// sums run in a fixed order, so the gradient is deterministic: kMemoWaves
// waves each take a contiguous part of the item's entries with their own key
// table, and wave 0 merges the tables in wave and key order.  An item with
// more than kMemoKeys keys is drained hit by hit instead.

constexpr int kMemoKeys = 128;      // keys per wave table and per item
constexpr int kMemoWaves = 4;       // waves per work item

// One wave's key table and chunk staging in LDS.
struct MemoLds {
    unsigned long long* kbits;   // [kMemoKeys] bits of kappa
    int* kmeta;                  // [kMemoKeys] mirror | front << 8 | reflected << 9
    double* gsum;                // [4][kMemoKeys] sums of G_s (re, im), G_p (re, im)
    int* sidx;                   // [64] key of each lane's entry in the current chunk (-1: none)
    double* sg;                  // [4][64] the lane's scaled cotangents
};

__host__ __device__ inline int memo_wave_bytes() { return kMemoKeys * (8 + 4 + 32) + 64 * (4 + 32); }

__device__ inline MemoLds memo_table(unsigned char* base, int w)
{
    unsigned char* mb = base + w * memo_wave_bytes();
    MemoLds mt;
    mt.kbits = (unsigned long long*)mb;
    mt.gsum = (double*)(mb + 8 * kMemoKeys);
    mt.sg = (double*)(mb + 40 * kMemoKeys);
    mt.kmeta = (int*)(mb + 40 * kMemoKeys + 32 * 64);
    mt.sidx = (int*)(mb + 44 * kMemoKeys + 32 * 64);
    return mt;
}

// Entry v (in item order) -> index of its record; cnt: the item's region counts.
__device__ inline int64_t entry_index(const AdjStore& st, int64_t item, const int32_t* cnt, int v)
{
    int rr = 0, k = v;
    while (k >= cnt[rr]) { k -= cnt[rr]; ++rr; }
    return (item * st.waves + rr) * st.cap_w + k;
}

// One wave: keys by first appearance in entries [v0, v1) and the dL/dI-scaled
// cotangents summed per key, in entry order (the next chunk's records are
// loaded while the current one is processed).  Returns the number of keys,
// or -1 if they exceed kMemoKeys.
__device__ inline int memo_collect(const SceneDev& sc, const AdjStore& st, int64_t item, const int32_t* cnt,
                                   const double* g_bins, int v0, int v1, const MemoLds& mt)
{
    const int lane = wave_lane();
    const double invN = 1.0 / (double)sc.N;
    int U = 0;
    for (int k = lane; k < 4 * kMemoKeys; k += 64) mt.gsum[k] = 0.0;
    double nk = 0.0, ng[4] = { 0.0, 0.0, 0.0, 0.0 };
    int64_t nmeta = -1;
    auto fetch = [&](int c) {
        const int v = c + lane;
        nmeta = -1;
        if (v < v1) {
            const int64_t e = entry_index(st, item, cnt, v);
            nk = st.ent[e];
            nmeta = (int64_t)st.ent[5 * st.total + e];
            for (int q = 0; q < 4; ++q) ng[q] = st.ent[(1 + q) * st.total + e];
        }
    };
    fetch(v0);
    for (int c = v0; c < v1; c += 64) {
        const double ck = nk;
        const int64_t cmeta = nmeta;
        const double cg0 = ng[0], cg1 = ng[1], cg2 = ng[2], cg3 = ng[3];
        if (c + 64 < v1) fetch(c + 64);
        double gscale = 0.0;
        if (cmeta >= 0) gscale = g_bins[(int)(cmeta >> 10)] * invN;
        const bool valid = gscale != 0.0;
        const unsigned long long kb = (unsigned long long)__double_as_longlong(ck);
        const int km = (int)(cmeta & 1023);
        int idx = -1;
        if (valid)
            for (int u = 0; u < U; ++u)
                if (mt.kbits[u] == kb && mt.kmeta[u] == km) { idx = u; break; }
        for (;;) {
            const unsigned long long open = __ballot(valid && idx < 0);
            if (open == 0ull) break;
            if (U == kMemoKeys) return -1;
            const int leader = __ffsll((long long)open) - 1;
            const unsigned long long lkb = __shfl(kb, leader, 64);
            const int lkm = __shfl(km, leader, 64);
            if (lane == 0) { mt.kbits[U] = lkb; mt.kmeta[U] = lkm; }
            if (valid && idx < 0 && kb == lkb && km == lkm) idx = U;
            ++U;
        }
        mt.sidx[lane] = valid ? idx : -1;
        mt.sg[lane] = cg0 * gscale; mt.sg[64 + lane] = cg1 * gscale;
        mt.sg[128 + lane] = cg2 * gscale; mt.sg[192 + lane] = cg3 * gscale;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xc07f);      // this wave's LDS writes are visible (lgkmcnt = 0)
        for (int k = lane; k < U; k += 64) {
            double a0 = mt.gsum[k], a1 = mt.gsum[kMemoKeys + k];
            double a2 = mt.gsum[2 * kMemoKeys + k], a3 = mt.gsum[3 * kMemoKeys + k];
            for (int j = 0; j < 64; ++j)
                if (mt.sidx[j] == k) {
                    a0 += mt.sg[j]; a1 += mt.sg[64 + j]; a2 += mt.sg[128 + j]; a3 += mt.sg[192 + j];
                }
            mt.gsum[k] = a0; mt.gsum[kMemoKeys + k] = a1;
            mt.gsum[2 * kMemoKeys + k] = a2; mt.gsum[3 * kMemoKeys + k] = a3;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xc07f);
    }
    return U;
}

// Wave 0 merges the key tables of waves 1.. into its own, in wave and key
// order (nk[w]: wave w's key count, -1 if its table overflowed).  Returns the
// merged key count, or -1 if a table overflowed or the merge would.
__device__ inline int memo_merge(unsigned char* mbase, const int* nk)
{
    const int lane = wave_lane();
    const MemoLds m0 = memo_table(mbase, 0);
    for (int w = 0; w < kMemoWaves; ++w)
        if (nk[w] < 0) return -1;
    int U = nk[0];
    for (int w = 1; w < kMemoWaves; ++w) {
        const MemoLds mw = memo_table(mbase, w);
        for (int u = 0; u < nk[w]; ++u) {
            const unsigned long long kb = mw.kbits[u];
            const int km = mw.kmeta[u];
            int idx = -1;
            for (int k = lane; k < U; k += 64)
                if (m0.kbits[k] == kb && m0.kmeta[k] == km) idx = k;
            const unsigned long long hit = __ballot(idx >= 0);
            if (hit) idx = __shfl(idx, __ffsll((long long)hit) - 1, 64);
            else {
                if (U == kMemoKeys) return -1;
                idx = U++;
                if (lane == 0) {
                    m0.kbits[idx] = kb; m0.kmeta[idx] = km;
                    for (int q = 0; q < 4; ++q) m0.gsum[q * kMemoKeys + idx] = 0.0;
                }
            }
            if (lane == 0)
                for (int q = 0; q < 4; ++q) m0.gsum[q * kMemoKeys + idx] += mw.gsum[q * kMemoKeys + u];
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0xc07f);
        }
    }
    return U;
}

template <bool LOSSLESS>
__global__ void __launch_bounds__(64 * kMemoWaves, 2) k_adj_memo(SceneDev sc, const double* __restrict__ dLdI,
                                                              double* __restrict__ partial, AdjStore st,
                                                              double* __restrict__ scratch,
                                                              unsigned long long* __restrict__ stats)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int B = sc.bins_x * sc.bins_y;
    const SmemLayout lay = smem_layout(sc.M, sc.Lmax, sc.n_slots, 64, B, false, 1);
    PointLds* pl = (PointLds*)(smem + lay.off_pl);
    double* s_thk = (double*)(smem + lay.off_thk);
    uint8_t* s_slot = (uint8_t*)(smem + lay.off_slot);
    double* s_sp = (double*)(smem + lay.off_sp);
    double* gw = (double*)(smem + lay.off_grad);
    unsigned long long* s_st = (unsigned long long*)(smem + lay.off_st);
    unsigned char* mbase = smem + align16(lay.total);
    int* s_nkeys = (int*)(mbase + kMemoWaves * memo_wave_bytes());
    const int tid = threadIdx.x, wave = tid / 64, lane = wave_lane();
    const MemoLds mt = memo_table(mbase, wave);
    const MemoLds m0 = memo_table(mbase, 0);
    const int ML = sc.M * sc.Lmax;
    const LaneSlots3 sl = { slot_lane_base(s_sp, sc.n_slots, LaneSlots3::kPer, lane), pl->nsq, pl->pxy };     // wave 0's lanes
    const int64_t nthreads = (int64_t)gridDim.x * 64;
    double* chk = scratch + (int64_t)blockIdx.x * 64 + lane;
    for (int k = tid; k < ST_WORDS; k += 64 * kMemoWaves) s_st[k] = 0ull;
    unsigned long long c_keys = 0, c_lay = 0;

    for (int64_t item = draw_item(stats + ST_NEXT0); item < sc.n_items; item = draw_item(stats + ST_NEXT0)) {
        if (st.ovf[item] != 0) continue;
        int64_t point, i0, i1;
        int d, l, f;
        decode_item(sc, item, &point, &d, &l, &f, &i0, &i1);
        stage_point(sc, d, l, f, pl, s_thk, s_slot);
        for (int k = tid; k < ML; k += 64 * kMemoWaves) gw[k] = 0.0;
        const double* g_bins = dLdI + point * B;
        const int32_t* cnt = st.cnt + item * st.waves;
        int total = 0;
        for (int w = 0; w < st.waves; ++w) total += cnt[w];
        // wave w takes a contiguous part of the entries
        const int per = (total + kMemoWaves - 1) / kMemoWaves;
        const int v0 = min(wave * per, total), v1 = min(v0 + per, total);
        const int nk = memo_collect(sc, st, item, cnt, g_bins, v0, v1, mt);
        if (lane == 0) s_nkeys[wave] = nk;
        __syncthreads();
        if (wave == 0) {
            const int U = memo_merge(mbase, s_nkeys);
            if (U < 0) {
                // too many keys: one thin-film adjoint per entry
                const double invN = 1.0 / (double)sc.N;
                for (int c = 0; c < total; c += 64) {
                    const int v = c + lane;
                    if (v < total) {
                        const int64_t e = entry_index(st, item, cnt, v);
                        const int64_t meta = (int64_t)st.ent[5 * st.total + e];
                        const double gscale = g_bins[(int)(meta >> 10)] * invN;
                        if (gscale != 0.0) {
                            const cd Gs = cscale(mk(st.ent[1 * st.total + e], st.ent[2 * st.total + e]), gscale);
                            const cd Gp = cscale(mk(st.ent[3 * st.total + e], st.ent[4 * st.total + e]), gscale);
                            const int mm = (int)(meta & 1023);
                            adjoint_hit<LOSSLESS>(sc, *pl, s_thk, s_slot, sl, gw, st.ent[e], Gs, Gp, mm, chk, nthreads);
                            c_keys += 1;
                            c_lay += (unsigned long long)pl->nlay[mm & 255];
                        }
                    }
                }
            } else {
                // one thin-film adjoint per key
                for (int b = 0; b < U; b += 64) {
                    const int k = b + lane;
                    if (k < U) {
                        const cd Gs = mk(m0.gsum[k], m0.gsum[kMemoKeys + k]);
                        const cd Gp = mk(m0.gsum[2 * kMemoKeys + k], m0.gsum[3 * kMemoKeys + k]);
                        const int mm = m0.kmeta[k];
                        adjoint_hit<LOSSLESS>(sc, *pl, s_thk, s_slot, sl, gw,
                                              __longlong_as_double((long long)m0.kbits[k]), Gs, Gp, mm, chk, nthreads);
                        c_keys += 1;
                        c_lay += (unsigned long long)pl->nlay[mm & 255];
                    }
                }
            }
        }
        __syncthreads();
        double* out = partial + item * (int64_t)ML;
        for (int k = tid; k < ML; k += 64 * kMemoWaves) out[k] = gw[k];
    }
    if (c_keys) atomicAdd(&s_st[ST_ADJ_HITS], c_keys);
    if (c_lay) atomicAdd(&s_st[ST_ADJ_LAYERS], c_lay);
    __syncthreads();
    for (int k = tid; k < ST_WORDS; k += 64 * kMemoWaves)
        if (s_st[k]) atomicAdd(&stats[k], s_st[k]);
}

size_t memo_smem_bytes(const SceneDev& sc)
{
    return (size_t)align16(smem_layout(sc.M, sc.Lmax, sc.n_slots, 64, sc.bins_x * sc.bins_y, false, 1).total) +
           (size_t)(kMemoWaves * memo_wave_bytes() + 16);
}
