// Angle-table thin film: table build and the table backward.  Included by
// gwg_kernels.hip inside namespace gwg, after the memoized adjoint.
//
// Forward: k_table_build solves every table entry (one per lane, lanes of a
// wave on consecutive angles of one mirror side, so they run the same layer
// loop); the trace kernels then interpolate (gwg_table.h).
//
// Backward, for a forward that stored adjoint entries:
//   1. k_absmax: the largest |dL/dI| (completes the fixed-point scale);
//   2. k_table_accum: per work item, the entries' dL/dI-scaled cotangents
//      are summed per (kappa, mirror, side, branch) key as in the memoized
//      adjoint, and each key's sums go to its four table entries (an item
//      with too many keys sends every entry on its own);
//   3. k_trace_bwd regenerates the items whose entry regions overflowed and
//      sends their cotangents to the accumulators the same way;
//   4. k_table_adj: one workgroup per (design, wavelength, mirror, side,
//      branch) runs one thin-film adjoint per table entry with a nonzero
//      cotangent into its LDS row;
//   5. k_table_reduce sums the rows over wavelengths, sides and branches in
//      a fixed order.
// Integer accumulation and fixed-order sums make the gradient bit-identical
// from run to run.

template <int MODE>
__global__ void __launch_bounds__(256) k_table_build(SceneDev sc, double* __restrict__ tab, int chunks,
                                                   unsigned long long* __restrict__ stats)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int WG = blockDim.x;
    const SmemLayout lay = smem_layout(sc.M, sc.Lmax, sc.n_slots, WG, sc.bins_x * sc.bins_y, false, 0,
                                       LaneSlots3::kPer, true);
    PointLds* pl = (PointLds*)(smem + lay.off_pl);
    LayerRec* s_rec = (LayerRec*)(smem + lay.off_thk);
    double* s_sp = (double*)(smem + lay.off_sp);
    const int tid = threadIdx.x;
    const LaneSlots3 sl = { slot_lane_base(s_sp, sc.n_slots, LaneSlots3::kPer, tid), pl->nsq, pl->pxy };
    const int64_t dl = blockIdx.x / chunks;
    const int chunk = blockIdx.x % chunks;
    const int d = (int)(dl / sc.n_lsel), l = (int)(dl % sc.n_lsel);
    stage_point(sc, d, l, 0, pl, nullptr, nullptr, s_rec, LaneSlots3::kPer);
    __syncthreads();
    const int n = sc.table_n;
    const int64_t per = (int64_t)sc.M * 2 * n;
    double* out = tab + dl * per * 8;
    unsigned long long n_fp64 = 0, n_lay = 0;
    for (int64_t q = (int64_t)chunk * WG + tid; q < per; q += (int64_t)chunks * WG) {
        const int j = (int)(q % n);
        const int ms = (int)(q / n);
        const int m = ms >> 1;
        bool u64 = false;
        const Coef4 c = hit_solve<MODE>(sc, *pl, RecStacks{ s_rec, sc.Lmax }, sl, m, (ms & 1) == 0, table_kappa(pl->ng, j, n), &u64);
        double* o = out + q * 8;
        o[0] = c.rs.re; o[1] = c.rs.im; o[2] = c.rp.re; o[3] = c.rp.im;
        o[4] = c.ts.re; o[5] = c.ts.im; o[6] = c.tp.re; o[7] = c.tp.im;
        n_fp64 += u64 ? 1ull : 0ull;
        n_lay += (unsigned long long)pl->nlay[m];
    }
    if (n_fp64) atomicAdd(&stats[ST_FP64], n_fp64);
    if (n_lay) atomicAdd(&stats[ST_LAYERS], n_lay);
}

// Largest |x| (as the bit pattern of a nonnegative double) into *out.
__global__ void k_absmax(const double* __restrict__ x, int64_t n, unsigned long long* __restrict__ out)
{
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = fabs(x[i]);
        mx = a > mx ? a : mx;
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0 && mx > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(mx));
}

__global__ void __launch_bounds__(64 * kMemoWaves) k_table_accum(SceneDev sc, const double* __restrict__ dLdI,
                                                                 AdjStore st)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int B = sc.bins_x * sc.bins_y;
    unsigned char* mbase = smem;
    int* s_nkeys = (int*)(mbase + kMemoWaves * memo_wave_bytes());
    const int tid = threadIdx.x, wave = tid / 64, lane = wave_lane();
    const MemoLds mt = memo_table(mbase, wave);
    const MemoLds m0 = memo_table(mbase, 0);
    const double fx = table_fx_scale(sc);
    const int n = sc.table_n;

    for (int64_t item = blockIdx.x; item < sc.n_items; item += gridDim.x) {
        if (st.ovf[item] != 0) continue;
        int64_t point, i0, i1;
        int d, l, f;
        decode_item(sc, item, &point, &d, &l, &f, &i0, &i1);
        const double ng = sc.lam_tab[(int64_t)l * LT_STRIDE + LT_NG];
        long long* acc_dl = sc.tab_acc + ((int64_t)d * sc.n_lsel + l) * sc.M * 4 * n * 4;
        const double* g_bins = dLdI + point * B;
        const int32_t* cnt = st.cnt + item * st.waves;
        int total = 0;
        for (int w = 0; w < st.waves; ++w) total += cnt[w];
        const int per = (total + kMemoWaves - 1) / kMemoWaves;
        const int v0 = min(wave * per, total), v1 = min(v0 + per, total);
        __syncthreads();
        const int nk = memo_collect(sc, st, item, cnt, g_bins, v0, v1, mt);
        if (lane == 0) s_nkeys[wave] = nk;
        __syncthreads();
        if (wave == 0) {
            const int U = memo_merge(mbase, s_nkeys);
            if (U < 0) {
                // too many keys: every entry on its own
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
                            table_emit(acc_dl, n, ng, st.ent[e], Gs, Gp, (int)(meta & 1023), fx);
                        }
                    }
                }
            } else {
                for (int b = 0; b < U; b += 64) {
                    const int k = b + lane;
                    if (k < U) {
                        const cd Gs = mk(m0.gsum[k], m0.gsum[kMemoKeys + k]);
                        const cd Gp = mk(m0.gsum[2 * kMemoKeys + k], m0.gsum[3 * kMemoKeys + k]);
                        table_emit(acc_dl, n, ng, __longlong_as_double((long long)m0.kbits[k]), Gs, Gp, m0.kmeta[k],
                                   fx);
                    }
                }
            }
        }
    }
}

size_t table_accum_smem_bytes()
{
    return (size_t)(kMemoWaves * memo_wave_bytes() + 16);
}

// One workgroup (two waves) per (design, wavelength, mirror, side, branch):
// block b covers accumulators [b n, (b + 1) n) and writes partial row b.
template <bool LOSSLESS>
__global__ void __launch_bounds__(128, 2) k_table_adj(SceneDev sc, double* __restrict__ partial,
                                                 double* __restrict__ scratch,
                                                 unsigned long long* __restrict__ stats)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int WG = blockDim.x;
    const int n_waves = WG / 64;
    const SmemLayout lay = smem_layout(sc.M, sc.Lmax, sc.n_slots, WG, sc.bins_x * sc.bins_y, false, n_waves);
    PointLds* pl = (PointLds*)(smem + lay.off_pl);
    double* s_thk = (double*)(smem + lay.off_thk);
    uint8_t* s_slot = (uint8_t*)(smem + lay.off_slot);
    double* s_sp = (double*)(smem + lay.off_sp);
    double* s_grad = (double*)(smem + lay.off_grad);
    int* s_list = (int*)(smem + lay.total);
    const int tid = threadIdx.x, wave = tid / 64, lane = wave_lane();
    const int ML = sc.M * sc.Lmax;
    double* gw = s_grad + (int64_t)wave * ML;
    int* lst = s_list + wave * 128;
    const LaneSlots3 sl = { slot_lane_base(s_sp, sc.n_slots, LaneSlots3::kPer, tid), pl->nsq, pl->pxy };
    double* chk = scratch + (int64_t)blockIdx.x * WG + tid;
    const int64_t cstride = (int64_t)gridDim.x * WG;
    const int64_t b = blockIdx.x;
    const int sb = (int)(b % 4);
    const int m = (int)((b / 4) % sc.M);
    const int64_t dl = b / 4 / sc.M;
    const int d = (int)(dl / sc.n_lsel), l = (int)(dl % sc.n_lsel);
    stage_point(sc, d, l, 0, pl, s_thk, s_slot);
    for (int k = tid; k < n_waves * ML; k += WG) s_grad[k] = 0.0;
    __syncthreads();
    const int n = sc.table_n;
    const long long* acc = sc.tab_acc + b * (int64_t)n * 4;
    const double inv = 1.0 / table_fx_scale(sc);
    const int meta = m | ((sb >> 1) == 0 ? 1 << 8 : 0) | ((sb & 1) << 9);
    unsigned long long c_keys = 0, c_lay = 0;
    auto run = [&](int j) {
        const long long* a = acc + (int64_t)j * 4;
        const cd Gs = mk((double)a[0] * inv, (double)a[1] * inv);
        const cd Gp = mk((double)a[2] * inv, (double)a[3] * inv);
        adjoint_hit<LOSSLESS>(sc, *pl, s_thk, s_slot, sl, gw, table_kappa(pl->ng, j, n), Gs, Gp, meta, chk, cstride);
        c_keys += 1;
        c_lay += (unsigned long long)pl->nlay[m];
    };
    // wave w: a contiguous part of the entries; nonzero ones are compacted
    // into the wave's LDS list and run 64 at a time
    const int per = (n + n_waves - 1) / n_waves;
    const int jb = min(wave * per, n), je = min(jb + per, n);
    int cntl = 0;                                        // wave-uniform list length (< 64 between chunks)
    for (int j0 = jb; j0 < je; j0 += 64) {
        const int j = j0 + lane;
        bool nz = false;
        if (j < je) {
            const long long* a = acc + (int64_t)j * 4;
            nz = (a[0] | a[1] | a[2] | a[3]) != 0;
        }
        const unsigned long long bal = __ballot(nz);
        const int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (nz) lst[cntl + pre] = j;
        cntl += __popcll(bal);
        wave_lds_sync();
        if (cntl >= 64) {
            const int mine = lst[lane];
            const int rem = cntl - 64;
            const int moved = lane < rem ? lst[64 + lane] : 0;
            wave_lds_sync();
            if (lane < rem) lst[lane] = moved;
            wave_lds_sync();
            cntl = rem;
            run(mine);
        }
    }
    if (cntl > 0) {
        const int mine = lane < cntl ? lst[lane] : -1;
        if (mine >= 0) run(mine);
    }
    __syncthreads();
    double* out = partial + b * (int64_t)sc.Lmax;
    for (int k = tid; k < sc.Lmax; k += WG) {
        double s = 0.0;
        for (int w = 0; w < n_waves; ++w) s += s_grad[(int64_t)w * ML + m * sc.Lmax + k];
        out[k] = s;
    }
    if (c_keys) atomicAdd(&stats[ST_ADJ_HITS], c_keys);
    if (c_lay) atomicAdd(&stats[ST_ADJ_LAYERS], c_lay);
}

int64_t table_adj_blocks(const SceneDev& sc)
{
    return (int64_t)sc.D * sc.n_lsel * sc.M * 4;
}

size_t table_adj_smem_bytes(const SceneDev& sc)
{
    return (size_t)smem_layout(sc.M, sc.Lmax, sc.n_slots, 128, sc.bins_x * sc.bins_y, false, 2).total + 2 * 128 * 4;
}

// grad[d][m][k] = sum over wavelengths, sides and branches (in that order) of
// the partial rows; zero beyond the mirror's layer count.
__global__ void k_table_reduce(const double* __restrict__ partial, int D, int n_lsel, int M, int Lmax,
                               const int32_t* __restrict__ nlay, double* __restrict__ grad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)D * M * Lmax) return;
    const int k = (int)(i % Lmax);
    const int m = (int)((i / Lmax) % M);
    const int d = (int)(i / Lmax / M);
    double s = 0.0;
    if (k < nlay[(int64_t)d * M + m])
        for (int l = 0; l < n_lsel; ++l)
            for (int sb = 0; sb < 4; ++sb)
                s += partial[((((int64_t)d * n_lsel + l) * M + m) * 4 + sb) * Lmax + k];
    grad[i] = s;
}
