// Learned reflection probabilities: score-function gradient.  Included by
// gwg_kernels.hip inside namespace gwg.
//
// (Methods, learned reflection probabilities) Before the thicknesses are
// optimised, the mirrors' reflection probabilities omega are optimised with
// every coating idealised as a scalar reflectance equal to omega, tracing
// geometry only.  A sampled branch then carries weight one and a ray adds 1/N
// to the bin it reaches, so the scalar irradiance is the bin count over N.
// For J = sum over points and bins of W * I (W: per-bin weights, e.g. 1 for
// the throughput or dL/dI of Eq. 1 at the scalar irradiance), the path
// probability prod(omega or 1 - omega) gives the score-function gradient
//     dJ/domega_m = sum_points 1/N sum_rays (W_bin - beta) S_m,
//     S_m = sum over the ray's hits on mirror m of
//           (reflected ? 1/omega_m : -1/(1 - omega_m)),
// unbiased for any per-point constant beta because E[S_m] = 0; beta is the
// point's own J from the forward's counts.  omega_m is the probability the
// sampling uses, thr_m / 2^32.  A ray that leaves the eyebox has W = 0.
//
// Same paths as the last forward (same items, seeds and decisions).  Each
// wave reduces its rays' contributions in a fixed butterfly order, the waves'
// sums are added in order per item, and the items in order afterwards: the
// gradient is deterministic.

struct ScoreHit {
    double* s;            // this lane's S_m at s[m * ls]
    int ls;
    const double* inc;    // [2 M]: 1/omega_m, -1/(1 - omega_m)
    __device__ void operator()(int, double, int) const {}
    __device__ void branch(int m, bool refl) const { s[m * ls] += inc[2 * m + (refl ? 0 : 1)]; }
};

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256) k_omega_grad(SceneDev sc, const double* __restrict__ W,
                                                  const uint32_t* __restrict__ counts, double* __restrict__ partial)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int WG = blockDim.x, n_waves = WG / 64;
    const int B = sc.bins_x * sc.bins_y, M = sc.M;
    const SmemLayout lay = smem_layout(sc.M, sc.Lmax, sc.n_slots, WG, B, false, 0);
    PointLds* pl = (PointLds*)(smem + lay.off_pl);
    double* s_thk = (double*)(smem + lay.off_thk);
    uint8_t* s_slot = (uint8_t*)(smem + lay.off_slot);
    double* s_S = (double*)(smem + lay.total);                // [M][WG]
    double* s_inc = s_S + (int64_t)M * WG;                     // [2 M]
    double* s_acc = s_inc + 2 * M;                             // [n_waves][M]
    double* s_red = s_acc + (int64_t)n_waves * M;              // [WG] baseline reduction
    const int tid = threadIdx.x, wave = tid / 64, lane = wave_lane();
    const ScoreHit score = { s_S + tid, WG, s_inc };
    const double invN = 1.0 / (double)sc.N;

    for (int64_t item = blockIdx.x; item < sc.n_items; item += gridDim.x) {
        int64_t point, i0, i1;
        int d, l, f;
        decode_item(sc, item, &point, &d, &l, &f, &i0, &i1);
        __syncthreads();
        stage_point(sc, d, l, f, pl, s_thk, s_slot);
        const double* Wp = W + point * B;
        const uint32_t* cp = counts + point * B;
        // the point's J (baseline): strided partial sums, then a fixed tree
        double part = 0.0;
        for (int b = tid; b < B; b += WG) part += Wp[b] * (double)cp[b];
        s_red[tid] = part;
        for (int k = tid; k < n_waves * M; k += WG) s_acc[k] = 0.0;
        __syncthreads();
        if (tid < 2 * M) {
            const int m = tid >> 1;
            const double p = (double)pl->thr[m] * (1.0 / 4294967296.0);
            s_inc[tid] = (tid & 1) ? -1.0 / (1.0 - p) : (p > 0.0 ? 1.0 / p : 0.0);
        }
        for (int w = WG / 2; w > 0; w >>= 1) {
            if (tid < w) s_red[tid] += s_red[tid + w];
            __syncthreads();
        }
        const double beta = s_red[0] * invN;
        const int64_t base = point * sc.N;
        for (int64_t round = 0;; ++round) {
            const int64_t first = i0 + (int64_t)wave * 64 + round * WG;
            if (first >= i1) break;                            // uniform across the wave
            const int64_t i = first + lane;
            for (int m = 0; m < M; ++m) s_S[m * WG + tid] = 0.0;
            double fw = 0.0;
            if (i < i1) {
                Ray r;
                Outcome o;
                TapeRef none = { nullptr, nullptr, 0 };
                ray_birth(sc, *pl, base + i, r);
                walk_ray<false, false>(sc, *pl, r, o, score, NoCoef{}, none, nullptr);
                fw = (o.cat == CAT_EYEBOX ? Wp[o.bin] : 0.0) - beta;
            }
            for (int m = 0; m < M; ++m) {
                const double c = wave_sum(i < i1 ? fw * s_S[m * WG + tid] : 0.0);
                if (lane == 0) s_acc[wave * M + m] += c;
            }
        }
        __syncthreads();
        if (tid < M) {
            double a = 0.0;
            for (int w = 0; w < n_waves; ++w) a += s_acc[w * M + tid];
            partial[item * M + tid] = a * invN;
        }
    }
}

size_t omega_smem_bytes(const SceneDev& sc, int wg)
{
    const int n_waves = wg / 64;
    return (size_t)smem_layout(sc.M, sc.Lmax, sc.n_slots, wg, sc.bins_x * sc.bins_y, false, 0).total +
           sizeof(double) * ((size_t)sc.M * wg + 2 * sc.M + (size_t)n_waves * sc.M + wg);
}

// grad[m] = sum over items, in item order, of partial[item][m].
__global__ void k_omega_reduce(const double* __restrict__ partial, int64_t n_items, int M, double* __restrict__ grad)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    double a = 0.0;
    for (int64_t it = 0; it < n_items; ++it) a += partial[it * M + m];
    grad[m] = a;
}
