// Angle-table thin film: device helpers.  Included by gwg_kernels.hip inside
// namespace gwg, before the trace kernels.
//
// (Methods, memory-saving strategies) The thin-film response of every
// (design, wavelength, mirror, side) is precomputed at n incidence angles
// theta_j = j (pi/2)/(n-1) in the glass and interpolated in between with a
// Catmull-Rom cubic in theta through the four surrounding angles.  The
// response depends on kappa^2 only, so it is even in theta and the angle
// before theta_0 is theta_1; the last segment repeats theta_{n-1}.
//
// A hit's coefficients are a fixed linear combination of four table entries,
// so the thin-film part of the gradient is the entries' own adjoints with the
// hits' cotangents summed per entry under the same weights.  The backward
// sums them in fixed point (int64 atomics: exact and independent of order)
// at a scale that bounds every sum below 2^62, then runs one thin-film
// adjoint per table entry with a nonzero cotangent.
//
// Table layout: tab[(((d n_lsel + l) M + m) 2 + side) n + j][8] with side 0
// = front, fields r_s, r_p, t_s, t_p as (re, im).  Cotangent accumulators:
// acc[((((d n_lsel + l) M + m) 2 + side) 2 + branch) n + j][4] with branch 1
// = reflected, fields G_s, G_p as (re, im).

constexpr double kHalfPi = 1.5707963267948966;

struct TabW {
    int j[4];
    double w[4];
};

// Table entries and weights of the hit angle with kappa = n_g sin(theta).
__device__ inline TabW table_weights(double kappa, double ng, int n)
{
    const double sn = kappa / ng;
    const double theta = asin(sn < 1.0 ? sn : 1.0);
    double x = theta / (kHalfPi / (double)(n - 1));
    if (!(x > 0.0)) x = 0.0;                     // also keeps a NaN angle inside the table
    if (x > (double)(n - 1)) x = (double)(n - 1);
    int j = (int)floor(x);
    j = j > n - 2 ? n - 2 : j;
    const double t = x - (double)j;
    const double t2 = t * t, t3 = t2 * t;
    TabW r;
    r.w[0] = 0.5 * (-t3 + 2.0 * t2 - t);
    r.w[1] = 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);
    r.w[2] = 0.5 * (-3.0 * t3 + 4.0 * t2 + t);
    r.w[3] = 0.5 * (t3 - t2);
    r.j[0] = j == 0 ? 1 : j - 1;
    r.j[1] = j;
    r.j[2] = j + 1;
    r.j[3] = j + 2 < n ? j + 2 : n - 1;
    return r;
}

// Table angle j's kappa.
__device__ inline double table_kappa(double ng, int j, int n)
{
    return ng * sin((double)j * (kHalfPi / (double)(n - 1)));
}

// Interpolated coefficients; tab_dl: the (design, wavelength) block.
__device__ inline Coef4 table_coef(const double* tab_dl, int n, int m, bool front, double kappa, double ng)
{
    const TabW tw = table_weights(kappa, ng, n);
    const double* b = tab_dl + (int64_t)(m * 2 + (front ? 0 : 1)) * n * 8;
    double a[8];
    for (int f = 0; f < 8; ++f) a[f] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double* e = b + (int64_t)tw.j[i] * 8;
#pragma unroll
        for (int f = 0; f < 8; ++f) a[f] += tw.w[i] * e[f];
    }
    Coef4 c;
    c.rs = mk(a[0], a[1]);
    c.rp = mk(a[2], a[3]);
    c.ts = mk(a[4], a[5]);
    c.tp = mk(a[6], a[7]);
    return c;
}

// Coefficients of a hit from the table block of its point: kappa from the
// direction exactly as the geometry walk computes it.
struct TabCoef {
    const double* tab;
    int tn;
    double ng, nx, nz;
    static constexpr bool kStoredBranch = false;
    __device__ bool refl(int) const { return false; }
    __device__ Coef4 operator()(int, double dx, double dy, double dz, int m, bool front) const
    {
        double c3[3];
        cross3(dx, dy, dz, nx, 0.0, nz, c3);
        const double kappa = ng * sqrt(c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
        return table_coef(tab, tn, m, front, kappa, ng);
    }
};

// Fixed-point scale of the cotangent accumulators.  The forward records the
// largest cotangent component (maxG, unscaled) and the number of cotangent
// pairs (n_e) of the rays that reached the eyebox; the backward the largest
// |dL/dI| (maxD).  A sum over any set of hits, with weights of magnitude at
// most 2 per entry, is then below B = 2 maxG maxD / N n_e, and the scale
// 2^(62 - e) with B < 2^e keeps every accumulator below 2^62.
__device__ inline double table_fx_scale(const SceneDev& sc)
{
    const double maxG = __longlong_as_double((long long)sc.tab_scale[0]);
    const double ne = (double)sc.tab_scale[1];
    const double maxD = __longlong_as_double((long long)sc.tab_scale[2]);
    const double B = 2.0 * maxG * maxD / (double)sc.N * (ne > 1.0 ? ne : 1.0);
    if (!(B > 0.0) || !(B < 1e300)) return 1.0;
    int e;
    (void)frexp(B, &e);
    return ldexp(1.0, 62 - e);
}

__device__ inline void fx_add(long long* a, double v)
{
    const long long q = (long long)rint(v);
    if (q != 0) atomicAdd((unsigned long long*)a, (unsigned long long)q);
}

// Adds one hit's (or one key's) dL/dI-scaled cotangents to the four table
// entries it interpolates from; acc_dl: the (design, wavelength) block,
// meta = mirror | front << 8 | reflected << 9, fx: the fixed-point scale.
__device__ inline void table_emit(long long* acc_dl, int n, double ng, double kappa, cd Gs, cd Gp, int meta,
                                  double fx)
{
    const TabW tw = table_weights(kappa, ng, n);
    const int m = meta & 255, side = ((meta >> 8) & 1) ? 0 : 1, br = (meta >> 9) & 1;
    long long* b = acc_dl + (int64_t)((m * 2 + side) * 2 + br) * n * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        long long* a = b + (int64_t)tw.j[i] * 4;
        const double v = tw.w[i] * fx;
        fx_add(a + 0, Gs.re * v);
        fx_add(a + 1, Gs.im * v);
        fx_add(a + 2, Gp.re * v);
        fx_add(a + 3, Gp.im * v);
    }
}

// Emits the entries of one regenerated ray into the accumulators.
struct TableEmit {
    long long* acc_dl;
    int n;
    double ng, gscale, fx;
    __device__ void operator()(double kappa, cd Gs, cd Gp, int meta) const
    {
        table_emit(acc_dl, n, ng, kappa, cscale(Gs, gscale), cscale(Gp, gscale), meta, fx);
    }
};

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}
