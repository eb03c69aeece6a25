// Host side of the C ABI declared in include/gwg.h: argument validation,
// scene tables, device buffers owned by the context, kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "gwg.h"
#include "gwg_internal.h"
#include "gwg_launch.h"

using namespace gwg;

namespace {

// Device buffer owned by the context (grow-only).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= bytes && p) return hipSuccess;
        if (p) { hipError_t e = hipFree(p); if (e != hipSuccess) return e; p = nullptr; bytes = 0; }
        size_t want = std::max<size_t>(n, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release() { if (p) (void)hipFree(p); p = nullptr; bytes = 0; }
};

uint64_t fnv(uint64_t h, const void* data, size_t n)
{
    const unsigned char* b = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h;
}
template <typename T> uint64_t fnv_v(uint64_t h, const T& v) { return fnv(h, &v, sizeof(T)); }

bool is_fin(double x) { return std::isfinite(x); }

std::string g_create_error;

// Ring of begin/end event pairs around one kernel's launches.
struct KernelTimer {
    hipEvent_t ev[GWG_TIMING_RING][2] = {};
    int64_t recorded = 0;
    hipError_t create()
    {
        for (auto& p : ev)
            for (hipEvent_t& e : p)
                if (!e) { hipError_t r = hipEventCreate(&e); if (r != hipSuccess) return r; }
        return hipSuccess;
    }
    void destroy()
    {
        for (auto& p : ev)
            for (hipEvent_t& e : p)
                if (e) { (void)hipEventDestroy(e); e = nullptr; }
        recorded = 0;
    }
    hipEvent_t begin() const { return ev[recorded % GWG_TIMING_RING][0]; }
    hipEvent_t end() const { return ev[recorded % GWG_TIMING_RING][1]; }
};

}  // namespace

// Adjoint entry capacity: entries per ray of a (work item, wave) region, and
// the most device memory the entries may take.
constexpr int64_t kAdjEntriesPerRay = 8;
constexpr double kAdjBudgetBytes = 96.0 * 1024 * 1024 * 1024;

// One built scene: its device tables and the SceneDev that points into them.
struct SceneEntry {
    uint64_t hash = 0;
    uint64_t last_use = 0;
    SceneDev sc{};
    DevBuf lam_tab, dir_tab, slot, nlay, pupil_xy;
    std::vector<int32_t> h_nlay;
    void release()
    {
        for (DevBuf* b : { &lam_tab, &dir_tab, &slot, &nlay, &pupil_xy }) b->release();
    }
};
// Scenes kept per context (least recently used evicted), so that calls
// that alternate between a few scenes (a batch traced in chunks of designs)
// rebuild nothing, and can be captured in one graph once each was built.
constexpr int kSceneCache = 128;

struct gwg_ctx {
    int device = -1;
    int n_cu = 0;
    std::string err;
    // scene tables: the current scene (a copy of its cache entry's) and the cache
    uint64_t scene_hash = 0;
    bool scene_valid = false;
    SceneDev sc{};
    std::vector<int32_t> h_nlay;
    std::vector<std::unique_ptr<SceneEntry>> scenes;
    uint64_t scene_clock = 0;
    // per-call buffers
    DevBuf stats, partial, scratch, fwd_scratch, loss_work, grad_tmp;
    // thin-film queries
    DevBuf tmm_tab, tmm_slot;
    // last forward
    bool have_forward = false;
    SceneDev fwd{};
    // adjoint entries recorded by the last forward (GWG_FWD_GRAD)
    DevBuf adj_ent, adj_cnt, adj_ovf, fwd_tape, adj_ck, adj_order;
    // per-(item, wave) mirror hits of the last forward, and the order the
    // next forward of the same decomposition takes its items in
    DevBuf item_work, fwd_order;
    int64_t work_items = -1;
    int work_waves = 0;
    bool adj_valid = false;
    bool memo = false;           // thin-film adjoints per distinct hit key (GWG_FWD_MEMO)
    AdjStore adj{};
    // angle table (GWG_FWD_TABLE): entries, fixed-point bound, backward accumulators
    DevBuf tab, tab_scale, tab_acc;
    bool tab_grad = false;       // the last forward was a table forward with GWG_FWD_GRAD
    // tuning
    gwg_tuning tune{};
    // kernel timing
    bool timing = false;
    KernelTimer timer[2];
    // optional device step counter read by the trace kernels
    const uint32_t* step_dev = nullptr;
    // occupancy queries, keyed by (kind, precision, block, LDS bytes)
    std::map<std::tuple<int, int, int, size_t>, int> occ;
    // autotuned launch parameters by scene signature, and scratch outputs
    std::map<uint64_t, gwg_tuning> tuned;
    DevBuf tune_q, tune_c, tune_g, tune_grad;
};

namespace {

int fail(gwg_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(gwg_ctx* c, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_error = buf;
    return code;
}

int hip_fail(gwg_ctx* c, hipError_t e, const char* what)
{
    return fail(c, GWG_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_CHECK(ctx, call, what)                          \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}

// Grow a context buffer; during stream capture nothing may be allocated.
int ensure_buf(gwg_ctx* c, DevBuf& b, size_t n, bool capturing, const char* what)
{
    if (b.p && n <= b.bytes) return GWG_OK;
    if (capturing)
        return fail(c, GWG_E_STATE, "%s would allocate during stream capture; make the same call once before capturing", what);
    HIP_CHECK(c, b.ensure(n), what);
    return GWG_OK;
}

int occupancy(gwg_ctx* c, int kind, int precision, int wg, size_t smem)
{
    const auto key = std::make_tuple(kind, precision, wg, smem);
    auto it = c->occ.find(key);
    if (it != c->occ.end()) return it->second;
    const int n = trace_blocks_per_cu(kind, precision, wg, smem);
    c->occ[key] = n;
    return n;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) { (void)hipGetDevice(&prev); if (prev != dev) (void)hipSetDevice(dev); }
    ~DeviceGuard() { int cur = -1; (void)hipGetDevice(&cur); if (prev >= 0 && cur != prev) (void)hipSetDevice(prev); }
};

// ------------------------------------------------------------ validation
int check_materials(gwg_ctx* c, const gwg_materials* m)
{
    if (!m) return fail(c, GWG_E_INVAL, "materials is NULL");
    if (m->n_lambda < 1 || m->n_lambda > 4096) return fail(c, GWG_E_INVAL, "n_lambda %d out of range", m->n_lambda);
    if (m->n_mat < 1 || m->n_mat > 255) return fail(c, GWG_E_INVAL, "n_mat %d out of range", m->n_mat);
    if (!m->lambda_nm || !m->n_re || !m->n_im) return fail(c, GWG_E_INVAL, "material table pointer is NULL");
    for (int i = 0; i < m->n_lambda; ++i)
        if (!is_fin(m->lambda_nm[i]) || m->lambda_nm[i] <= 0.0) return fail(c, GWG_E_INVAL, "lambda_nm[%d] invalid", i);
    for (int i = 0; i < m->n_lambda * m->n_mat; ++i) {
        if (!is_fin(m->n_re[i]) || m->n_re[i] <= 0.0) return fail(c, GWG_E_INVAL, "n_re[%d] invalid", i);
        if (!is_fin(m->n_im[i]) || m->n_im[i] < 0.0) return fail(c, GWG_E_INVAL, "n_im[%d] invalid", i);
    }
    return GWG_OK;
}

bool lossless(const gwg_materials* m, int mat)
{
    for (int l = 0; l < m->n_lambda; ++l)
        if (m->n_im[l * m->n_mat + mat] != 0.0) return false;
    return true;
}

int check_scene(gwg_ctx* c, const gwg_slab* sl, const gwg_prma* pr, const gwg_materials* mt,
                const gwg_stacks* st, const gwg_rays* ry)
{
    int rc = check_materials(c, mt);
    if (rc) return rc;
    if (!sl || !pr || !st || !ry) return fail(c, GWG_E_INVAL, "NULL scene argument");
    if (!(is_fin(sl->T_mm) && sl->T_mm > 0 && is_fin(sl->L_mm) && sl->L_mm > 0 && is_fin(sl->eye_relief_mm) &&
          sl->eye_relief_mm >= 0))
        return fail(c, GWG_E_INVAL, "slab dimensions invalid");
    if (sl->mat_glass < 0 || sl->mat_glass >= mt->n_mat || sl->mat_air < 0 || sl->mat_air >= mt->n_mat)
        return fail(c, GWG_E_INVAL, "slab material index out of range");
    if (!lossless(mt, sl->mat_glass) || !lossless(mt, sl->mat_air))
        return fail(c, GWG_E_INVAL, "slab glass and air must be lossless");
    if (!(is_fin(sl->pupil_x0_mm) && is_fin(sl->pupil_w_mm) && sl->pupil_w_mm >= 0 && is_fin(sl->pupil_h_mm) &&
          sl->pupil_h_mm >= 0))
        return fail(c, GWG_E_INVAL, "pupil window invalid");
    if (!(is_fin(sl->eye_x0_mm) && is_fin(sl->eye_y0_mm) && is_fin(sl->eye_w_mm) && sl->eye_w_mm > 0 &&
          is_fin(sl->eye_h_mm) && sl->eye_h_mm > 0))
        return fail(c, GWG_E_INVAL, "eyebox rectangle invalid");
    if (sl->bins_x < 1 || sl->bins_x > 4096 || sl->bins_y < 1 || sl->bins_y > 4096)
        return fail(c, GWG_E_INVAL, "bins %d x %d out of range", sl->bins_x, sl->bins_y);
    if (sl->n_eye_pupils < 0 || sl->n_eye_pupils > kMaxPupils)
        return fail(c, GWG_E_INVAL, "n_eye_pupils %d out of range 0..%d", sl->n_eye_pupils, kMaxPupils);
    if (sl->n_eye_pupils > 0) {
        const int np = sl->n_eye_pupils;
        const double r = sl->eye_pupil_radius_mm;
        if (!(is_fin(r) && r > 0.0)) return fail(c, GWG_E_INVAL, "eye pupil radius must be finite and > 0");
        if (!sl->eye_pupil_xy_mm) return fail(c, GWG_E_INVAL, "eye_pupil_xy_mm is NULL");
        if (sl->bins_x != np || sl->bins_y != 1)
            return fail(c, GWG_E_INVAL, "with %d eye pupils bins must be %d x 1, not %d x %d", np, np, sl->bins_x,
                        sl->bins_y);
        const double* xy = sl->eye_pupil_xy_mm;
        for (int p = 0; p < 2 * np; ++p)
            if (!is_fin(xy[p])) return fail(c, GWG_E_INVAL, "eye pupil centre %d is not finite", p / 2);
        for (int p = 0; p < np; ++p)
            for (int q = p + 1; q < np; ++q) {
                const double dx = xy[2 * p] - xy[2 * q], dy = xy[2 * p + 1] - xy[2 * q + 1];
                if (dx * dx + dy * dy < 4.0 * r * r)
                    return fail(c, GWG_E_INVAL, "eye pupils %d and %d overlap", p, q);
            }
    }
    if (pr->n_mirrors < 1 || pr->n_mirrors > kMaxMirrors) return fail(c, GWG_E_INVAL, "n_mirrors %d out of range", pr->n_mirrors);
    if (!pr->omega) return fail(c, GWG_E_INVAL, "omega is NULL");
    for (int m = 0; m < pr->n_mirrors; ++m)
        if (!(is_fin(pr->omega[m]) && pr->omega[m] > 0.0 && pr->omega[m] < 1.0))
            return fail(c, GWG_E_INVAL, "omega[%d] must be in (0, 1)", m);
    if (!(is_fin(pr->tilt_deg) && pr->tilt_deg > 0.0 && pr->tilt_deg < 90.0)) return fail(c, GWG_E_INVAL, "tilt_deg invalid");
    if (!(is_fin(pr->pitch_mm) && is_fin(pr->center_x_mm))) return fail(c, GWG_E_INVAL, "mirror placement invalid");
    if (st->n_designs < 1 || st->n_mirrors != pr->n_mirrors) return fail(c, GWG_E_INVAL, "stacks shape mismatch");
    if (st->max_layers < 1 || st->max_layers > kMaxLayers) return fail(c, GWG_E_INVAL, "max_layers %d out of range", st->max_layers);
    if (!st->thk_nm || !st->mat || !st->n_layers) return fail(c, GWG_E_INVAL, "stack pointer is NULL");
    int64_t DM = (int64_t)st->n_designs * st->n_mirrors;
    for (int64_t k = 0; k < DM; ++k) {
        int nl = st->n_layers[k];
        if (nl < 0 || nl > st->max_layers) return fail(c, GWG_E_INVAL, "n_layers[%lld] = %d out of range", (long long)k, nl);
        for (int j = 0; j < nl; ++j) {
            int mm = st->mat[k * st->max_layers + j];
            if (mm >= mt->n_mat) return fail(c, GWG_E_INVAL, "layer material %d out of range", mm);
        }
    }
    if (ry->n_lambda_sel < 1 || !ry->lambda_sel) return fail(c, GWG_E_INVAL, "no wavelength selected");
    for (int i = 0; i < ry->n_lambda_sel; ++i)
        if (ry->lambda_sel[i] < 0 || ry->lambda_sel[i] >= mt->n_lambda) return fail(c, GWG_E_INVAL, "lambda_sel[%d] out of range", i);
    if (ry->fov_mode != 0 && ry->fov_mode != 1) return fail(c, GWG_E_INVAL, "fov_mode must be 0 or 1");
    if (!ry->fov_deg) return fail(c, GWG_E_INVAL, "fov_deg is NULL");
    if (ry->fov_mode == 0) {
        if (ry->n_fov < 1) return fail(c, GWG_E_INVAL, "n_fov must be >= 1");
        for (int i = 0; i < 2 * ry->n_fov; ++i)
            if (!(is_fin(ry->fov_deg[i]) && std::fabs(ry->fov_deg[i]) < 60.0)) return fail(c, GWG_E_INVAL, "fov_deg[%d] invalid", i);
    } else {
        if (ry->n_fov != 1) return fail(c, GWG_E_INVAL, "fov_mode 1 requires n_fov == 1");
        for (int i = 0; i < 4; ++i)
            if (!(is_fin(ry->fov_deg[i]) && std::fabs(ry->fov_deg[i]) < 60.0)) return fail(c, GWG_E_INVAL, "fov bound %d invalid", i);
    }
    if (ry->rays_per_point < 1 || ry->rays_per_point > (int64_t(1) << 40)) return fail(c, GWG_E_INVAL, "rays_per_point out of range");
    if (ry->max_events < 1 || ry->max_events > kMaxEvents) return fail(c, GWG_E_INVAL, "max_events out of range");
    if (ry->first_design < 0) return fail(c, GWG_E_INVAL, "first_design must be >= 0");
    {
        const double F = ry->fov_mode == 0 ? (double)ry->n_fov : 1.0;
        const double ids = ((double)ry->first_design + (double)st->n_designs) * ry->n_lambda_sel * F *
                           (double)ry->rays_per_point;
        if (ids > 4.0e18) return fail(c, GWG_E_INVAL, "ray ids of the batch exceed 2^62");
    }
    return GWG_OK;
}

// Guided direction of field angles (thx, thy) in degrees (same operation
// sequence as the device, so the grid table and per-ray directions agree).
void field_direction_host(double thx, double thy, double ng, double nx, double nz, double* d)
{
    double tx = std::tan(thx * (3.14159265358979323846 / 180.0));
    double ty = std::tan(thy * (3.14159265358979323846 / 180.0));
    double inv = 1.0 / std::sqrt(tx * tx + ty * ty + 1.0);
    double ax = tx * inv, ay = ty * inv;
    double gx = ax / ng, gy = ay / ng, gz = std::sqrt(1.0 - (ax * ax + ay * ay) / (ng * ng));
    double gn = nx * gx + nz * gz;
    double t2 = 2.0 * gn;
    d[0] = gx - t2 * nx;
    d[1] = gy;
    d[2] = gz - t2 * nz;
}

// Near-critical margin of the mixed-precision rule: 2 degrees around the
// critical angle glass -> slot material, as a kappa interval.
constexpr double kCritMarginDeg = 2.0;

void crit_interval(double ng, double ns, double nsi, double* lo, double* hi)
{
    *lo = 0.0; *hi = 0.0;
    if (nsi != 0.0 || ns >= ng) return;
    double th = std::asin(ns / ng);
    double m = kCritMarginDeg * (3.14159265358979323846 / 180.0);
    double a = th - m, b = th + m;
    if (b > 1.5707963267948966) b = 1.5707963267948966;
    *lo = ng * std::sin(a);
    *hi = ng * std::sin(b);
}

int build_scene(gwg_ctx* c, const gwg_slab* sl, const gwg_prma* pr, const gwg_materials* mt,
                const gwg_stacks* st, const gwg_rays* ry, hipStream_t stream)
{
    // content hash of everything the tables depend on
    uint64_t h = 1469598103934665603ull;
    h = fnv_v(h, *sl);
    if (sl->n_eye_pupils > 0) h = fnv(h, sl->eye_pupil_xy_mm, sizeof(double) * 2 * sl->n_eye_pupils);
    h = fnv_v(h, pr->n_mirrors); h = fnv_v(h, pr->tilt_deg); h = fnv_v(h, pr->pitch_mm); h = fnv_v(h, pr->center_x_mm);
    h = fnv(h, pr->omega, sizeof(double) * pr->n_mirrors);
    h = fnv_v(h, mt->n_lambda); h = fnv_v(h, mt->n_mat);
    h = fnv(h, mt->lambda_nm, sizeof(double) * mt->n_lambda);
    h = fnv(h, mt->n_re, sizeof(double) * mt->n_lambda * mt->n_mat);
    h = fnv(h, mt->n_im, sizeof(double) * mt->n_lambda * mt->n_mat);
    h = fnv_v(h, st->n_designs); h = fnv_v(h, st->n_mirrors); h = fnv_v(h, st->max_layers);
    int64_t DML = (int64_t)st->n_designs * st->n_mirrors * st->max_layers;
    h = fnv(h, st->mat, (size_t)DML);
    h = fnv(h, st->n_layers, sizeof(int32_t) * st->n_designs * st->n_mirrors);
    h = fnv_v(h, ry->n_lambda_sel);
    h = fnv(h, ry->lambda_sel, sizeof(int32_t) * ry->n_lambda_sel);
    h = fnv_v(h, ry->fov_mode); h = fnv_v(h, ry->n_fov);
    h = fnv(h, ry->fov_deg, sizeof(double) * (ry->fov_mode == 0 ? 2 * ry->n_fov : 4));
    h = fnv_v(h, ry->rays_per_point); h = fnv_v(h, ry->max_events); h = fnv_v(h, ry->first_design);
    if (c->scene_valid && h == c->scene_hash) return GWG_OK;
    for (auto& e : c->scenes)
        if (e->hash == h) {
            e->last_use = ++c->scene_clock;
            c->sc = e->sc;
            c->h_nlay = e->h_nlay;
            c->scene_hash = h;
            c->scene_valid = true;
            return GWG_OK;
        }
    if (stream_capturing(stream))
        return fail(c, GWG_E_STATE, "the scene changed during stream capture; make the same call once before capturing");
    c->scene_valid = false;
    // a cache entry for the new scene: a fresh one, or the least recently used
    SceneEntry* ent = nullptr;
    if ((int)c->scenes.size() < kSceneCache) {
        c->scenes.emplace_back(new SceneEntry());
        ent = c->scenes.back().get();
    } else {
        ent = c->scenes[0].get();
        for (auto& e : c->scenes)
            if (e->last_use < ent->last_use) ent = e.get();
    }
    ent->hash = 0;

    SceneDev& s = ent->sc;
    s = SceneDev{};
    s.T = sl->T_mm; s.Lx = sl->L_mm; s.ER = sl->eye_relief_mm;
    s.px0 = sl->pupil_x0_mm; s.pw = sl->pupil_w_mm; s.ph = sl->pupil_h_mm;
    s.ex0 = sl->eye_x0_mm; s.ey0 = sl->eye_y0_mm; s.ew = sl->eye_w_mm; s.eh = sl->eye_h_mm;
    s.bins_x = sl->bins_x; s.bins_y = sl->bins_y;
    s.n_pupils = sl->n_eye_pupils;
    s.pupil_r2 = s.n_pupils > 0 ? sl->eye_pupil_radius_mm * sl->eye_pupil_radius_mm : 0.0;
    s.M = pr->n_mirrors;
    double beta = pr->tilt_deg * (3.14159265358979323846 / 180.0);
    s.nx = -std::sin(beta);
    s.nz = std::cos(beta);
    for (int m = 0; m < s.M; ++m) {
        double xm = pr->center_x_mm + ((double)m - (double)(s.M - 1) * 0.5) * pr->pitch_mm;
        s.h[m] = s.nx * xm + s.nz * (sl->T_mm * 0.5);
        double t = std::floor(pr->omega[m] * 4294967296.0);
        t = std::min(std::max(t, 0.0), 4294967295.0);
        s.thr[m] = (uint32_t)t;
        double p = (double)s.thr[m] / 4294967296.0;
        if (!(p > 0.0 && p < 1.0)) return fail(c, GWG_E_INVAL, "omega[%d] rounds to 0 or 1", m);
        s.sc_r[m] = 1.0 / std::sqrt(p);
        s.sc_t[m] = 1.0 / std::sqrt(1.0 - p);
    }
    // compact material slots of the stacks
    std::map<int, int> slot_of;
    std::vector<int> mat_of_slot;
    std::vector<uint8_t> slots((size_t)DML, 0);
    int64_t DM = (int64_t)st->n_designs * st->n_mirrors;
    for (int64_t k = 0; k < DM; ++k)
        for (int j = 0; j < st->n_layers[k]; ++j) {
            int mm = st->mat[k * st->max_layers + j];
            auto it = slot_of.find(mm);
            if (it == slot_of.end()) {
                if ((int)mat_of_slot.size() == kMaxSlots)
                    return fail(c, GWG_E_INVAL, "more than %d distinct layer materials", kMaxSlots);
                it = slot_of.emplace(mm, (int)mat_of_slot.size()).first;
                mat_of_slot.push_back(mm);
            }
            slots[(size_t)(k * st->max_layers + j)] = (uint8_t)it->second;
        }
    if (mat_of_slot.empty()) mat_of_slot.push_back(sl->mat_glass);
    s.n_slots = (int)mat_of_slot.size();
    s.slot_complex = 0;
    for (int q = 0; q < s.n_slots; ++q)
        if (!lossless(mt, mat_of_slot[q])) s.slot_complex |= 1u << q;
    s.D = st->n_designs;
    s.Lmax = st->max_layers;
    // wavelength table
    s.n_lsel = ry->n_lambda_sel;
    std::vector<double> lt((size_t)s.n_lsel * LT_STRIDE, 0.0);
    for (int i = 0; i < s.n_lsel; ++i) {
        int l = ry->lambda_sel[i];
        double* row = &lt[(size_t)i * LT_STRIDE];
        row[LT_K0] = 2.0 * 3.14159265358979323846 / mt->lambda_nm[l];
        row[LT_NG] = mt->n_re[l * mt->n_mat + sl->mat_glass];
        row[LT_NA] = mt->n_re[l * mt->n_mat + sl->mat_air];
        for (int q = 0; q < s.n_slots; ++q) {
            double nr = mt->n_re[l * mt->n_mat + mat_of_slot[q]], ni = mt->n_im[l * mt->n_mat + mat_of_slot[q]];
            row[LT_SLOT + 2 * q] = nr;
            row[LT_SLOT + 2 * q + 1] = ni;
            crit_interval(row[LT_NG], nr, ni, &row[LT_CRIT + 2 * q], &row[LT_CRIT + 2 * q + 1]);
        }
        row[LT_NSLOT] = s.n_slots;
    }
    s.fov_mode = ry->fov_mode;
    s.F = ry->fov_mode == 0 ? ry->n_fov : 1;
    std::vector<double> dirs;
    if (s.fov_mode == 0) {
        dirs.assign((size_t)s.n_lsel * s.F * 4, 0.0);
        for (int i = 0; i < s.n_lsel; ++i)
            for (int f = 0; f < s.F; ++f)
                field_direction_host(ry->fov_deg[2 * f], ry->fov_deg[2 * f + 1], lt[(size_t)i * LT_STRIDE + LT_NG],
                                     s.nx, s.nz, &dirs[((size_t)i * s.F + f) * 4]);
    } else {
        s.fov_x0 = ry->fov_deg[0]; s.fov_x1 = ry->fov_deg[1];
        s.fov_y0 = ry->fov_deg[2]; s.fov_y1 = ry->fov_deg[3];
        dirs.assign(4, 0.0);
    }
    s.N = ry->rays_per_point;
    s.id_base = (int64_t)ry->first_design * s.n_lsel * s.F * s.N;
    s.Kmax = ry->max_events;
    // the entry may have been in use by the stream's earlier kernels
    HIP_CHECK(c, hipStreamSynchronize(stream), "scene rebuild");
    HIP_CHECK(c, ent->lam_tab.ensure(lt.size() * sizeof(double)), "alloc lam_tab");
    HIP_CHECK(c, ent->dir_tab.ensure(dirs.size() * sizeof(double)), "alloc dir_tab");
    HIP_CHECK(c, ent->slot.ensure(slots.size()), "alloc slot");
    HIP_CHECK(c, ent->nlay.ensure(sizeof(int32_t) * DM), "alloc nlay");
    HIP_CHECK(c, ent->pupil_xy.ensure(sizeof(double) * 2 * (size_t)std::max(s.n_pupils, 1)), "alloc pupil table");
    if (s.n_pupils > 0)
        HIP_CHECK(c, hipMemcpyAsync(ent->pupil_xy.p, sl->eye_pupil_xy_mm, sizeof(double) * 2 * s.n_pupils,
                                    hipMemcpyHostToDevice, stream), "upload pupil table");
    HIP_CHECK(c, hipMemcpyAsync(ent->lam_tab.p, lt.data(), lt.size() * sizeof(double), hipMemcpyHostToDevice, stream), "upload lam_tab");
    HIP_CHECK(c, hipMemcpyAsync(ent->dir_tab.p, dirs.data(), dirs.size() * sizeof(double), hipMemcpyHostToDevice, stream), "upload dir_tab");
    HIP_CHECK(c, hipMemcpyAsync(ent->slot.p, slots.data(), slots.size(), hipMemcpyHostToDevice, stream), "upload slots");
    HIP_CHECK(c, hipMemcpyAsync(ent->nlay.p, st->n_layers, sizeof(int32_t) * DM, hipMemcpyHostToDevice, stream), "upload n_layers");
    HIP_CHECK(c, hipStreamSynchronize(stream), "scene upload");
    s.lam_tab = (const double*)ent->lam_tab.p;
    s.dir_tab = (const double*)ent->dir_tab.p;
    s.slot = (const uint8_t*)ent->slot.p;
    s.nlay = (const int32_t*)ent->nlay.p;
    s.pupil_xy = (const double*)ent->pupil_xy.p;
    ent->h_nlay.assign(st->n_layers, st->n_layers + DM);
    ent->hash = h;
    ent->last_use = ++c->scene_clock;
    c->sc = s;
    c->h_nlay = ent->h_nlay;
    c->scene_hash = h;
    c->scene_valid = true;
    return GWG_OK;
}

int pick_fwd_wg(gwg_ctx* c, const SceneDev& s, bool lds_bins)
{
    if (c->tune.block_threads) return c->tune.block_threads;
    for (int wg : { 256, 128, 64 })
        if (fwd_smem_bytes(s, wg, lds_bins) <= 65536) return wg;
    return 64;
}

int pick_bwd_wg(gwg_ctx* c, const SceneDev& s)
{
    if (c->tune.bwd_block_threads) return c->tune.bwd_block_threads;
    for (int wg : { 128, 64 })
        if (bwd_smem_bytes(s, wg) <= 65536) return wg;
    return 64;
}

void set_tiles(SceneDev& s, int64_t rays_per_tile, int wg, int n_cu)
{
    const int64_t points = (int64_t)s.D * s.n_lsel * s.F;
    int64_t rpt = rays_per_tile;
    if (rpt <= 0) {
        // Whole points while there are at least ~32 per CU (about 16 items
        // per resident workgroup at two per CU, so the launch's tail, at
        // most about one item, costs little); otherwise split every point
        // into equal tiles of at least 4 rays per lane.  Memoized solves
        // share keys within an item, and take half as many, larger items.
        const int64_t target = (int64_t)std::max(n_cu, 1) * (s.memo ? 16 : 32);
        const int64_t tiles = points >= target ? 1 : (target + points - 1) / points;
        rpt = (s.N + tiles - 1) / tiles;
        rpt = std::max<int64_t>(rpt, (int64_t)wg * 4);
        rpt = ((rpt + wg - 1) / wg) * wg;
    }
    if (rpt > s.N) rpt = s.N;
    s.rays_per_tile = rpt;
    s.tiles_per_point = (s.N + rpt - 1) / rpt;
    s.n_items = points * s.tiles_per_point;
}

int read_stats(gwg_ctx* c, hipStream_t s, gwg_stats* stats)
{
    uint64_t w[ST_WORDS];
    HIP_CHECK(c, hipMemcpyAsync(w, c->stats.p, sizeof(w), hipMemcpyDeviceToHost, s), "read stats");
    HIP_CHECK(c, hipStreamSynchronize(s), "kernel execution");
    std::memset(stats, 0, sizeof(*stats));
    stats->rays = (int64_t)w[ST_RAYS];
    stats->interactions = (int64_t)w[ST_EVENTS];
    stats->prma_hits = (int64_t)w[ST_PRMA];
    stats->layer_steps = (int64_t)w[ST_LAYERS];
    stats->fp64_hits = (int64_t)w[ST_FP64];
    stats->saturated = (int64_t)w[ST_SAT];
    stats->adjoint_rays = (int64_t)w[ST_ADJ_RAYS];
    stats->adjoint_hits = (int64_t)w[ST_ADJ_HITS];
    stats->adjoint_layer_steps = (int64_t)w[ST_ADJ_LAYERS];
    stats->adjoint_stored_layer_steps = (int64_t)w[ST_ADJ_STORED];
    for (int k = 0; k < GWG_NCAT; ++k) {
        stats->n_cat[k] = (int64_t)w[ST_CAT + k];
        stats->power[k] = (double)w[ST_POW + k] / 16777216.0;
    }
    return GWG_OK;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

int32_t gwg_abi_version(void) { return GWG_ABI_VERSION; }

#ifndef GWG_SOURCE_HASH
#error "GWG_SOURCE_HASH must be defined by the build (hash of the library's sources)"
#endif
const char* gwg_source_hash(void) { return GWG_SOURCE_HASH; }

int gwg_create(gwg_ctx** out, int32_t device)
{
    if (!out) return fail(nullptr, GWG_E_INVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(nullptr, GWG_E_NODEVICE, "no HIP device");
    if (device < 0 || device >= n) return fail(nullptr, GWG_E_NODEVICE, "device %d does not exist", device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(nullptr, GWG_E_NODEVICE, "device query failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, GWG_E_NODEVICE, "device %d is %s, not gfx950", device, prop.gcnArchName);
    {
        // the allocation-free loss's scratch address on this device
        DeviceGuard g(device);
        const hipError_t e = loss_scratch_setup(device);
        if (e != hipSuccess)
            return fail(nullptr, GWG_E_HIP, "scratch symbol lookup on device %d: %s", device, hipGetErrorString(e));
    }
    gwg_ctx* c = new gwg_ctx();
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    *out = c;
    return GWG_OK;
}

int gwg_destroy(gwg_ctx* c)
{
    if (!c) return GWG_E_INVAL;
    {
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        for (auto& e : c->scenes) e->release();
        for (DevBuf* b : { &c->stats, &c->partial, &c->scratch, &c->fwd_scratch,
                           &c->loss_work, &c->tmm_tab, &c->tmm_slot, &c->adj_ent, &c->adj_cnt, &c->adj_ovf, &c->fwd_tape,
                           &c->tab, &c->tab_scale, &c->tab_acc, &c->tune_q, &c->tune_c, &c->tune_g, &c->tune_grad,
                           &c->adj_ck, &c->grad_tmp, &c->adj_order, &c->item_work, &c->fwd_order })
            b->release();
        for (KernelTimer& t : c->timer) t.destroy();
    }
    delete c;
    return GWG_OK;
}

const char* gwg_last_error(const gwg_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int gwg_set_tuning(gwg_ctx* c, const gwg_tuning* t)
{
    if (!c || !t) return GWG_E_INVAL;
    for (int wg : { t->block_threads, t->bwd_block_threads })
        if (wg != 0 && wg != 64 && wg != 128 && wg != 256) return fail(c, GWG_E_INVAL, "block size must be 64, 128 or 256");
    if (t->bwd_block_threads > 128) return fail(c, GWG_E_INVAL, "adjoint block size must be 64 or 128");
    if (t->rays_per_block < 0 || t->bwd_rays_per_block < 0) return fail(c, GWG_E_INVAL, "negative tile");
    if (t->adj_entries_per_ray < 0 || t->adj_entries_per_ray > 64) return fail(c, GWG_E_INVAL, "adj_entries_per_ray out of range");
    if (t->memo_keys < 0 || t->memo_keys > kFwdMemoKeys) return fail(c, GWG_E_INVAL, "memo_keys out of range");
    if (t->ck_entries_per_ray < -1 || t->ck_entries_per_ray > 64)
        return fail(c, GWG_E_INVAL, "ck_entries_per_ray must be -1, 0 or in [1, 64]");
    if (t->table_nodes != 0 && (t->table_nodes < 4 || t->table_nodes > kTableNodesMax))
        return fail(c, GWG_E_INVAL, "table_nodes must be 0 or in [4, %d]", kTableNodesMax);
    c->tune = *t;
    return GWG_OK;
}

int gwg_get_tuning(const gwg_ctx* c, gwg_tuning* t)
{
    if (!c || !t) return GWG_E_INVAL;
    *t = c->tune;
    return GWG_OK;
}

int gwg_set_timing(gwg_ctx* c, int32_t enable)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    DeviceGuard g(c->device);
    if (enable) {
        for (KernelTimer& t : c->timer) {
            HIP_CHECK(c, t.create(), "create timing events");
            t.recorded = 0;
        }
    }
    c->timing = enable != 0;
    return GWG_OK;
}

int gwg_kernel_times(gwg_ctx* c, int32_t kernel, int32_t n, double* ms)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    if (!c->timing) return fail(c, GWG_E_STATE, "kernel timing is not enabled");
    if (kernel != GWG_KERNEL_FORWARD && kernel != GWG_KERNEL_ADJOINT) return fail(c, GWG_E_INVAL, "unknown kernel id %d", kernel);
    const KernelTimer& t = c->timer[kernel];
    if (!ms || n < 1 || n > GWG_TIMING_RING || n > t.recorded)
        return fail(c, GWG_E_INVAL, "n=%d: between 1 and min(%d, %lld recorded)", n, GWG_TIMING_RING, (long long)t.recorded);
    DeviceGuard g(c->device);
    for (int k = 0; k < n; ++k) {
        const int64_t slot = (t.recorded - n + k) % GWG_TIMING_RING;
        HIP_CHECK(c, hipEventSynchronize(t.ev[slot][1]), "wait for timing event");
        float v = 0.f;
        HIP_CHECK(c, hipEventElapsedTime(&v, t.ev[slot][0], t.ev[slot][1]), "elapsed time");
        ms[k] = v;
    }
    return GWG_OK;
}

int gwg_tmm_rt(gwg_ctx* c, const gwg_stack* stack, const gwg_materials* mats, int64_t n_q,
               const int32_t* d_lambda_idx, const double* d_theta, int32_t precision, double* d_out,
               void* stream)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    int rc = check_materials(c, mats);
    if (rc) return rc;
    if (!stack) return fail(c, GWG_E_INVAL, "stack is NULL");
    if (stack->n_layers < 0 || stack->n_layers > 4096) return fail(c, GWG_E_INVAL, "n_layers out of range");
    if (stack->n_layers > 0 && (!stack->thk_nm || !stack->mat)) return fail(c, GWG_E_INVAL, "stack pointer is NULL");
    if (stack->mat_in < 0 || stack->mat_in >= mats->n_mat || stack->mat_out < 0 || stack->mat_out >= mats->n_mat)
        return fail(c, GWG_E_INVAL, "medium index out of range");
    if (!lossless(mats, stack->mat_in)) return fail(c, GWG_E_INVAL, "incident medium must be lossless");
    if (n_q < 0) return fail(c, GWG_E_INVAL, "n_q < 0");
    if (precision < GWG_FP64 || precision > GWG_FP32) return fail(c, GWG_E_INVAL, "precision out of range");
    if (n_q > 0 && (!d_lambda_idx || !d_theta || !d_out)) return fail(c, GWG_E_INVAL, "query pointer is NULL");
    if (n_q == 0) return GWG_OK;
    std::map<int, int> slot_of;
    std::vector<int> mats_of;
    std::vector<uint8_t> sl((size_t)std::max(stack->n_layers, 1), 0);
    for (int j = 0; j < stack->n_layers; ++j) {
        int mm = stack->mat[j];
        if (mm >= mats->n_mat) return fail(c, GWG_E_INVAL, "layer material %d out of range", mm);
        auto it = slot_of.find(mm);
        if (it == slot_of.end()) {
            if ((int)mats_of.size() == kMaxSlots) return fail(c, GWG_E_INVAL, "more than %d distinct layer materials", kMaxSlots);
            it = slot_of.emplace(mm, (int)mats_of.size()).first;
            mats_of.push_back(mm);
        }
        sl[j] = (uint8_t)it->second;
    }
    int n_slots = std::max<int>(1, (int)mats_of.size());
    if (mats_of.empty()) mats_of.push_back(stack->mat_in);
    uint32_t cplx = 0;
    std::vector<double> lt((size_t)mats->n_lambda * LT_STRIDE, 0.0);
    for (int l = 0; l < mats->n_lambda; ++l) {
        double* row = &lt[(size_t)l * LT_STRIDE];
        row[LT_K0] = 2.0 * 3.14159265358979323846 / mats->lambda_nm[l];
        row[LT_NG] = mats->n_re[l * mats->n_mat + stack->mat_in];
        row[LT_NA] = mats->n_re[l * mats->n_mat + stack->mat_out];
        row[LT_NA + 1] = mats->n_im[l * mats->n_mat + stack->mat_out];
        for (int q = 0; q < n_slots; ++q) {
            double nr = mats->n_re[l * mats->n_mat + mats_of[q]], ni = mats->n_im[l * mats->n_mat + mats_of[q]];
            row[LT_SLOT + 2 * q] = nr;
            row[LT_SLOT + 2 * q + 1] = ni;
            if (ni != 0.0) cplx |= 1u << q;
            crit_interval(row[LT_NG], nr, ni, &row[LT_CRIT + 2 * q], &row[LT_CRIT + 2 * q + 1]);
        }
    }
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    HIP_CHECK(c, c->tmm_tab.ensure(lt.size() * sizeof(double)), "alloc table");
    HIP_CHECK(c, c->tmm_slot.ensure(sl.size()), "alloc slots");
    HIP_CHECK(c, hipMemcpyAsync(c->tmm_tab.p, lt.data(), lt.size() * sizeof(double), hipMemcpyHostToDevice, s), "upload table");
    HIP_CHECK(c, hipMemcpyAsync(c->tmm_slot.p, sl.data(), sl.size(), hipMemcpyHostToDevice, s), "upload slots");
    HIP_CHECK(c, hipStreamSynchronize(s), "upload");
    if (tmm_smem_bytes(stack->n_layers, n_slots, 256) > 65536) return fail(c, GWG_E_INVAL, "stack too large for one workgroup");
    HIP_CHECK(c, launch_tmm_rt(precision, stack->thk_nm, (const uint8_t*)c->tmm_slot.p, stack->n_layers,
                               (const double*)c->tmm_tab.p, mats->n_lambda, n_slots, cplx, d_lambda_idx, d_theta,
                               n_q, d_out, s),
              "tmm kernel");
    return GWG_OK;
}

int gwg_trace_forward(gwg_ctx* c, const gwg_slab* slab, const gwg_prma* prma, const gwg_materials* mats,
                      const gwg_stacks* stacks, const gwg_rays* rays, uint64_t seed, uint64_t step,
                      int32_t precision, uint32_t flags, const gwg_eyebox* out, gwg_ray_record* records, int64_t record_stride,
                      gwg_stats* stats, void* stream)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    int rc = check_scene(c, slab, prma, mats, stacks, rays);
    if (rc) return rc;
    if (precision < GWG_FP64 || precision > GWG_FP32) return fail(c, GWG_E_INVAL, "precision out of range");
    if (step >= (uint64_t(1) << 32)) return fail(c, GWG_E_INVAL, "step must be < 2^32");
    if (!out || !out->q_bins || !out->counts) return fail(c, GWG_E_INVAL, "eyebox outputs are NULL");
    if (out->fp_shift < 0 || out->fp_shift > 40) return fail(c, GWG_E_INVAL, "fp_shift out of range");
    if (records && record_stride < 1) return fail(c, GWG_E_INVAL, "record_stride must be >= 1");
    if (flags & ~(uint32_t)(GWG_FWD_GRAD | GWG_FWD_MEMO | GWG_FWD_TABLE)) return fail(c, GWG_E_INVAL, "unknown flags 0x%x", flags);
    if ((flags & GWG_FWD_MEMO) && (flags & GWG_FWD_TABLE))
        return fail(c, GWG_E_INVAL, "GWG_FWD_MEMO and GWG_FWD_TABLE exclude each other");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const bool cap = stream_capturing(s);
    if (cap && stats) return fail(c, GWG_E_STATE, "stats need a synchronization: not available during stream capture");
    c->adj_valid = false;
    c->have_forward = false;
    c->tab_grad = false;
    rc = build_scene(c, slab, prma, mats, stacks, rays, s);
    if (rc) return rc;
    SceneDev sc = c->sc;
    sc.thk = stacks->thk_nm;
    sc.fp_shift = out->fp_shift;
    sc.key0 = (uint32_t)seed;
    sc.key1 = (uint32_t)(seed >> 32) ^ (uint32_t)step;
    sc.seed_hi = (uint32_t)(seed >> 32);
    sc.step_host = (uint32_t)step;
    sc.step_dev = c->step_dev;
    sc.precision = precision;
    const int B = sc.bins_x * sc.bins_y;
    const bool lds_bins = B <= 2048;
    // memoized solves need collimated beams (shared hit keys) and room for the key tables
    sc.memo = ((flags & GWG_FWD_MEMO) && sc.fov_mode == 0) ? (c->tune.memo_keys ? c->tune.memo_keys : kFwdMemoKeys) : 0;
    sc.table = nullptr;
    sc.table_n = 0;
    sc.tab_scale = nullptr;
    sc.tab_acc = nullptr;
    int wg = pick_fwd_wg(c, sc, lds_bins);
    if (sc.memo && fwd_smem_bytes(sc, wg, lds_bins) > 65536) {
        sc.memo = 0;                                   // per-hit solves (their own slot table size)
        wg = pick_fwd_wg(c, sc, lds_bins);
    }
    set_tiles(sc, c->tune.rays_per_block, wg, c->n_cu);
    if (fwd_smem_bytes(sc, wg, lds_bins) > 65536) return fail(c, GWG_E_INVAL, "scene too large for one workgroup's LDS");
    if (sc.n_items > 0x7fffffff) return fail(c, GWG_E_INVAL, "too many work items; raise rays_per_block");
    const int64_t nbins = (int64_t)sc.D * sc.n_lsel * sc.F * B;
    const bool table = (flags & GWG_FWD_TABLE) != 0;
    // per-hit solves take a wave's rays in pools of rounds (all of an item's
    // rounds, up to kPoolMax); the memoized and table forwards round by round
    sc.pool = (sc.memo || table) ? 1 : (int32_t)std::min<int64_t>(kPoolMax, (sc.rays_per_tile + wg - 1) / wg);
    if (table) {
        const int n = c->tune.table_nodes ? c->tune.table_nodes : kTableNodesDefault;
        const size_t tab_b = sizeof(double) * 8 * (size_t)sc.D * sc.n_lsel * sc.M * 2 * (size_t)n;
        if (!cap) {
            size_t free_b = 0, total_b = 0;
            (void)hipMemGetInfo(&free_b, &total_b);
            if ((double)tab_b > 0.5 * (double)free_b + (double)c->tab.bytes)
                return fail(c, GWG_E_INVAL, "angle table of %zu bytes does not fit in device memory; lower table_nodes", tab_b);
        }
        rc = ensure_buf(c, c->tab, tab_b, cap, "alloc angle table");
        if (rc) return rc;
        rc = ensure_buf(c, c->tab_scale, sizeof(uint64_t) * 4, cap, "alloc table scale");
        if (rc) return rc;
        sc.table = (const double*)c->tab.p;
        sc.table_n = n;
        sc.tab_scale = (unsigned long long*)c->tab_scale.p;
    }
    // adjoint entries: per (item, wave) region of cap_w entries, if they fit the budget
    bool adj = false;
    bool adj_sweep = false;      // the forward runs the path adjoint (with or without room for entries)
    if (flags & GWG_FWD_GRAD) {
        const int waves = wg / 64;
        const int64_t per_ray = c->tune.adj_entries_per_ray > 0 ? c->tune.adj_entries_per_ray : kAdjEntriesPerRay;
        const int64_t cap_w = ((sc.rays_per_tile + wg - 1) / wg) * 64 * per_ray;
        const int64_t total = sc.n_items * waves * cap_w;
        const size_t ent_b = sizeof(double) * (size_t)(total * kEntFields);
        const size_t cnt_b = sizeof(int32_t) * (size_t)(sc.n_items * waves);
        const size_t ovf_b = sizeof(int32_t) * (size_t)sc.n_items;
        bool fits;
        if (cap) {
            // nothing may be allocated: use the entries if the buffers already hold them
            fits = c->adj_ent.p && c->adj_ent.bytes >= ent_b && c->adj_cnt.bytes >= cnt_b && c->adj_ovf.bytes >= ovf_b;
        } else {
            size_t free_b = 0, total_b = 0;
            (void)hipMemGetInfo(&free_b, &total_b);
            const double bytes = (double)ent_b + (double)cnt_b + (double)ovf_b;
            fits = bytes <= std::min<double>(kAdjBudgetBytes, 0.5 * (double)free_b + (double)c->adj_ent.bytes);
        }
        if (fits) {
            rc = ensure_buf(c, c->adj_ent, ent_b, cap, "alloc adjoint entries");
            if (rc) return rc;
            rc = ensure_buf(c, c->adj_cnt, cnt_b, cap, "alloc entry counts");
            if (rc) return rc;
            rc = ensure_buf(c, c->adj_ovf, ovf_b, cap, "alloc overflow flags");
            if (rc) return rc;
            HIP_CHECK(c, launch_fill_u32((uint32_t*)c->adj_ovf.p, sc.n_items, 0u, s), "zero overflow flags");
            c->adj = AdjStore{ (double*)c->adj_ent.p, (int32_t*)c->adj_cnt.p, (int32_t*)c->adj_ovf.p, cap_w, total, waves,
                               nullptr, 0, 0, nullptr };
            adj = true;
            // The FP64 solve can keep the adjoint's sweep checkpoints of the
            // first ck_cap entries of every region (kCkEntriesPerRay per ray,
            // fewer if memory is short); the adjoint then skips that sweep.
            const int64_t ck_per = c->tune.ck_entries_per_ray == 0 ? kCkEntriesPerRay : c->tune.ck_entries_per_ray;
            if (precision == GWG_FP64 && !(flags & GWG_FWD_MEMO) && sc.slot_complex == 0u && ck_per > 0) {
                const int64_t blocks = ck_blocks(sc.Lmax);
                const int64_t rays_w = (sc.rays_per_tile + wg - 1) / wg * 64;
                // in quarter entries per ray, down to a quarter
                for (int64_t per4 = 4 * ck_per; per4 >= 1; --per4) {
                    const int64_t ck_cap = std::min<int64_t>(cap_w, rays_w * per4 / 4);
                    const int64_t ck_total = sc.n_items * waves * ck_cap;
                    const size_t ck_b = sizeof(double) * 8 * (size_t)blocks * (size_t)ck_total;
                    bool ok;
                    if (cap) {
                        ok = c->adj_ck.p && c->adj_ck.bytes >= ck_b;
                    } else {
                        size_t free_b = 0, total_b = 0;
                        (void)hipMemGetInfo(&free_b, &total_b);
                        ok = (double)ck_b <= std::min<double>(kCkBudgetBytes, 0.5 * (double)free_b + (double)c->adj_ck.bytes);
                    }
                    if (!ok) continue;
                    rc = ensure_buf(c, c->adj_ck, ck_b, cap, "alloc sweep checkpoints");
                    if (rc) return rc;
                    c->adj.ck = (double*)c->adj_ck.p;
                    c->adj.ck_cap = ck_cap;
                    c->adj.ck_total = ck_total;
                    break;
                }
            }
        } else if (table) {
            // the table backward needs the sweep's cotangent bound even when no
            // entry can be kept: regions of zero entries, every item regenerated
            rc = ensure_buf(c, c->adj_cnt, cnt_b, cap, "alloc entry counts");
            if (rc) return rc;
            rc = ensure_buf(c, c->adj_ovf, ovf_b, cap, "alloc overflow flags");
            if (rc) return rc;
            c->adj = AdjStore{ nullptr, (int32_t*)c->adj_cnt.p, (int32_t*)c->adj_ovf.p, 0, 0, waves, nullptr, 0, 0, nullptr };
        }
        adj_sweep = adj || table;
    }
    // persistent grid: as many workgroups as fit on the device at once
    const int kind_f = adj_sweep ? (table ? KIND_FWD_ADJ_TAB : sc.memo ? KIND_FWD_ADJ_MEMO : KIND_FWD_ADJ)
                                 : (table ? KIND_FWD_TAB : sc.memo ? KIND_FWD_MEMO : KIND_FWD);
    const int per_cu = occupancy(c, kind_f, precision, wg, fwd_smem_bytes(sc, wg, lds_bins));
    const int64_t grid = std::min<int64_t>(sc.n_items, (int64_t)std::max(c->n_cu, 1) * per_cu);
    rc = ensure_buf(c, c->fwd_scratch, sizeof(double) * (size_t)fwd_scratch_doubles(sc, grid, wg), cap, "alloc hit queues");
    if (rc) return rc;
    if (adj_sweep) {
        rc = ensure_buf(c, c->fwd_tape, sizeof(double) * (size_t)(grid * wg * (int64_t)sc.Kmax * kTapeStride), cap,
                        "alloc forward tape");
        if (rc) return rc;
    }
    rc = ensure_buf(c, c->stats, sizeof(uint64_t) * ST_WORDS, cap, "alloc stats");
    if (rc) return rc;
    HIP_CHECK(c, launch_fill_u64(out->q_bins, nbins, 0, s), "zero bins");
    HIP_CHECK(c, launch_fill_u32(out->counts, nbins, 0, s), "zero counts");
    HIP_CHECK(c, launch_fill_u64((uint64_t*)c->stats.p, ST_WORDS, 0, s), "zero stats");
    if (table) {
        HIP_CHECK(c, launch_fill_u64((uint64_t*)c->tab_scale.p, 4, 0, s), "zero table scale");
        HIP_CHECK(c, launch_table_build(sc, (double*)c->tab.p, c->n_cu, (unsigned long long*)c->stats.p, s),
                  "angle table kernel");
    }
    {
        // items are taken in decreasing order of the mirror hits that the last
        // forward of the same decomposition recorded (its first call: item
        // order), so the workgroups finish together; results do not depend on it
        const int waves_f = wg / 64;
        rc = ensure_buf(c, c->item_work, sizeof(int32_t) * (size_t)(sc.n_items * waves_f), cap, "alloc item work");
        if (rc) return rc;
        rc = ensure_buf(c, c->fwd_order, sizeof(int32_t) * (size_t)sc.n_items, cap, "alloc forward order");
        if (rc) return rc;
        sc.fwd_order = nullptr;
        if (c->work_items == sc.n_items && c->work_waves == waves_f) {
            HIP_CHECK(c, launch_item_order((const int32_t*)c->item_work.p, waves_f, sc.n_items,
                                           sc.rays_per_tile * (int64_t)sc.Kmax, (int32_t*)c->fwd_order.p, s),
                      "forward item order");
            sc.fwd_order = (const int32_t*)c->fwd_order.p;
        }
        sc.item_work = (int32_t*)c->item_work.p;
        c->work_items = sc.n_items;
        c->work_waves = waves_f;
    }
    if (c->timing && !cap) HIP_CHECK(c, hipEventRecord(c->timer[GWG_KERNEL_FORWARD].begin(), s), "timing event");
    HIP_CHECK(c, launch_trace_fwd(sc, wg, (int)grid, lds_bins, out->q_bins, out->counts, (unsigned long long*)c->stats.p,
                                  records, record_stride, (double*)c->fwd_scratch.p, adj_sweep ? &c->adj : nullptr,
                                  (double*)c->fwd_tape.p, s),
              "forward kernel");
    if (c->timing && !cap) {
        HIP_CHECK(c, hipEventRecord(c->timer[GWG_KERNEL_FORWARD].end(), s), "timing event");
        ++c->timer[GWG_KERNEL_FORWARD].recorded;
    }
    if (out->irradiance)
        HIP_CHECK(c, launch_irradiance(out->q_bins, nbins, std::ldexp(1.0, -out->fp_shift) / (double)sc.N, out->irradiance, s),
                  "irradiance kernel");
    c->fwd = sc;
    c->have_forward = true;
    c->adj_valid = adj;
    c->memo = (flags & GWG_FWD_MEMO) != 0;
    c->tab_grad = table && adj_sweep;
    if (stats) {
        rc = read_stats(c, s, stats);
        if (rc) return rc;
        if (stats->saturated) return fail(c, GWG_E_OVERFLOW, "%lld bin contributions saturated", (long long)stats->saturated);
    }
    return GWG_OK;
}

int gwg_trace_backward(gwg_ctx* c, const double* d_dL_dI, double* d_grad, int64_t sample_stride,
                       gwg_stats* stats, void* stream)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    if (!c->have_forward) return fail(c, GWG_E_STATE, "gwg_trace_backward called before gwg_trace_forward");
    if (!d_dL_dI || !d_grad) return fail(c, GWG_E_INVAL, "NULL gradient pointer");
    if (sample_stride < 1) return fail(c, GWG_E_INVAL, "sample_stride must be >= 1");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const bool cap = stream_capturing(s);
    if (cap && stats) return fail(c, GWG_E_STATE, "stats need a synchronization: not available during stream capture");
    int rc = GWG_OK;
    SceneDev sc = c->fwd;
    if (sc.table && !c->tab_grad)
        return fail(c, GWG_E_STATE, "the angle-table backward needs a forward run with GWG_FWD_GRAD");
    const int wg = pick_bwd_wg(c, sc);
    // With entries from the forward, the backward keeps the forward's work
    // items: the entry kernel covers items whose regions fit, the
    // regenerating kernel the rest.  Otherwise every item is regenerated.
    const bool entries = c->adj_valid && sample_stride == 1;
    if (!entries) set_tiles(sc, c->tune.bwd_rays_per_block, wg, c->n_cu);
    if (bwd_smem_bytes(sc, wg) > 65536) return fail(c, GWG_E_INVAL, "scene too large for one workgroup's LDS");
    // persistent grids: as many workgroups as fit on the device at once
    const size_t smem = bwd_smem_bytes(sc, wg);
    const int64_t n_cu = std::max(c->n_cu, 1);
    const int64_t grid = std::min<int64_t>(
        sc.n_items, n_cu * occupancy(c, sc.table ? KIND_BWD_REGEN_TAB : KIND_BWD_REGEN, sc.precision, wg, smem));
    const int kind_e = sc.slot_complex == 0u ? KIND_ADJ_LOSSLESS : KIND_ADJ_ENTRIES;
    const int64_t grid_e = std::min<int64_t>(sc.n_items, n_cu * occupancy(c, kind_e, sc.precision, wg, smem));
    const int kind_m = sc.slot_complex == 0u ? KIND_ADJ_MEMO_LOSSLESS : KIND_ADJ_MEMO;
    const int64_t grid_m = std::min<int64_t>(sc.n_items, n_cu * occupancy(c, kind_m, sc.precision, 64, memo_smem_bytes(sc)));
    const int ML = sc.M * sc.Lmax;
    int64_t scratch_d = std::max(bwd_scratch_doubles(sc, grid, wg), entries ? adj_scratch_doubles(sc, grid_e, wg) : 0);
    if (entries && c->memo) scratch_d = std::max(scratch_d, adj_scratch_doubles(sc, grid_m, 64));
    if (sc.table) scratch_d = std::max(scratch_d, adj_scratch_doubles(sc, table_adj_blocks(sc), 128));
    rc = ensure_buf(c, c->scratch, sizeof(double) * (size_t)scratch_d, cap, "alloc adjoint scratch");
    if (rc) return rc;
    const int64_t partial_d = sc.table ? table_adj_blocks(sc) * sc.Lmax : sc.n_items * (int64_t)ML;
    rc = ensure_buf(c, c->partial, sizeof(double) * (size_t)partial_d, cap, "alloc partial gradients");
    if (rc) return rc;
    rc = ensure_buf(c, c->stats, sizeof(uint64_t) * ST_WORDS, cap, "alloc stats");
    if (rc) return rc;
    HIP_CHECK(c, launch_fill_u64((uint64_t*)c->stats.p, ST_WORDS, 0, s), "zero stats");
    if (sc.table) {
        // angle table: cotangents of the table entries, then one adjoint per entry
        if (table_adj_smem_bytes(sc) > 65536) return fail(c, GWG_E_INVAL, "scene too large for the table adjoint's LDS");
        const int64_t n_acc = table_adj_blocks(sc) * (int64_t)sc.table_n * 4;
        rc = ensure_buf(c, c->tab_acc, sizeof(int64_t) * (size_t)n_acc, cap, "alloc table cotangents");
        if (rc) return rc;
        sc.tab_acc = (long long*)c->tab_acc.p;
        const int64_t nbins = (int64_t)sc.D * sc.n_lsel * sc.F * sc.bins_x * sc.bins_y;
        const int64_t grid_t = std::min<int64_t>(sc.n_items, n_cu * occupancy(c, KIND_TABLE_ACCUM, sc.precision, 256,
                                                                              table_accum_smem_bytes()));
        HIP_CHECK(c, launch_fill_u64((uint64_t*)c->tab_acc.p, n_acc, 0, s), "zero table cotangents");
        HIP_CHECK(c, launch_fill_u64((uint64_t*)(sc.tab_scale + 2), 1, 0, s), "zero dL/dI bound");
        HIP_CHECK(c, launch_absmax(d_dL_dI, nbins, sc.tab_scale + 2, s), "dL/dI bound");
        if (c->timing && !cap) HIP_CHECK(c, hipEventRecord(c->timer[GWG_KERNEL_ADJOINT].begin(), s), "timing event");
        if (entries) HIP_CHECK(c, launch_table_accum(sc, (int)grid_t, d_dL_dI, c->adj, s), "table cotangent kernel");
        HIP_CHECK(c, launch_trace_bwd(sc, wg, (int)grid, d_dL_dI, (unsigned long long*)c->stats.p, (double*)c->partial.p,
                                      (double*)c->scratch.p, sample_stride, entries ? c->adj.ovf : nullptr, s),
                  "adjoint kernel");
        HIP_CHECK(c, launch_table_adj(sc, (double*)c->partial.p, (double*)c->scratch.p, (unsigned long long*)c->stats.p, s),
                  "table adjoint kernel");
        if (c->timing && !cap) {
            HIP_CHECK(c, hipEventRecord(c->timer[GWG_KERNEL_ADJOINT].end(), s), "timing event");
            ++c->timer[GWG_KERNEL_ADJOINT].recorded;
        }
        HIP_CHECK(c, launch_table_reduce((const double*)c->partial.p, sc, d_grad, s), "gradient reduction");
        if (stats) return read_stats(c, s, stats);
        return GWG_OK;
    }
    if (c->timing && !cap) HIP_CHECK(c, hipEventRecord(c->timer[GWG_KERNEL_ADJOINT].begin(), s), "timing event");
    if (entries && c->memo)
        HIP_CHECK(c, launch_adj_memo(sc, (int)grid_m, d_dL_dI, (unsigned long long*)c->stats.p, (double*)c->partial.p,
                                     c->adj, (double*)c->scratch.p, s),
                  "memoized adjoint kernel");
    else if (entries) {
        // the entry kernel takes items largest first (entry counts from the
        // forward), so its workgroups finish together
        rc = ensure_buf(c, c->adj_order, sizeof(int32_t) * (size_t)sc.n_items, cap, "alloc item order");
        if (rc) return rc;
        AdjStore st = c->adj;
        st.order = (const int32_t*)c->adj_order.p;
        HIP_CHECK(c, launch_item_order(st.cnt, st.waves, sc.n_items, (int64_t)st.waves * st.cap_w,
                                       (int32_t*)c->adj_order.p, s),
                  "item order");
        HIP_CHECK(c, launch_adj_entries(sc, wg, (int)grid_e, d_dL_dI, (unsigned long long*)c->stats.p, (double*)c->partial.p,
                                        st, (double*)c->scratch.p, s),
                  "adjoint entry kernel");
    }
    HIP_CHECK(c, launch_trace_bwd(sc, wg, (int)grid, d_dL_dI, (unsigned long long*)c->stats.p, (double*)c->partial.p,
                                  (double*)c->scratch.p, sample_stride, entries ? c->adj.ovf : nullptr, s),
              "adjoint kernel");
    if (c->timing && !cap) {
        HIP_CHECK(c, hipEventRecord(c->timer[GWG_KERNEL_ADJOINT].end(), s), "timing event");
        ++c->timer[GWG_KERNEL_ADJOINT].recorded;
    }
    rc = ensure_buf(c, c->grad_tmp, sizeof(double) * (size_t)grad_reduce_tmp_doubles(ML, sc.D), cap,
                    "alloc gradient reduction");
    if (rc) return rc;
    HIP_CHECK(c, launch_grad_reduce((const double*)c->partial.p, sc.n_items / sc.D, ML, sc.D, (double*)c->grad_tmp.p,
                                    d_grad, sc.nlay, sc.M, sc.Lmax, s),
              "gradient reduction");
    if (stats) return read_stats(c, s, stats);
    return GWG_OK;
}

int gwg_loss(gwg_ctx* c, const double* d_irr, int32_t D, int32_t n_l, int32_t F, int32_t B, int32_t kind,
             double w_f, double w_e, double* d_loss, double* d_dL_dI, void* stream)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    if (!d_irr || !d_loss) return fail(c, GWG_E_INVAL, "NULL loss pointer");
    if (D < 1 || n_l < 1 || F < 1 || B < 1) return fail(c, GWG_E_INVAL, "loss shape invalid");
    if ((int64_t)D * n_l * F > 0x7fffffff) return fail(c, GWG_E_INVAL, "loss shape too large");
    if (kind < 0 || kind > 2) return fail(c, GWG_E_INVAL, "kind must be 0, 1 or 2");
    if (!(is_fin(w_f) && is_fin(w_e))) return fail(c, GWG_E_INVAL, "weights must be finite");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const bool cap = stream_capturing(s);
    int rc = GWG_OK;
    size_t n = (size_t)loss_work_doubles(D, n_l, F, B);
    rc = ensure_buf(c, c->loss_work, n * sizeof(double), cap, "alloc loss work");
    if (rc) return rc;
    HIP_CHECK(c, launch_loss(d_irr, D, n_l, F, B, kind, w_f, w_e, (double*)c->loss_work.p, d_loss, d_dL_dI, s),
              "loss kernels");
    return GWG_OK;
}

int gwg_loss_noalloc(gwg_ctx* c, const double* d_irr, int32_t D, int32_t n_l, int32_t F, int32_t B, int32_t kind,
                     double w_f, double w_e, double* d_loss, double* d_dL_dI, void* stream)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    if (!d_irr || !d_loss) return fail(c, GWG_E_INVAL, "NULL loss pointer");
    if (D < 1 || n_l < 1 || F < 1 || B < 1) return fail(c, GWG_E_INVAL, "loss shape invalid");
    if ((int64_t)D * n_l * F > 0x7fffffff) return fail(c, GWG_E_INVAL, "loss shape too large");
    if (kind < 0 || kind > 2) return fail(c, GWG_E_INVAL, "kind must be 0, 1 or 2");
    if (!(is_fin(w_f) && is_fin(w_e))) return fail(c, GWG_E_INVAL, "weights must be finite");
    const int64_t need = loss_work_doubles(D, n_l, F, B);
    if (need > kLossScratchDoubles)
        return fail(c, GWG_E_INVAL,
                    "loss shape needs %lld doubles of scratch, more than the fixed %lld (D*(n_l*F + B + F + 8) "
                    "must not exceed %lld); use gwg_loss",
                    (long long)need, (long long)kLossScratchDoubles, (long long)kLossScratchDoubles);
    DeviceGuard g(c->device);
    double* work = loss_scratch(c->device);
    if (!work) return fail(c, GWG_E_STATE, "no scratch address for device %d", c->device);
    // every scratch word the kernels read is written by an earlier kernel of
    // the same call, so nothing needs clearing
    HIP_CHECK(c, launch_loss(d_irr, D, n_l, F, B, kind, w_f, w_e, work, d_loss, d_dL_dI, (hipStream_t)stream),
              "loss kernels");
    return GWG_OK;
}

int gwg_omega_gradient(gwg_ctx* c, const double* d_W, const uint32_t* d_counts, double* d_grad, void* stream)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    if (!c->have_forward) return fail(c, GWG_E_STATE, "gwg_omega_gradient called before gwg_trace_forward");
    if (!d_W || !d_counts || !d_grad) return fail(c, GWG_E_INVAL, "NULL pointer");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const bool cap = stream_capturing(s);
    const SceneDev sc = c->fwd;                    // the forward's items, seeds and decisions
    const int wg = 256;
    const size_t smem = omega_smem_bytes(sc, wg);
    if (smem > 65536) return fail(c, GWG_E_INVAL, "scene too large for one workgroup's LDS");
    const int64_t n_cu = std::max(c->n_cu, 1);
    const int64_t grid = std::min<int64_t>(sc.n_items, n_cu * occupancy(c, KIND_OMEGA, sc.precision, wg, smem));
    int rc = ensure_buf(c, c->partial, sizeof(double) * (size_t)sc.n_items * sc.M, cap, "alloc partial gradients");
    if (rc) return rc;
    HIP_CHECK(c, launch_omega_grad(sc, (int)grid, wg, d_W, d_counts, (double*)c->partial.p, d_grad, s),
              "reflection-probability gradient kernel");
    return GWG_OK;
}

int gwg_forward_kept_entries(const gwg_ctx* c, int32_t* kept)
{
    if (!c || !kept) return GWG_E_INVAL;
    *kept = (c->have_forward && c->adj_valid) ? 1 : 0;
    return GWG_OK;
}

int gwg_set_step_source(gwg_ctx* c, const uint32_t* d_step)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    c->step_dev = d_step;
    return GWG_OK;
}

int gwg_autotune(gwg_ctx* c, const gwg_slab* slab, const gwg_prma* prma, const gwg_materials* mats,
                 const gwg_stacks* stacks, const gwg_rays* rays, uint64_t seed, int32_t precision, uint32_t flags,
                 const char* cache_path, gwg_tuning* out, void* stream)
{
    if (!c) return GWG_E_INVAL;
    c->err.clear();
    if (!out) return fail(c, GWG_E_INVAL, "out is NULL");
    int rc = check_scene(c, slab, prma, mats, stacks, rays);
    if (rc) return rc;
    if (precision < GWG_FP64 || precision > GWG_FP32) return fail(c, GWG_E_INVAL, "precision out of range");
    if (flags & ~(uint32_t)(GWG_FWD_GRAD | GWG_FWD_MEMO)) return fail(c, GWG_E_INVAL, "unknown flags 0x%x", flags);
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (stream_capturing(s)) return fail(c, GWG_E_STATE, "gwg_autotune cannot run during stream capture");
    rc = build_scene(c, slab, prma, mats, stacks, rays, s);
    if (rc) return rc;
    uint64_t key = fnv_v(c->scene_hash, precision);
    key = fnv_v(key, flags);
    key = fnv_v(key, c->n_cu);
    auto hit = c->tuned.find(key);
    if (hit != c->tuned.end()) {
        *out = c->tune = hit->second;
        return GWG_OK;
    }
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            unsigned long long k = 0;
            long long rpb = 0, brpb = 0;
            int wg = 0, bwg = 0, adj = 0;
            bool found = false;
            while (std::fscanf(f, "%llx %d %lld %d %lld %d", &k, &wg, &rpb, &bwg, &brpb, &adj) == 6)
                if (k == key) {
                    found = true;
                    break;
                }
            std::fclose(f);
            if (found) {
                gwg_tuning t{ wg, rpb, bwg, brpb, adj, c->tune.memo_keys, c->tune.table_nodes, c->tune.ck_entries_per_ray };
                if (gwg_set_tuning(c, &t) == GWG_OK) {
                    c->tuned[key] = t;
                    *out = t;
                    return GWG_OK;
                }
            }
        }
    }
    const SceneDev sc0 = c->sc;
    const int B = sc0.bins_x * sc0.bins_y;
    const bool lds_bins = B <= 2048;
    const int64_t nbins = (int64_t)sc0.D * sc0.n_lsel * sc0.F * B;
    const int64_t ngrad = (int64_t)sc0.D * sc0.M * sc0.Lmax;
    HIP_CHECK(c, c->tune_q.ensure(sizeof(uint64_t) * (size_t)nbins), "alloc autotune bins");
    HIP_CHECK(c, c->tune_c.ensure(sizeof(uint32_t) * (size_t)nbins), "alloc autotune counts");
    HIP_CHECK(c, c->tune_g.ensure(sizeof(double) * (size_t)nbins), "alloc autotune dL/dI");
    HIP_CHECK(c, c->tune_grad.ensure(sizeof(double) * (size_t)ngrad), "alloc autotune gradient");
    HIP_CHECK(c, launch_fill_f64((double*)c->tune_g.p, nbins, 1.0, s), "fill dL/dI");
    gwg_eyebox eb{};
    eb.q_bins = (uint64_t*)c->tune_q.p;
    eb.counts = (uint32_t*)c->tune_c.p;
    eb.irradiance = nullptr;
    eb.fp_shift = 24;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_CHECK(c, hipEventCreate(&e0), "event");
    HIP_CHECK(c, hipEventCreate(&e1), "event");
    const gwg_tuning saved = c->tune;
    // times one call (after one warm-up call); -1 on error
    auto timed = [&](auto&& call) -> double {
        if (call() != GWG_OK) return -1.0;
        if (hipEventRecord(e0, s) != hipSuccess) return -1.0;
        if (call() != GWG_OK) return -1.0;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
        return ms;
    };
    auto forward = [&]() {
        return gwg_trace_forward(c, slab, prma, mats, stacks, rays, seed, 0, precision, flags, &eb, nullptr, 1,
                                 nullptr, stream);
    };
    // with a gradient to follow, a tile is timed over forward + backward: the
    // adjoint takes its work items from the forward's decomposition
    const bool with_bwd = (flags & GWG_FWD_GRAD) != 0;
    auto step = [&]() {
        const int r = forward();
        if (r != GWG_OK || !with_bwd) return r;
        return gwg_trace_backward(c, (const double*)c->tune_g.p, (double*)c->tune_grad.p, 1, nullptr, stream);
    };
    // forward candidates: block size x ray tile; bins must not depend on them
    std::vector<gwg_tuning> cands;
    for (int wg : { 256, 128 }) {
        if (fwd_smem_bytes(sc0, wg, lds_bins) > 65536) continue;
        SceneDev t = sc0;
        set_tiles(t, 0, wg, c->n_cu);
        std::vector<int64_t> seen;
        for (int shift : { 0, -1, 1, -2, 2 }) {
            int64_t rpt = shift >= 0 ? t.rays_per_tile << shift : t.rays_per_tile >> -shift;
            rpt = std::max<int64_t>(rpt, (int64_t)wg * 4);
            rpt = std::min<int64_t>(((rpt + wg - 1) / wg) * wg, sc0.N);
            if (std::find(seen.begin(), seen.end(), rpt) != seen.end()) continue;
            seen.push_back(rpt);
            gwg_tuning cand = saved;
            cand.block_threads = wg;
            cand.rays_per_block = rpt;
            cands.push_back(cand);
        }
    }
    const bool verify = nbins <= (int64_t)1 << 24;
    std::vector<uint64_t> ref, cur;
    double best_ms = -1.0;
    gwg_tuning best = saved;
    for (size_t i = 0; i < cands.size(); ++i) {
        c->tune = cands[i];
        const double ms = timed(step);
        if (ms < 0.0) continue;
        if (verify) {
            cur.resize((size_t)nbins);
            if (hipMemcpy(cur.data(), c->tune_q.p, sizeof(uint64_t) * (size_t)nbins, hipMemcpyDeviceToHost) != hipSuccess)
                continue;
            if (ref.empty()) ref = cur;
            else if (cur != ref) {
                (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
                c->tune = saved;
                c->have_forward = false;
                return fail(c, GWG_E_STATE, "eyebox bins differ between launch configurations");
            }
        }
        if (best_ms < 0.0 || ms < best_ms) { best_ms = ms; best = cands[i]; }
    }
    // adjoint block size, with the chosen forward
    {
        double bbest = -1.0;
        gwg_tuning bsel = best;
        for (int bwg : { 128, 64 }) {
            gwg_tuning cand = best;
            cand.bwd_block_threads = bwg;
            c->tune = cand;
            if (forward() != GWG_OK) continue;
            const double ms = timed([&]() {
                return gwg_trace_backward(c, (const double*)c->tune_g.p, (double*)c->tune_grad.p, 1, nullptr, stream);
            });
            if (ms < 0.0) continue;
            if (bbest < 0.0 || ms < bbest) { bbest = ms; bsel = cand; }
        }
        best = bsel;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->have_forward = false;      // the tuning runs leave nothing for a backward
    if (best_ms < 0.0) {
        c->tune = saved;
        return fail(c, GWG_E_STATE, "no launch configuration ran: %s", c->err.c_str());
    }
    c->tune = best;
    c->tuned[key] = best;
    *out = best;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "%llx %d %lld %d %lld %d\n", (unsigned long long)key, best.block_threads,
                         (long long)best.rays_per_block, best.bwd_block_threads, (long long)best.bwd_rays_per_block,
                         best.adj_entries_per_ray);
            std::fclose(f);
        }
    }
    return GWG_OK;
}

}  // extern "C"
