// Internal layout shared by the host API and the HIP kernels.
//
// The host turns the caller's scene description into one SceneDev value
// (passed by value to every trace kernel) plus a few small device tables:
//   - lam_tab  [n_lsel][LT_STRIDE] f64: per selected wavelength the free-space
//              wavenumber, glass and air indices, the complex index of every
//              material slot used by the stacks and the near-critical kappa
//              intervals of the mixed-precision rule;
//   - dir_tab  [n_lsel][F][4] f64: guided direction of every grid FoV point;
//   - slot     [D][M][Lmax] u8: compact material slot of every layer.
// Thicknesses stay in the caller's device array [D][M][Lmax] f64.
#pragma once
#include <stdint.h>

namespace gwg {

constexpr int kMaxMirrors = 16;
constexpr int kMaxPupils = 64;        // eye pupils on the eyebox plane
constexpr int kMaxSlots = 8;          // distinct layer materials in one scene
constexpr int kMaxLayers = 1024;
constexpr int kMaxEvents = 256;
constexpr int LT_STRIDE = 64;         // doubles per wavelength in lam_tab
// lam_tab columns
constexpr int LT_K0 = 0;              // 2 pi / lambda, per nm
constexpr int LT_NG = 1;              // glass index (real)
constexpr int LT_NA = 2;              // air index (real)
constexpr int LT_SLOT = 4;            // slot s: (re, im) at LT_SLOT + 2 s
constexpr int LT_CRIT = 24;           // slot s: near-critical kappa interval (lo, hi) at LT_CRIT + 2 s
constexpr int LT_NSLOT = 40;          // number of slots (as double)

constexpr int kTapeLine = 8;          // doubles of a tape event line
constexpr int kTapeMir = 4;           // doubles of a tape mirror record
constexpr int kTapeStride = kTapeLine + kTapeMir;  // tape doubles per lane and event slot
constexpr int kSeg = 4;               // layers per recomputation segment (backward)
// Checkpoint interval of the lossless adjoint's sweep (the adjoint walks each
// interval down from its top checkpoint with inverse layer matrices): kSegL
// for a hit that meets an evanescent lossless layer, kSegLC for one whose
// layers all propagate.  A walk's rounding error grows at most like the
// square of the interval's transfer growth: with circular layers that is
// polynomial in the interval except inside a reflection band, where a
// quarter-wave pair of index ratio 1.64 grows it 1.64-fold; 32 layers keep it
// below 1e7 there.  Hyperbolic layers grow it exponentially in their
// thickness, so their hits keep the shorter interval.
constexpr int kSegL = 16;
constexpr int kSegLC = 32;                 // both powers of two
__host__ __device__ inline int ck_interval(bool evanescent) { return evanescent ? kSegL : kSegLC; }
// checkpoint blocks per stored adjoint entry: v_0 and v_{g K}, g >= 1, for
// either interval K
__host__ __device__ inline int64_t ck_blocks(int lmax) { return lmax / kSegL + 1; }

enum EventType { EV_NONE = 0, EV_TIR = 1, EV_EXIT = 2, EV_LEAK = 3, EV_END = 4, EV_MIRROR = 5 };
enum Category { CAT_EYEBOX = 0, CAT_MISS = 1, CAT_LEAK = 2, CAT_END = 3, CAT_TRUNC = 4,
                CAT_LOST = 5, CAT_FACE_R = 6, NCAT = 8 };
enum Surface { SURF_TOP = 1000, SURF_BOTTOM = 1001, SURF_END0 = 1002, SURF_END1 = 1003 };

// stats layout (u64 words, device)
enum StatWord { ST_RAYS = 0, ST_EVENTS = 1, ST_PRMA = 2, ST_FP64 = 3, ST_SAT = 4,
                ST_LAYERS = 5, ST_ADJ_RAYS = 6, ST_ADJ_HITS = 7, ST_ADJ_LAYERS = 8,
                ST_CAT = 9,           // 8 words of counts
                ST_POW = 17,          // 8 words of power (fixed point 2^-24)
                ST_ADJ_STORED = 25,   // adjoint layer steps whose sweep the forward stored
                ST_NEXT0 = 26,        // work-item counter of the call's first item kernel
                ST_NEXT1 = 27,        // ... and of its second (the backward's regenerating kernel)
                ST_WORDS = 28 };

// Adjoint entries recorded by the forward trace for the backward: per
// (work item, forward wave) a region of cap_w entries, field f of entry e at
// ent[f * total + e], e = (item * waves + wave) * cap_w + k.  Fields: kappa,
// G_s (re, im), G_p (re, im) without the dL/dI factor, meta = mirror |
// front << 8 | reflected << 9 | bin << 10 (an exact integer in a double).
// cnt[item * waves + wave] = entries of that region; ovf[item] != 0 when a
// region of the item overflowed (the backward then regenerates that item).
constexpr int kEntFields = 6;
constexpr int kFwdMemoKeys = 128;      // largest key table per wave of the memoized forward
constexpr int kTableNodesDefault = 8192;
constexpr int kCkEntriesPerRay = 4;        // sweep checkpoints kept per ray (entry regions)
constexpr int kPoolMax = 8;                // per-hit forward: rounds of 64 rays per wave pool, at most
constexpr double kCkBudgetBytes = 128.0 * (1ull << 30);
constexpr int kTableNodesMax = 1 << 20;
struct AdjStore {
    double* ent;
    int32_t* cnt;
    int32_t* ovf;
    int64_t cap_w;
    int64_t total;
    int32_t waves;
    // Sweep checkpoints of the first ck_cap entries of every region, stored
    // by the FP64 forward solve (null: the adjoint recomputes them).  Entry
    // slot c (c = region * ck_cap + k) owns ck_blocks(Lmax) blocks of 8
    // doubles (64 bytes, written and read whole), block-major so that the
    // consecutive entries a wave solves or adjoins share lines: field f of
    // block g at ck[(g * ck_total + c) * 8 + f]; g = 0 holds v_0, g >= 1
    // v_{g kSegL}.
    double* ck;
    int64_t ck_cap;
    int64_t ck_total;
    // Order in which the entry kernel takes items (null: item order); set by
    // the backward, largest entry regions first.
    const int32_t* order;
};

struct SceneDev {
    // slab
    double T, Lx, ER;
    double px0, pw, ph;
    double ex0, ey0, ew, eh;
    int32_t bins_x, bins_y;
    // eye pupils (n_pupils > 0: bin p is pupil p, bins_x = n_pupils, bins_y = 1)
    int32_t n_pupils;
    double pupil_r2;                  // radius squared
    const double* pupil_xy;           // [n_pupils][2] centres
    // mirrors
    int32_t M;
    double nx, nz;                    // mirror normal (nx, 0, nz)
    double h[kMaxMirrors];            // plane offsets n . c_m
    uint32_t thr[kMaxMirrors];        // reflect iff word < thr
    double sc_r[kMaxMirrors];         // 1 / sqrt(p_eff)
    double sc_t[kMaxMirrors];         // 1 / sqrt(1 - p_eff)
    // stacks
    int32_t D, Lmax, n_slots;
    uint32_t slot_complex;            // bit s set: slot s is absorbing
    const double* thk;                // [D][M][Lmax]
    const uint8_t* slot;              // [D][M][Lmax]
    const int32_t* nlay;              // [D][M]
    // wavelengths and field
    int32_t n_lsel;
    const double* lam_tab;            // [n_lsel][LT_STRIDE]
    int32_t fov_mode, F;
    const double* dir_tab;            // [n_lsel][F][4]
    double fov_x0, fov_x1, fov_y0, fov_y1;  // random mode bounds, degrees
    int64_t N;                        // rays per point
    int64_t id_base;                  // added to a ray's id in its random stream (first_design n_lsel F N)
    int32_t Kmax;
    int32_t fp_shift;
    uint32_t key0, key1;              // Philox key (seed_lo, seed_hi ^ step)
    uint32_t seed_hi, step_host;      // with step_dev: key1 = seed_hi ^ (step_host + *step_dev)
    const uint32_t* step_dev;         // optional device step counter (graph replays)
    int32_t precision;
    int32_t memo;                     // forward: key table capacity per wave (0: solve every hit)
    int32_t pool;                     // forward: rounds of 64 rays per pool of a wave (per-hit solves; else 1)
    // angle table (table_n = 0: exact per-hit thin film)
    const double* table;              // [D][n_lsel][M][2 sides][table_n][8]
    int32_t table_n;
    unsigned long long* tab_scale;    // [maxG bits, cotangent pairs, maxD bits] (fixed-point scale)
    long long* tab_acc;               // backward: [D][n_lsel][M][2][2 branches][table_n][4]
    // work decomposition
    int64_t tiles_per_point;
    int64_t rays_per_tile;
    int64_t n_items;
    // forward: order in which items are taken (null: item order), and the
    // per-(item, wave) mirror-hit counts it records for the next forward's
    // order (null: none)
    const int32_t* fwd_order;
    int32_t* item_work;
};

}  // namespace gwg
