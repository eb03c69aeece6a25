// Launch wrappers of the HIP kernels (defined in gwg_kernels.hip), called by
// the host API only.
#pragma once
#include <hip/hip_runtime.h>
#include "gwg.h"
#include "gwg_internal.h"

namespace gwg {

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);

size_t fwd_smem_bytes(const SceneDev& sc, int wg, bool lds_bins);
size_t bwd_smem_bytes(const SceneDev& sc, int wg);
size_t tmm_smem_bytes(int L, int n_slots, int wg);
int64_t bwd_scratch_doubles(const SceneDev& sc, int64_t grid_blocks, int wg);

enum { KIND_FWD = 0, KIND_FWD_ADJ = 1, KIND_BWD_REGEN = 2, KIND_ADJ_ENTRIES = 3, KIND_ADJ_LOSSLESS = 4,
       KIND_ADJ_MEMO = 5, KIND_ADJ_MEMO_LOSSLESS = 6, KIND_TABLE_ACCUM = 7, KIND_FWD_TAB = 8, KIND_FWD_ADJ_TAB = 9,
       KIND_BWD_REGEN_TAB = 10, KIND_OMEGA = 11, KIND_FWD_MEMO = 12, KIND_FWD_ADJ_MEMO = 13 };
int trace_blocks_per_cu(int kind, int precision, int wg, size_t smem);
int64_t fwd_scratch_doubles(const SceneDev& sc, int64_t grid_blocks, int wg);
int64_t adj_scratch_doubles(const SceneDev& sc, int64_t grid_blocks, int wg);
hipError_t launch_trace_fwd(const SceneDev& sc, int wg, int grid_blocks, bool lds_bins, uint64_t* q, uint32_t* c,
                            unsigned long long* stats, gwg_ray_record* rec, int64_t rec_stride, double* scratch,
                            const AdjStore* adj, double* tape, hipStream_t s);
hipError_t launch_trace_bwd(const SceneDev& sc, int wg, int grid_blocks, const double* dLdI, unsigned long long* stats,
                            double* partial, double* scratch, int64_t sample_stride, const int32_t* regen,
                            hipStream_t s);
hipError_t launch_adj_entries(const SceneDev& sc, int wg, int grid_blocks, const double* dLdI,
                              unsigned long long* stats, double* partial, const AdjStore& st, double* scratch,
                              hipStream_t s);
size_t memo_smem_bytes(const SceneDev& sc);
hipError_t launch_adj_memo(const SceneDev& sc, int grid_blocks, const double* dLdI, unsigned long long* stats,
                           double* partial, const AdjStore& st, double* scratch, hipStream_t s);
hipError_t launch_table_build(const SceneDev& sc, double* tab, int n_cu, unsigned long long* stats, hipStream_t s);
hipError_t launch_absmax(const double* x, int64_t n, unsigned long long* out, hipStream_t s);
size_t table_accum_smem_bytes();
hipError_t launch_table_accum(const SceneDev& sc, int grid_blocks, const double* dLdI, const AdjStore& st, hipStream_t s);
int64_t table_adj_blocks(const SceneDev& sc);
size_t table_adj_smem_bytes(const SceneDev& sc);
hipError_t launch_table_adj(const SceneDev& sc, double* partial, double* scratch, unsigned long long* stats,
                            hipStream_t s);
hipError_t launch_table_reduce(const double* partial, const SceneDev& sc, double* grad, hipStream_t s);
size_t omega_smem_bytes(const SceneDev& sc, int wg);
hipError_t launch_omega_grad(const SceneDev& sc, int grid_blocks, int wg, const double* W, const uint32_t* counts,
                             double* partial, double* grad, hipStream_t s);
hipError_t launch_grad_reduce(const double* partial, int64_t items_per_design, int ML, int D, double* tmp,
                              double* grad, const int32_t* nlay, int M, int Lmax, hipStream_t s);
int64_t grad_reduce_tmp_doubles(int ML, int D);
hipError_t launch_item_order(const int32_t* cnt, int waves, int64_t n_items, int64_t max_count, int32_t* order,
                             hipStream_t s);
hipError_t launch_irradiance(const uint64_t* q, int64_t n, double scale, double* irr, hipStream_t s);
hipError_t launch_tmm_rt(int precision, const double* thk, const uint8_t* slot, int L,
                         const double* lam_tab, int n_lambda, int n_slots, uint32_t cplx_mask,
                         const int32_t* lidx, const double* theta, int64_t nq, double* out,
                         hipStream_t s);
hipError_t launch_loss(const double* I, int D, int nl, int F, int B, int kind, double w_f, double w_e,
                       double* work, double* loss, double* G, hipStream_t s);
// Doubles of work a loss of shape (D, nl, F, B) uses (launch_loss's work).
inline int64_t loss_work_doubles(int64_t D, int64_t nl, int64_t F, int64_t B)
{
    return D * nl * F + D * B + D * F + D * 8;
}
// Fixed-size device scratch of gwg_loss_noalloc (4 MiB per GPU).
constexpr int64_t kLossScratchDoubles = 1 << 19;
// Look up this device's scratch address (with `device` current); once per
// device, thread-safe.
hipError_t loss_scratch_setup(int device);
// The device address of `device`'s scratch, or null before its setup.
double* loss_scratch(int device);

}  // namespace gwg
