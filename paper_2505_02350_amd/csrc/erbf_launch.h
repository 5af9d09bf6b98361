// Launch wrappers between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "erbf_internal.h"

namespace erbf {

struct StatsArgs {
  int32_t mode;
  float lambda;
  const float* lambda_dev;
  int32_t l1_active;
  const int32_t* l1_active_dev;   // per-shape flags, or nullptr
  float tau_m;
  int32_t* step_inc;              // per-shape Adam step counters to increment with the statistics, or nullptr
  const int32_t* hold;            // [1] or nullptr: while non-zero the step counters stay as they are
};

struct AdamArgs {
  float lr;
  const float* lr_dev;
  float beta1, beta2, eps;
  const int32_t* hold;   // [1] or nullptr: while non-zero the pass changes nothing
};


hipError_t launch_scan(const int32_t* in, int n, int32_t* blocks, int32_t* out, int64_t* total,
                       hipStream_t s);
// kernel records, then the tile -> kernel lists
hipError_t launch_buckets(const Dev& D, const float* p, const int32_t* m_dev, int n_slots, hipStream_t s);
// `ev` (optional): start/stop events of each launched kernel, recorded at
// the kernel's own start and end (forward: 2 events; backward: 4).
// with_bwd: the grid tiles' backward moments are formed by the same kernel
// (the fused step kernel, for the loss); launch_backward then skips its tile
// kernel (tiles_done).
hipError_t launch_forward(const Dev& D, int n_slots, bool loss, float* f_out, float tau1, float tau2,
                          const hipEvent_t* ev, hipStream_t s, bool with_bwd = false);
// With timing events ev (backward tiles' start/stop, reduce's start/stop):
// when fwd_stop is the stop event of a forward launched just before, a
// kernel that directly follows the previous timed kernel takes that
// kernel's stop event as its start (bit 0 of *shared: the tiles start at
// fwd_stop; bit 1: the reduce starts at the tiles' stop), so fewer events
// sit between the kernels.
hipError_t launch_backward(const Dev& D, int n_slots, const float* p, const float* G, float* grad,
                           const hipEvent_t* ev, hipStream_t s, bool tiles_done = false,
                           hipEvent_t fwd_stop = nullptr, uint8_t* shared = nullptr);
// mode 2 with apply = false leaves the L2 gradient in grad (the combine then
// runs in launch_adam with combine = true)
hipError_t launch_stats(const Dev& D, int mode, const float* p, const int32_t* m_dev, float* grad,
                        erbf_stats* out, const StatsArgs& a, hipStream_t s, bool apply = true);
hipError_t launch_adam(const Dev& D, float* p, const int32_t* m_dev, float* g, float* m1, float* m2,
                       int32_t* step, const AdamArgs& a, bool combine, hipStream_t s);
hipError_t launch_mask_copy(const Dev& D, int li, int64_t npts, const float* src, hipStream_t s);
hipError_t launch_fill_f32(float* x, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_targets(const float* S, int64_t n, float m, float* t, hipStream_t s);
hipError_t launch_band_bits(const float* S, int64_t n, float band, uint32_t* bits, hipStream_t s);
hipError_t launch_octree_bits(const float* Sp, const uint32_t* pbits, int np, uint32_t* bits, hipStream_t s);
hipError_t launch_sdf_min(const float* S, int64_t n, float* out, int accumulate, int* key_scratch,
                          hipStream_t s);
hipError_t launch_tile_flags(const Dev& D, int li, int ntt, int32_t* flags, hipStream_t s);
hipError_t launch_tile_assign(const Dev& D, int li, int ntt, const int32_t* flags, const int32_t* excl,
                              int slot0, hipStream_t s);
hipError_t launch_seed_select(const Dev& D, int shape, int64_t npts, const float* resid, float scale,
                              float floor_abs, float r_nms, int64_t k_cand, hipStream_t s);
// counts left by launch_seed_select (synchronises the stream); 0 on success
int seed_misc_counts(const Dev& D, int32_t* n_cand, int32_t* n_kept, hipStream_t s);
// dbar (eq. 3-24) from the nearest sample of the listed sample levels (level
// table index and registered count each) when any holds a sample, else |S|
hipError_t launch_seed_write(const Dev& D, int shape, int n_add, float* p, int32_t* m_dev, const float* resid,
                             float scale, float* m1, float* m2, float eps, int w_rule, float h_fine,
                             const int* samp_levels, const int64_t* samp_counts, int n_samp_levels, hipStream_t s);
// marks (1) the slots holding the batch's points in sel, after clearing it
hipError_t launch_batch_tiles(const Dev& D, int n_slots, const int64_t* pts, int n_pts, int32_t* sel, hipStream_t s);
hipError_t launch_batch_step(const Dev& D, int n_slots, const int64_t* pts, int n_pts, const float* p,
                             const int32_t* m_dev, float* grad, float* f_out, erbf_stats* out, float tau1, float tau2,
                             const StatsArgs& a, hipStream_t s);
hipError_t launch_init_inscribed(const Dev& D, int shape, uint32_t npts, bool samples, int m_max, int cap, float gamma,
                                 float* p, int32_t* m_dev, float* m1, float* m2, hipStream_t s);
// (centres, uncovered candidates) left by launch_init_inscribed (synchronises the stream); 0 on success
int init_results(const Dev& D, int32_t* n_centres, int64_t* n_left, hipStream_t s);
// counts per cube and their 64-bit total (*total64 must start at 0)
hipError_t launch_mt_count(const float* F, const float* ax, int n, float iso, int32_t* cnt, int64_t* total64,
                           hipStream_t s);
hipError_t launch_mt_emit(const float* F, const float* ax, int n, float iso, const int32_t* off, float* tris,
                          int64_t cap, hipStream_t s);
hipError_t launch_surface_sample(const float* tris, int64_t nt, const float* u, int64_t ns, double* area, float* pts,
                                 float* nrm, int32_t* which, hipStream_t s);
hipError_t launch_surface_metrics(const float* Pt, const float* Nt, int64_t nt, const float* Pr, const float* Nr,
                                  int64_t nr, double* scratch, double* out, hipStream_t s);
hipError_t launch_sdf_from_targets(const float* t, int64_t n, float m, float* S, hipStream_t s);
// ranked tile lists (atomic placement, per-tile bitmap ranks): shape
// capacities up to this many kernel slots
constexpr int kRankMaxCap = 32768;
// erbf_surface_metrics_noalloc: at most this many points over both sets
constexpr int64_t kNoallocMetricsPoints = (int64_t)1 << 20;
// device address of the metrics scratch on the current device (looked up on
// the first call on each device)
hipError_t noalloc_metrics_scratch(double** out);
hipError_t launch_sched_init(const Dev& D, const erbf_sched_state& st, const erbf_sched_cfg& a, hipStream_t s);
hipError_t launch_sched_step(const Dev& D, const float* p_const, float* p, int32_t* m_dev, float* m1, float* m2,
                             const erbf_sched_state& st, const erbf_sched_cfg& a, const erbf_stats* stats,
                             hipStream_t s);

}  // namespace erbf
