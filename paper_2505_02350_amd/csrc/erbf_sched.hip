// Training control of Algorithm 3 on the device: after each step, per
// shape, the effective basis count b_f (eq. add_activate), the rings of the
// last L2 values and b_f values, the decisions of Algorithm 3 in its order
// (pruning by eq. 3-27, L1 on by eq. l1_activate, kernel addition by eq.
// add_activate, the final L2 phase with its cosine learning rate, level
// requests) and the pruning itself.  Every decision is a deterministic
// function of the device state, so the control can run inside a captured
// step.  With a hold word, a call that leaves a request the caller will act
// on sets it, and calls that find it set (and the steps given it) change
// nothing until the caller clears it.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "erbf_device.h"
#include "erbf_internal.h"
#include "erbf_launch.h"

namespace erbf {

// b_f = #{ j < m : |w_j| >= tau_d } of each shape.  Also notes whether the
// call is held (its hold word set by an earlier call), before this call's
// decisions may set the word again.
__global__ __launch_bounds__(256) void k_sched_count(Dev D, const float* __restrict__ p,
                                                     const int32_t* __restrict__ m_dev, float tau_d,
                                                     int32_t* __restrict__ bf, const int32_t* __restrict__ hold) {
  __shared__ int sh[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int held = hold != nullptr && *hold != 0;
  if (tid == 0) D.sched_held[b] = held;
  if (held) return;
  const ShapeDev S = D.shapes[b];
  const int m = min(max(m_dev[b], 0), S.cap);
  int c = 0;
  for (int k = tid; k < m; k += 256) c += fabsf(p[S.kbase + k]) >= tau_d ? 1 : 0;
  c = wave_sum(c);
  if ((tid & 63) == 0) sh[tid >> 6] = c;
  __syncthreads();
  if (tid == 0) bf[b] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// One thread per shape: the bookkeeping of Algorithm 3 after step e.
__global__ __launch_bounds__(64) void k_sched_decide(Dev D, erbf_sched_state st, erbf_sched_cfg a,
                                                     const erbf_stats* __restrict__ stats) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= D.n_shapes) return;
  if (D.sched_held[b]) {
    // a held call: the state stays as the requesting call left it
    D.prune_flag[b] = 0;
    return;
  }
  const int e = st.epoch[b] + 1;
  int l1 = st.l1_active[b], fin = st.final_phase[b];
  int add = 0, ref = 0, prune = 0;
  double* l2r = st.l2_ring + (int64_t)b * a.k_l2;
  int32_t* bfr = st.bf_ring + (int64_t)b * a.k_l1;
  l2r[(e - 1) % a.k_l2] = stats[b].L2;
  bfr[(e - 1) % a.k_l1] = st.b_f[b];
  if (!fin) {
    if (e % a.k_l2 == 0 && l1 && e < a.T_e) prune = 1;
    if (!l1 && e >= a.k_l2) {
      // population standard deviation of the last k_l2 values (eq. l1_activate)
      double mean = 0.0;
      for (int i = 0; i < a.k_l2; ++i) mean += l2r[i];
      mean /= a.k_l2;
      double var = 0.0;
      for (int i = 0; i < a.k_l2; ++i) var += (l2r[i] - mean) * (l2r[i] - mean);
      if (sqrt(var / a.k_l2) < (double)a.tau_l2) l1 = 1;
    }
    if (l1 && e >= a.k_l1) {
      // spread of the last k_l1 basis counts (eq. add_activate)
      int mx = bfr[0], mn = bfr[0];
      for (int i = 1; i < a.k_l1; ++i) {
        mx = max(mx, bfr[i]);
        mn = min(mn, bfr[i]);
      }
      if ((float)(mx - mn) < a.tau_l1) {
        add = 1;
        l1 = 0;
      }
    }
  }
  if (e == a.T_e) {
    fin = 1;
    l1 = 0;
  }
  for (int i = 0; i < 4; ++i)
    if (a.refine_epochs[i] > 0 && e == a.refine_epochs[i]) ref = 1;
  double lr = a.lr0;
  if (fin) {
    const double frac = fmin(fmax((double)(e + 1 - a.T_e) / (double)(a.M_e - a.T_e), 0.0), 1.0);
    lr = a.lr_min + 0.5 * (a.lr_final - a.lr_min) * (1.0 + cos(3.14159265358979323846 * frac));
  }
  st.epoch[b] = e;
  st.l1_active[b] = l1;
  st.final_phase[b] = fin;
  st.add_request[b] = add;
  st.refine_request[b] = ref;
  st.lr[b] = (float)lr;
  D.prune_flag[b] = prune;
}

// With a hold word: a request the caller will act on -- kernels asked for
// while the shape has room and a non-empty id_all, or a grid level -- holds
// the caller's next steps (every such shape stores the same value).
__device__ __forceinline__ void sched_hold_after(const Dev& D, const erbf_sched_state& st, const erbf_stats* stats,
                                                 int b, int m_after) {
  if (!st.hold) return;
  const bool add = st.add_request[b] && m_after < D.shapes[b].cap && stats[b].n_idall > 0;
  if (add || st.refine_request[b]) *st.hold = 1;
}

// eq. 3-27 for the shapes whose flag is set: keep |w| >= tau_d in order,
// compacting parameters and Adam moments in place.  One block per shape;
// chunks of 1024 kernels are read completely before any of their kept
// entries is written, and a kept entry never moves up, so no unread
// entry is overwritten.  Then the hold word, from the live count after
// pruning.
__global__ __launch_bounds__(1024) void k_sched_prune(Dev D, float* __restrict__ p, int32_t* __restrict__ m_dev,
                                                      float* __restrict__ m1, float* __restrict__ m2, float tau_d,
                                                      erbf_sched_state st, const erbf_stats* __restrict__ stats) {
  __shared__ int sh[32];
  __shared__ int written;
  const int b = blockIdx.x, tid = threadIdx.x;
  int32_t* __restrict__ n_pruned = st.n_pruned;
  if (D.sched_held[b]) {
    if (tid == 0) n_pruned[b] = 0;
    return;
  }
  const ShapeDev S = D.shapes[b];
  if (!D.prune_flag[b]) {
    if (tid == 0) {
      n_pruned[b] = 0;
      sched_hold_after(D, st, stats, b, min(max(m_dev[b], 0), S.cap));
    }
    return;
  }
  const int C = D.cap_total;
  const int m = min(max(m_dev[b], 0), S.cap);
  if (tid == 0) written = 0;
  __syncthreads();
  for (int c0 = 0; c0 < m; c0 += 1024) {
    const int k = c0 + tid;
    const int j = S.kbase + k;
    const bool in = k < m;
    float vp[11], v1[11], v2[11];
#pragma unroll
    for (int seg = 0; seg < 11; ++seg) {
      vp[seg] = in ? p[seg * C + j] : 0.f;
      v1[seg] = in && m1 ? m1[seg * C + j] : 0.f;
      v2[seg] = in && m2 ? m2[seg * C + j] : 0.f;
    }
    const bool keep = in && fabsf(vp[0]) >= tau_d;
    int total;
    const int ex = block_excl_scan_1024(keep ? 1 : 0, sh, total);   // barriers: every read above is done
    if (keep) {
      const int dst = S.kbase + written + ex;
#pragma unroll
      for (int seg = 0; seg < 11; ++seg) {
        p[seg * C + dst] = vp[seg];
        if (m1) m1[seg * C + dst] = v1[seg];
        if (m2) m2[seg * C + dst] = v2[seg];
      }
    }
    __syncthreads();
    if (tid == 0) written += total;
    __syncthreads();
  }
  const int nm = written;
  // moments of the freed slots start from zero when the slots are reused
  for (int k = nm + tid; k < m; k += 1024)
    for (int seg = 0; seg < 11; ++seg) {
      if (m1) m1[seg * C + S.kbase + k] = 0.f;
      if (m2) m2[seg * C + S.kbase + k] = 0.f;
    }
  if (tid == 0) {
    m_dev[b] = nm;
    n_pruned[b] = m - nm;
    sched_hold_after(D, st, stats, b, nm);
  }
}

__global__ __launch_bounds__(64) void k_sched_init(Dev D, erbf_sched_state st, erbf_sched_cfg a) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= D.n_shapes) return;
  st.epoch[b] = 0;
  st.l1_active[b] = 0;
  st.final_phase[b] = 0;
  st.add_request[b] = 0;
  st.refine_request[b] = 0;
  st.b_f[b] = 0;
  st.n_pruned[b] = 0;
  st.lr[b] = a.lr0;
  for (int i = 0; i < a.k_l2; ++i) st.l2_ring[(int64_t)b * a.k_l2 + i] = 0.0;
  for (int i = 0; i < a.k_l1; ++i) st.bf_ring[(int64_t)b * a.k_l1 + i] = 0;
  D.prune_flag[b] = 0;
  if (b == 0 && st.hold) *st.hold = 0;
}

static inline unsigned nblk64(int n) { return (unsigned)((n + 63) / 64); }

hipError_t launch_sched_init(const Dev& D, const erbf_sched_state& st, const erbf_sched_cfg& a, hipStream_t s) {
  hipLaunchKernelGGL(k_sched_init, dim3(nblk64(D.n_shapes)), dim3(64), 0, s, D, st, a);
  return hipGetLastError();
}

hipError_t launch_sched_step(const Dev& D, const float* p_const, float* p, int32_t* m_dev, float* m1, float* m2,
                             const erbf_sched_state& st, const erbf_sched_cfg& a, const erbf_stats* stats,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_sched_count, dim3(D.n_shapes), dim3(256), 0, s, D, p_const, m_dev, a.tau_d, st.b_f,
                     st.hold);
  hipLaunchKernelGGL(k_sched_decide, dim3(nblk64(D.n_shapes)), dim3(64), 0, s, D, st, a, stats);
  hipLaunchKernelGGL(k_sched_prune, dim3(D.n_shapes), dim3(1024), 0, s, D, p, m_dev, m1, m2, a.tau_d, st, stats);
  return hipGetLastError();
}

}  // namespace erbf
