// Seeding new kernels at local maxima of the residual (Algorithm 2 with
// eq. 3-22, 3-24 and 3-25), for one shape.
//
//   1. candidates: the K = ceil(top_frac * n_idall) points with the largest
//      |E|, ties to the lower index.  Every point gets the unique 64-bit key
//      ((~bits|E|) << 32 | index), so "largest |E|, then lowest index" is
//      "smallest key"; a four-digit radix select finds the K-th smallest key
//      without sorting.  Candidates also need |E| > max(min_abs_err, eps).
//      Surface samples are not candidates (a centre on a sample has
//      distance 0 to P, where eq. 3-24 gives no scale).
//   2. extreme points: a candidate survives if no point of V within r_nms
//      (grid points of any active level of the shape, and its registered
//      surface samples) has a larger |E|.  Points outside id_all have E = 0
//      and cannot suppress anything.
//   3. the first k_new survivors by key (a second radix select, then one
//      sorted block).
//   4. eq. 3-24 parameters, appended after the shape's live kernels; their
//      Adam moments are cleared.  dbar is the distance from the centre to
//      the nearest registered sample (the minimum of the squared distances
//      is exact whatever the order, so atomics give the same result), or
//      |S| at the centre when the shape has no sample registered; in both
//      cases at least the finest grid spacing.
// Lists are built with atomics but every result is defined by the keys, so
// the outcome does not depend on the order of the atomics.

#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <stdint.h>

#include "erbf_internal.h"
#include "erbf_launch.h"

namespace erbf {

namespace {

constexpr int kHist = 65536;

__device__ __forceinline__ uint64_t point_key(float e, uint32_t index) {
  const uint32_t b = __float_as_uint(fabsf(e));
  return ((uint64_t)(~b) << 32) | index;
}

// misc layout (int32 words of seed_misc):
//   [0..1]  prefix (uint64) of the radix select
//   [2..3]  k remaining (int64)
//   [4]     candidate count
//   [5]     kept count
//   [6]     selected count
//   [8..9]  final threshold key (uint64)
struct SeedMisc {
  uint64_t prefix;
  int64_t k_rem;
  int32_t n_cand, n_kept, n_sel, pad;
  uint64_t thresh;
};

// digit d (0 = most significant 16 bits) of a key
__device__ __forceinline__ uint32_t digit(uint64_t k, int d) { return (uint32_t)(k >> (48 - 16 * d)) & 0xffffu; }

__device__ __forceinline__ bool prefix_match(uint64_t k, uint64_t prefix, int d) {
  if (d == 0) return true;
  const int sh = 64 - 16 * d;
  return (k >> sh) == (prefix >> sh);
}

// residual of shape-local point i for seeding: surface samples are not
// seeded (their entries read as 0)
__device__ __forceinline__ float seed_resid(const Dev& D, const ShapeDev& S, const float* __restrict__ resid,
                                            int64_t i, bool samples) {
  if (samples) {
    int64_t off = 0;
    for (int li = 0; li < S.n_active; ++li) {
      const LevelDev& L = D.levels[S.lvl0 + li];
      if (i < off + L.npts) {
        if (L.kind != kLevelGrid) return 0.f;
        break;
      }
      off += L.npts;
    }
  }
  return resid[S.pt_base + i];
}

// histogram pass over the shape's points
__global__ __launch_bounds__(256) void k_sel_hist_points(Dev D, int shape, const float* __restrict__ resid,
                                                         int d) {
  const ShapeDev S = D.shapes[shape];
  const SeedMisc* M = reinterpret_cast<const SeedMisc*>(D.seed_misc);
  const uint64_t prefix = M->prefix;
  // points of the active levels are contiguous from S.pt_base
  int64_t npts = 0;
  bool samples = false;
  for (int li = 0; li < S.n_active; ++li) {
    const LevelDev L = D.levels[S.lvl0 + li];
    npts += L.npts;
    samples |= L.kind != kLevelGrid;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = point_key(seed_resid(D, S, resid, i, samples), (uint32_t)i);
    if (prefix_match(k, prefix, d)) atomicAdd(&D.seed_hist[digit(k, d)], 1u);
  }
}

// histogram pass over a materialised key list
__global__ __launch_bounds__(256) void k_sel_hist_list(Dev D, const uint64_t* __restrict__ keys, int d) {
  const SeedMisc* M = reinterpret_cast<const SeedMisc*>(D.seed_misc);
  const uint64_t prefix = M->prefix;
  const int n = M->n_kept;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    if (prefix_match(k, prefix, d)) atomicAdd(&D.seed_hist[digit(k, d)], 1u);
  }
}

// one workgroup: find the digit where the running count reaches k_rem, extend
// the prefix, and clear the histogram for the next pass
__global__ __launch_bounds__(1024) void k_sel_pick(Dev D, int d) {
  __shared__ uint32_t part[1024];
  __shared__ int found_bin;
  __shared__ uint32_t below;
  SeedMisc* M = reinterpret_cast<SeedMisc*>(D.seed_misc);
  const int tid = threadIdx.x;
  const int64_t k_rem = M->k_rem;
  // each thread sums 64 consecutive bins
  uint32_t s = 0;
  for (int b = 0; b < 64; ++b) s += D.seed_hist[tid * 64 + b];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    uint64_t run = 0;
    int chunk = -1;
    for (int c = 0; c < 1024; ++c) {
      if (run + part[c] >= (uint64_t)k_rem) { chunk = c; break; }
      run += part[c];
    }
    int bin = kHist - 1;
    if (chunk >= 0) {
      for (int b = chunk * 64; b < chunk * 64 + 64; ++b) {
        if (run + D.seed_hist[b] >= (uint64_t)k_rem) { bin = b; break; }
        run += D.seed_hist[b];
      }
    }
    found_bin = bin;
    below = (uint32_t)run;
  }
  __syncthreads();
  if (tid == 0) {
    const int sh = 48 - 16 * d;
    const uint64_t keep_hi = d == 0 ? 0ull : (M->prefix >> (sh + 16)) << (sh + 16);
    M->prefix = keep_hi | ((uint64_t)found_bin << sh);
    M->k_rem = k_rem - below;
  }
  for (int b = tid; b < kHist; b += 1024) D.seed_hist[b] = 0u;
}

// candidates: key <= threshold and |E| above the floor
__global__ __launch_bounds__(256) void k_collect_cand(Dev D, int shape, const float* __restrict__ resid, float scale,
                                                      float floor_abs) {
  const ShapeDev S = D.shapes[shape];
  SeedMisc* M = reinterpret_cast<SeedMisc*>(D.seed_misc);
  const uint64_t T = M->prefix;
  int64_t npts = 0;
  bool samples = false;
  for (int li = 0; li < S.n_active; ++li) {
    const LevelDev L = D.levels[S.lvl0 + li];
    npts += L.npts;
    samples |= L.kind != kLevelGrid;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (int64_t)gridDim.x * blockDim.x) {
    const float r = seed_resid(D, S, resid, i, samples);
    const uint64_t k = point_key(r, (uint32_t)i);
    if (k <= T && fabsf(r * scale) > floor_abs) {
      const int at = atomicAdd(&M->n_cand, 1);
      if (at < D.cand_cap) D.seed_cand[at] = (int64_t)i;
    }
  }
}

// locate a shape-local point index: level, grid indices
__device__ __forceinline__ int locate(const Dev& D, const ShapeDev& S, int64_t g, int& li_out, int& i, int& j,
                                      int& k) {
  int64_t off = 0;
  for (int li = 0; li < S.n_active; ++li) {
    const LevelDev L = D.levels[S.lvl0 + li];
    const int64_t np = L.npts;
    if (g < off + np) {
      if (L.kind != kLevelGrid) return 0;
      const int64_t loc = g - off;
      li_out = S.lvl0 + li;
      i = (int)(loc % L.n);
      j = (int)((loc / L.n) % L.n);
      k = (int)(loc / ((int64_t)L.n * L.n));
      return 1;
    }
    off += np;
  }
  return 0;
}

// Does a registered sample of sample level L within r_nms of (xi, yi, zi)
// have a larger |E| than ei?  The samples are binned into the 8^3-cell tiles
// of the level's n^3-cell grid; the tiles meeting the neighbourhood's box
// (widened by a cell) are searched.
__device__ bool sample_suppresses(const Dev& D, const LevelDev& L, const float* __restrict__ resid, float xi,
                                  float yi, float zi, float r_nms, float r2, float ei) {
  if (L.n_samples <= 0) return false;
  const int n = L.n, nt = L.nt;
  const float inv = 1.0f / L.h;
  const int cx0 = max(0, (int)floorf((xi - r_nms + 1.f) * inv) - 1), cx1 = min(n - 1, (int)floorf((xi + r_nms + 1.f) * inv) + 1);
  const int cy0 = max(0, (int)floorf((yi - r_nms + 1.f) * inv) - 1), cy1 = min(n - 1, (int)floorf((yi + r_nms + 1.f) * inv) + 1);
  const int cz0 = max(0, (int)floorf((zi - r_nms + 1.f) * inv) - 1), cz1 = min(n - 1, (int)floorf((zi + r_nms + 1.f) * inv) + 1);
  for (int tz = cz0 / kTile; tz <= cz1 / kTile; ++tz)
    for (int ty = cy0 / kTile; ty <= cy1 / kTile; ++ty)
      for (int tx = cx0 / kTile; tx <= cx1 / kTile; ++tx) {
        const int slot = D.tile_map[L.tmap0 + (tz * nt + ty) * nt + tx];
        if (slot < 0) continue;
        const int s0 = L.sstart[slot - L.slot0], s1 = L.sstart[slot - L.slot0 + 1];
        for (int q = s0; q < s1; ++q) {
          const float4 P = L.spos[q];
          const float dx = P.x - xi, dy = P.y - yi, dz = P.z - zi;
          if (dx * dx + dy * dy + dz * dz > r2) continue;
          if (fabsf(resid[L.pt_base + __float_as_int(P.w)]) > ei) return true;
        }
      }
  return false;
}

// extreme-point test of each candidate; survivors' keys go to the keep list
__global__ __launch_bounds__(256) void k_nms(Dev D, int shape, const float* __restrict__ resid, float r_nms) {
  const ShapeDev S = D.shapes[shape];
  SeedMisc* M = reinterpret_cast<SeedMisc*>(D.seed_misc);
  const int nc = min((int64_t)M->n_cand, D.cand_cap);
  const float r2 = r_nms * r_nms;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    const int64_t g = D.seed_cand[c];
    int li, i, j, k;
    if (!locate(D, S, g, li, i, j, k)) continue;
    const float ei = fabsf(resid[S.pt_base + g]);
    const LevelDev Lc = D.levels[li];
    const float xi = Lc.axis[i], yi = Lc.axis[j], zi = Lc.axis[k];
    bool ok = true;
    int64_t off = 0;
    for (int l = 0; l < S.n_active && ok; ++l) {
      const LevelDev L = D.levels[S.lvl0 + l];
      const int n = L.n;
      if (L.kind != kLevelGrid) {
        if (!sample_suppresses(D, L, resid, xi, yi, zi, r_nms, r2, ei)) {
          off += L.npts;
          continue;
        }
        ok = false;
        break;
      }
      // conservative index ranges, then the exact distance test
      int x0 = max(0, (int)floorf((xi - r_nms - L.lo) / L.h) - 1), x1 = min(n - 1, (int)ceilf((xi + r_nms - L.lo) / L.h) + 1);
      int y0 = max(0, (int)floorf((yi - r_nms - L.lo) / L.h) - 1), y1 = min(n - 1, (int)ceilf((yi + r_nms - L.lo) / L.h) + 1);
      int z0 = max(0, (int)floorf((zi - r_nms - L.lo) / L.h) - 1), z1 = min(n - 1, (int)ceilf((zi + r_nms - L.lo) / L.h) + 1);
      for (int zz = z0; zz <= z1 && ok; ++zz) {
        const float dz = L.axis[zz] - zi;
        for (int yy = y0; yy <= y1 && ok; ++yy) {
          const float dy = L.axis[yy] - yi;
          const float dyz = dy * dy + dz * dz;
          if (dyz > r2) continue;
          for (int xx = x0; xx <= x1; ++xx) {
            const float dx = L.axis[xx] - xi;
            if (dx * dx + dyz > r2) continue;
            const float ek = fabsf(resid[S.pt_base + off + ((int64_t)zz * n + yy) * n + xx]);
            if (ek > ei) { ok = false; break; }
          }
        }
      }
      off += L.npts;
    }
    if (ok) {
      const int at = atomicAdd(&M->n_kept, 1);
      reinterpret_cast<uint64_t*>(D.seed_keep)[at] = point_key(resid[S.pt_base + g], (uint32_t)g);
    }
  }
}

// keys <= threshold (exactly the k_new smallest) into the selection buffer
__global__ __launch_bounds__(256) void k_collect_sel(Dev D) {
  SeedMisc* M = reinterpret_cast<SeedMisc*>(D.seed_misc);
  const uint64_t T = M->prefix;
  const int n = M->n_kept;
  const uint64_t* keys = reinterpret_cast<const uint64_t*>(D.seed_keep);
  uint64_t* sel = reinterpret_cast<uint64_t*>(D.seed_cand);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (keys[i] <= T) {
      const int at = atomicAdd(&M->n_sel, 1);
      sel[at] = keys[i];
    }
  }
}

// one workgroup: sort the selection by key (ascending: largest |E| first,
// ties to the lower index) in place, and clear the squared nearest-sample
// distances
__global__ __launch_bounds__(1024) void k_seed_sort(Dev D, int n_add) {
  __shared__ uint64_t buf[4096];
  uint64_t* sel = reinterpret_cast<uint64_t*>(D.seed_cand);
  uint32_t* dmin2 = reinterpret_cast<uint32_t*>(D.seed_keep);
  const int tid = threadIdx.x;
  int pw = 1;
  while (pw < n_add) pw <<= 1;
  for (int i = tid; i < pw; i += 1024) buf[i] = i < n_add ? sel[i] : ~0ull;
  __syncthreads();
  for (int k = 2; k <= pw; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = tid; i < pw; i += 1024) {
        const int ixj = i ^ jj;
        if (ixj > i) {
          const uint64_t a = buf[i], b = buf[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) { buf[i] = b; buf[ixj] = a; }
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n_add; i += 1024) {
    sel[i] = buf[i];
    dmin2[i] = __float_as_uint(INFINITY);
  }
}

// squared distance from each new centre to its nearest registered sample of
// the shape: blocks take slices of a sample level's samples (staged in LDS)
// and the centres; the minimum goes through an unsigned atomic min on the
// float bits (non-negative floats order as their bits), exact in any order
__global__ __launch_bounds__(256) void k_seed_dbar(Dev D, int shape, int li, int n_add) {
  __shared__ float4 sp[256];
  const ShapeDev S = D.shapes[shape];
  const LevelDev L = D.levels[li];
  const uint64_t* sel = reinterpret_cast<const uint64_t*>(D.seed_cand);
  uint32_t* dmin2 = reinterpret_cast<uint32_t*>(D.seed_keep);
  const int tid = threadIdx.x;
  const int64_t ns = L.n_samples;
  for (int64_t q0 = (int64_t)blockIdx.x * 256; q0 < ns; q0 += (int64_t)gridDim.x * 256) {
    const int nq = (int)min((int64_t)256, ns - q0);
    __syncthreads();   // the previous slice is no longer read
    if (tid < nq) sp[tid] = L.spos[q0 + tid];
    __syncthreads();
    for (int r = blockIdx.y * 256 + tid; r < n_add; r += gridDim.y * 256) {
      const int64_t g = (int64_t)(uint32_t)(sel[r] & 0xffffffffull);
      int lc, i, j, k;
      if (!locate(D, S, g, lc, i, j, k)) continue;
      const LevelDev Lc = D.levels[lc];
      const float cx = Lc.axis[i], cy = Lc.axis[j], cz = Lc.axis[k];
      float best = INFINITY;
      for (int q = 0; q < nq; ++q) {
        const float dx = sp[q].x - cx, dy = sp[q].y - cy, dz = sp[q].z - cz;
        best = fminf(best, dx * dx + dy * dy + dz * dz);
      }
      atomicMin(&dmin2[r], __float_as_uint(best));
    }
  }
}

// eq. 3-24 parameters of the sorted selection, appended after the live kernels
__global__ __launch_bounds__(256) void k_seed_write(Dev D, int shape, float* __restrict__ p,
                                                    const int32_t* __restrict__ m_dev, const float* __restrict__ resid,
                                                    float scale, float* __restrict__ m1, float* __restrict__ m2,
                                                    float eps, int w_rule, float h_fine, int n_add, int use_samples) {
  const ShapeDev S = D.shapes[shape];
  const uint64_t* sel = reinterpret_cast<const uint64_t*>(D.seed_cand);
  const uint32_t* dmin2 = reinterpret_cast<const uint32_t*>(D.seed_keep);
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n_add) return;
  const int m = m_dev[shape];
  const int C = D.cap_total;
  const int64_t g = (int64_t)(uint32_t)(sel[r] & 0xffffffffull);
  int li, i, j, k;
  locate(D, S, g, li, i, j, k);
  const LevelDev L = D.levels[li];
  const float E = resid[S.pt_base + g] * scale;
  const float aE = fabsf(E);
  const float sg = E > 0.f ? 1.f : (E < 0.f ? -1.f : 0.f);
  const float w = w_rule == 0 ? -sg * aE : -sg * sqrtf(aE);
  const float dist = use_samples ? sqrtf(__uint_as_float(dmin2[r])) : fabsf(L.sdf[((int64_t)k * L.n + j) * L.n + i]);
  const float dbar = fmaxf(dist, h_fine);
  const float dd = sqrtf(logf(aE / eps)) / dbar;
  const float s = logf(dd);
  const int slot = S.kbase + m + r;
  p[slot] = w;
  p[C + slot] = L.axis[i];
  p[2 * C + slot] = L.axis[j];
  p[3 * C + slot] = L.axis[k];
  p[4 * C + slot] = s;
  p[5 * C + slot] = s;
  p[6 * C + slot] = s;
  p[7 * C + slot] = D.orientation == ERBF_ORIENT_EULER ? 0.f : 1.f;   // identity rotation
  p[8 * C + slot] = 0.f;
  p[9 * C + slot] = 0.f;
  p[10 * C + slot] = 0.f;
  for (int seg = 0; seg < 11; ++seg) {
    if (m1) m1[seg * C + slot] = 0.f;
    if (m2) m2[seg * C + slot] = 0.f;
  }
}

// the shape's live count grows by the appended kernels
__global__ void k_seed_count(int32_t* m_dev, int shape, int n_add) { m_dev[shape] += n_add; }

__global__ __launch_bounds__(1024) void k_fill_u32_hist(Dev D) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kHist; i += gridDim.x * blockDim.x) D.seed_hist[i] = 0u;
}

__global__ void k_seed_init(Dev D, int64_t k) {
  SeedMisc* M = reinterpret_cast<SeedMisc*>(D.seed_misc);
  M->prefix = 0;
  M->k_rem = k;
  M->n_cand = 0;
  M->n_kept = 0;
  M->n_sel = 0;
  M->thresh = 0;
}

__global__ void k_seed_reset_select(Dev D, int64_t k) {
  SeedMisc* M = reinterpret_cast<SeedMisc*>(D.seed_misc);
  M->prefix = 0;
  M->k_rem = k;
}

inline unsigned gs(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

}  // namespace

int seed_misc_counts(const Dev& D, int32_t* n_cand, int32_t* n_kept, hipStream_t s) {
  SeedMisc m;
  if (hipMemcpyAsync(&m, D.seed_misc, sizeof(SeedMisc), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  *n_cand = m.n_cand;
  *n_kept = m.n_kept;
  return 0;
}

// Stage 1-2: candidates and extreme points.  Leaves counts in seed_misc.
hipError_t launch_seed_select(const Dev& D, int shape, int64_t npts, const float* resid, float scale,
                              float floor_abs, float r_nms, int64_t k_cand, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_init, dim3(1), dim3(1), 0, s, D, k_cand);
  hipLaunchKernelGGL(k_fill_u32_hist, dim3(64), dim3(1024), 0, s, D);
  for (int d = 0; d < 4; ++d) {
    hipLaunchKernelGGL(k_sel_hist_points, dim3(gs(npts)), dim3(256), 0, s, D, shape, resid, d);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1024), 0, s, D, d);
  }
  hipLaunchKernelGGL(k_collect_cand, dim3(gs(npts)), dim3(256), 0, s, D, shape, resid, scale, floor_abs);
  hipLaunchKernelGGL(k_nms, dim3(gs(D.cand_cap)), dim3(256), 0, s, D, shape, resid, r_nms);
  return hipGetLastError();
}

// Stage 3-4: the first n_add survivors by key, written as new kernels.
hipError_t launch_seed_write(const Dev& D, int shape, int n_add, float* p, int32_t* m_dev, const float* resid,
                             float scale, float* m1, float* m2, float eps, int w_rule, float h_fine,
                             const int* samp_levels, const int64_t* samp_counts, int n_samp_levels, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_reset_select, dim3(1), dim3(1), 0, s, D, (int64_t)n_add);
  const uint64_t* keys = reinterpret_cast<const uint64_t*>(D.seed_keep);
  for (int d = 0; d < 4; ++d) {
    hipLaunchKernelGGL(k_sel_hist_list, dim3(gs(D.cand_cap)), dim3(256), 0, s, D, keys, d);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1024), 0, s, D, d);
  }
  hipLaunchKernelGGL(k_collect_sel, dim3(gs(D.cand_cap)), dim3(256), 0, s, D);
  hipLaunchKernelGGL(k_seed_sort, dim3(1), dim3(1024), 0, s, D, n_add);
  int use_samples = 0;
  for (int a = 0; a < n_samp_levels; ++a) {
    if (samp_counts[a] <= 0) continue;
    use_samples = 1;
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((samp_counts[a] + 255) / 256, 2048));
    const unsigned gy = (unsigned)((n_add + 255) / 256);
    hipLaunchKernelGGL(k_seed_dbar, dim3(gx, gy), dim3(256), 0, s, D, shape, samp_levels[a], n_add);
  }
  hipLaunchKernelGGL(k_seed_write, dim3((n_add + 255) / 256), dim3(256), 0, s, D, shape, p, m_dev, resid, scale, m1,
                     m2, eps, w_rule, h_fine, n_add, use_samples);
  hipLaunchKernelGGL(k_seed_count, dim3(1), dim3(1), 0, s, m_dev, shape, n_add);
  return hipGetLastError();
}

}  // namespace erbf
