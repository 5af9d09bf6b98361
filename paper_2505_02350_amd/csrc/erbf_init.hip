// Inscribed-sphere initialisation of one shape (Algorithm 1 with eq. 3-11
// and eq. 3-12).
//
// Candidates are the interior training points of the shape's registered
// levels: 1 < target < 2 (eq. 3-10).  Each round takes the candidate with the
// largest |S| (its distance to the surface; ties to the lower point index) as
// a centre whose weight is its target and whose sphere radius is r = |S|, and
// drops every candidate within distance r of it.  Rounds repeat until no
// candidate is left or the centre limit is reached.
//
// The rounds depend on each other, so they run in one workgroup.  The
// candidates are a bit mask over the shape's points, and the workgroup keeps
// the list of mask words that still hold a candidate: a round costs the live
// words, not the grid.  One round is one pass over the live words that both
// removes the last centre's sphere and finds the next centre, with one
// barrier.  Distances are compared in double precision with every product
// and sum rounded on its own (no fused multiply-add), as
// ((dx*dx + dy*dy) + dz*dz) <= r*r, so the chosen centres are reproducible
// exactly by a float64 evaluation of the same expression.
//
// With surface samples registered for the shape (sample levels), the
// distance to the surface is, as in the algorithm, the distance to the
// nearest sample: its square r^2 (double, each operation rounded) is the
// sphere's squared radius and, rounded to float, the depth order.
//
// eq. 3-12 then gives each centre the isotropic scale
// d = 2 sqrt(-ln(gamma / w^2)) / dhat, dhat the distance to the nearest other
// centre (2, the width of the domain, when there is a single centre), and the
// identity rotation.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "erbf_device.h"
#include "erbf_internal.h"
#include "erbf_launch.h"

namespace erbf {

namespace {

// scratch of the initialisation: nearest-sample squared distances (double,
// per shape point), candidate mask, two candidate lists, result words
__device__ __forceinline__ double* init_dmin2(const Dev& D) { return reinterpret_cast<double*>(D.init_scratch); }
__device__ __forceinline__ uint32_t* init_mask(const Dev& D) { return D.init_scratch + 2 * D.init_cand_cap; }
__device__ __forceinline__ uint32_t* init_list(const Dev& D, int which) {
  return init_mask(D) + D.init_words + which * D.init_cand_cap;
}
__device__ __forceinline__ uint32_t* init_res(const Dev& D) { return init_list(D, 2); }

// level and grid indices of a shape-local point index (the shape's active
// levels are contiguous, each x fastest); the shape has < 2^32 points.  For
// a point of a sample level only the level is meaningful.
__device__ __forceinline__ const LevelDev* init_locate(const Dev& D, const ShapeDev& S, uint32_t g, uint32_t& loc,
                                                       int& i, int& j, int& k) {
  uint32_t off = 0;
  int l = 0;
  for (; l < S.n_active - 1; ++l) {
    const uint32_t np = (uint32_t)D.levels[S.lvl0 + l].npts;
    if (g - off < np) break;
    off += np;
  }
  const LevelDev* L = &D.levels[S.lvl0 + l];
  const uint32_t n = (uint32_t)L->n;
  loc = g - off;
  i = (int)(loc % n);
  j = (int)((loc / n) % n);
  k = (int)(loc / (n * n));
  return L;
}

// squared distance with each operation rounded separately
__device__ __forceinline__ double dist2_rounded(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  const double xx = dx * dx;
  const double yy = dy * dy;
  const double zz = dz * dz;
  return (xx + yy) + zz;
}

// candidate mask: bit b of word w is point 32 w + b of the shape
__global__ __launch_bounds__(256) void k_init_mark(Dev D, int shape, uint32_t npts, uint32_t nw) {
  const ShapeDev S = D.shapes[shape];
  uint32_t* mask = init_mask(D);
  for (uint32_t w = blockIdx.x * 256u + threadIdx.x; w < nw; w += gridDim.x * 256u) {
    uint32_t word = 0u;
    for (int b = 0; b < 32; ++b) {
      const uint32_t g = w * 32u + (uint32_t)b;
      if (g >= npts) break;
      uint32_t loc;
      int i, j, k;
      const LevelDev* L = init_locate(D, S, g, loc, i, j, k);
      if (L->kind != kLevelGrid) continue;   // samples are on the surface, never interior
      const bool act = !L->bits || ((L->bits[loc >> 5] >> (loc & 31u)) & 1u);
      const float t = L->target[loc];
      const float sv = L->sdf[loc];
      if (act && t > 1.0f && t < 2.0f && isfinite(sv)) word |= 1u << b;
    }
    mask[w] = word;
  }
}

// nearest-sample squared distance of every candidate: blocks of 256 points
// stream the shape's samples through LDS; blocks without a candidate leave
__global__ __launch_bounds__(256) void k_init_nearest(Dev D, int shape, uint32_t npts) {
  __shared__ float4 sp[256];
  const ShapeDev S = D.shapes[shape];
  const uint32_t g = blockIdx.x * 256u + threadIdx.x;
  const uint32_t* mask = init_mask(D);
  const bool cand = g < npts && ((mask[g >> 5] >> (g & 31u)) & 1u);
  if (!__syncthreads_or(cand ? 1 : 0)) return;
  double px = 0.0, py = 0.0, pz = 0.0;
  if (cand) {
    uint32_t loc;
    int i, j, k;
    const LevelDev* L = init_locate(D, S, g, loc, i, j, k);
    px = (double)L->axis[i];
    py = (double)L->axis[j];
    pz = (double)L->axis[k];
  }
  double best = INFINITY;
  for (int l = 0; l < S.n_active; ++l) {
    const LevelDev& L = D.levels[S.lvl0 + l];
    if (L.kind != kLevelSamples) continue;
    for (int s0 = 0; s0 < L.n_samples; s0 += 256) {
      const int q = s0 + (int)threadIdx.x;
      __syncthreads();
      if (q < L.n_samples) sp[threadIdx.x] = make_float4(L.sxyz[3 * q], L.sxyz[3 * q + 1], L.sxyz[3 * q + 2], 0.f);
      __syncthreads();
      const int nq = min(256, L.n_samples - s0);
      if (cand)
        for (int u = 0; u < nq; ++u) {
          const float4 P = sp[u];
          best = fmin(best, dist2_rounded((double)P.x - px, (double)P.y - py, (double)P.z - pz));
        }
    }
  }
  if (cand) init_dmin2(D)[g] = best;
}

// agent-scope load: bypasses this CU's vector cache, so it sees bits that
// other waves cleared with atomics
__device__ __forceinline__ uint32_t load_word(const uint32_t* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// sort key of a candidate: deeper first (|S|, or the nearest-sample
// squared distance rounded to float)
__device__ __forceinline__ uint32_t depth_key(const Dev& D, const ShapeDev& S, uint32_t g, bool samples) {
  if (samples) return ~__float_as_uint((float)init_dmin2(D)[g]);
  uint32_t loc;
  int i, j, k;
  const LevelDev* L = init_locate(D, S, g, loc, i, j, k);
  return ~__float_as_uint(fabsf(L->sdf[loc]));
}

struct InitSlot {
  double r2;          // squared sphere radius
  int32_t e;          // position in the sorted candidate list, INT32_MAX if none
  uint32_t g;         // point index
  float x, y, z, r;   // centre; r bounds the radius from above (index boxes)
};

// The greedy rounds, one workgroup:
//   A. candidates in point order (block scans over the mask words);
//   B. stable LSD radix sort by depth key (4 passes of 8 bits), so the
//      list runs by |S| descending, point index ascending: the first
//      uncovered entry is always the next centre of Algorithm 1;
//   C. rounds over the sorted list, 1024 entries at a time held in
//      registers: the first uncovered entry becomes the centre; every thread
//      tests its own entry against it, and the centre's sphere is cleared
//      from the mask over its index box on every level (atomics), so a
//      block loaded later starts from the current cover.
// Writes centre, weight and identity rotation of each centre, the count to
// m_dev and (count, uncovered candidates) to the result words.
__global__ __launch_bounds__(1024) void k_init_greedy(Dev D, int shape, uint32_t nw, int samples, int m_max,
                                                      float* __restrict__ p, int32_t* __restrict__ m_dev) {
  __shared__ int scan_sh[32];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t base[256];
  __shared__ uint32_t cnt[16][256];
  __shared__ InitSlot slot[2][16];
  __shared__ uint32_t left_sh[16];
  uint32_t* mask = init_mask(D);
  uint32_t* A = init_list(D, 0);
  uint32_t* Bv = init_list(D, 1);
  uint32_t* res = init_res(D);
  const ShapeDev S = D.shapes[shape];
  const int C = D.cap_total;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;

  // A. compaction in point order
  uint32_t n_in = 0;
  for (uint32_t w0 = 0; w0 < nw; w0 += 1024u) {
    const uint32_t w = w0 + (uint32_t)tid;
    const uint32_t bits = w < nw ? mask[w] : 0u;
    int total;
    const int ex = block_excl_scan_1024<int>(__popc(bits), scan_sh, total);
    uint32_t at = n_in + (uint32_t)ex, rest = bits;
    while (rest) {
      const int b = __builtin_ctz(rest);
      rest &= rest - 1u;
      A[at++] = w * 32u + (uint32_t)b;
    }
    n_in += (uint32_t)total;
  }
  __syncthreads();

  // B. four stable passes, A -> Bv -> A -> Bv -> A
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    const uint32_t* src = (pass & 1) ? Bv : A;
    uint32_t* dst = (pass & 1) ? A : Bv;
    if (tid < 256) hist[tid] = 0u;
    __syncthreads();
    for (uint32_t e = (uint32_t)tid; e < n_in; e += 1024u)
      atomicAdd(&hist[(depth_key(D, S, src[e], samples) >> shift) & 255u], 1u);
    __syncthreads();
    if (tid < 64) {
      // exclusive scan of the 256 digit counts by one wave, 4 per lane
      const uint32_t h0 = hist[4 * tid], h1 = hist[4 * tid + 1], h2 = hist[4 * tid + 2], h3 = hist[4 * tid + 3];
      uint32_t x = h0 + h1 + h2 + h3;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      uint32_t b0 = x - (h0 + h1 + h2 + h3);
      base[4 * tid] = b0;
      base[4 * tid + 1] = b0 + h0;
      base[4 * tid + 2] = b0 + h0 + h1;
      base[4 * tid + 3] = b0 + h0 + h1 + h2;
    }
    for (uint32_t c0 = 0; c0 < n_in; c0 += 1024u) {
      for (int q = tid; q < 16 * 256; q += 1024) cnt[q >> 8][q & 255] = 0u;
      __syncthreads();
      const uint32_t e = c0 + (uint32_t)tid;
      const bool valid = e < n_in;
      const uint32_t g = valid ? src[e] : 0u;
      const uint32_t d = valid ? (depth_key(D, S, g, samples) >> shift) & 255u : 0u;
      // lanes of this wave holding the same digit
      uint64_t match = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const uint64_t bb = __ballot((d >> bit) & 1u);
        match &= ((d >> bit) & 1u) ? bb : ~bb;
      }
      const uint32_t wrank = (uint32_t)__popcll(match & lt_mask);
      if (valid && wrank == 0u) cnt[wv][d] = (uint32_t)__popcll(match);
      __syncthreads();
      if (tid < 256) {
        uint32_t acc = base[tid];
        for (int q = 0; q < 16; ++q) {
          const uint32_t t = cnt[q][tid];
          cnt[q][tid] = acc;
          acc += t;
        }
        base[tid] = acc;
      }
      __syncthreads();
      if (valid) dst[cnt[wv][d] + wrank] = g;
      __syncthreads();
    }
    __syncthreads();
  }

  // C. rounds
  int m = 0;
  uint32_t c0 = 0;            // first list position of the block in registers
  bool unc = false;           // my entry is a candidate no sphere covers yet
  uint32_t my_g = 0u;
  float mx = 0.f, my = 0.f, mz = 0.f, mr = 0.f;
  double mr2 = 0.0;
  bool need_load = true;
  for (int it = 0; m < m_max; ++it) {
    if (need_load) {
      if (c0 >= n_in) break;                              // uniform: list exhausted
      const uint32_t e = c0 + (uint32_t)tid;
      unc = false;
      if (e < n_in) {
        my_g = A[e];
        unc = (load_word(&mask[my_g >> 5]) >> (my_g & 31u)) & 1u;
        uint32_t loc;
        int i, j, k;
        const LevelDev* L = init_locate(D, S, my_g, loc, i, j, k);
        mx = L->axis[i];
        my = L->axis[j];
        mz = L->axis[k];
        if (samples) {
          mr2 = init_dmin2(D)[my_g];
          mr = (float)sqrt(mr2) * (1.0f + 1e-6f) + 1e-30f;
        } else {
          mr = fabsf(L->sdf[loc]);
          mr2 = (double)mr * (double)mr;
        }
      }
      need_load = false;
    }
    // first uncovered entry of this block
    const uint64_t bal = __ballot(unc);
    if (lane == (bal ? __builtin_ctzll(bal) : 0)) {
      InitSlot sl;
      sl.e = bal ? (int32_t)(c0 + (uint32_t)tid) : INT32_MAX;
      sl.g = my_g;
      sl.x = mx;
      sl.y = my;
      sl.z = mz;
      sl.r = mr;
      sl.r2 = mr2;
      slot[it & 1][wv] = sl;
    }
    __syncthreads();
    int win = 0;
#pragma unroll
    for (int q = 1; q < 16; ++q)
      if (slot[it & 1][q].e < slot[it & 1][win].e) win = q;
    const InitSlot cs = slot[it & 1][win];
    if (cs.e == INT32_MAX) {
      c0 += 1024u;                                        // uniform: nothing left in this block
      need_load = true;
      continue;
    }
    const double cx = (double)cs.x, cy = (double)cs.y, cz = (double)cs.z;
    const double r2 = cs.r2;
    if (tid == 0) {
      uint32_t loc;
      int i, j, k;
      const LevelDev* L = init_locate(D, S, cs.g, loc, i, j, k);
      const int sl = S.kbase + m;
      p[sl] = L->target[loc];
      p[C + sl] = cs.x;
      p[2 * C + sl] = cs.y;
      p[3 * C + sl] = cs.z;
      p[7 * C + sl] = D.orientation == ERBF_ORIENT_EULER ? 0.f : 1.f;   // identity rotation
      p[8 * C + sl] = 0.f;
      p[9 * C + sl] = 0.f;
      p[10 * C + sl] = 0.f;
    }
    ++m;
    // my entry against the new sphere (the centre covers itself)
    if (unc && dist2_rounded((double)mx - cx, (double)my - cy, (double)mz - cz) <= r2) unc = false;
    // clear the sphere from the mask on every level, over its index box
    uint32_t off = 0;
    for (int l = 0; l < S.n_active; ++l) {
      const LevelDev& L = D.levels[S.lvl0 + l];
      const int n = L.n;
      if (L.kind != kLevelGrid) {   // samples are never candidates
        off += (uint32_t)L.npts;
        continue;
      }
      int lo3[3], hi3[3];
      const float cc[3] = {cs.x, cs.y, cs.z};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo3[a] = max(0, (int)floorf((cc[a] - cs.r - L.lo) / L.h) - 1);
        hi3[a] = min(n - 1, (int)ceilf((cc[a] + cs.r - L.lo) / L.h) + 1);
      }
      const int bx = hi3[0] - lo3[0] + 1, by = hi3[1] - lo3[1] + 1, bz = hi3[2] - lo3[2] + 1;
      if (bx > 0 && by > 0 && bz > 0) {
        // one flat loop over the box, or slab by slab when it exceeds int
        const bool flat = (int64_t)bx * by * bz <= (int64_t)INT32_MAX;
        const int nz = flat ? 1 : bz;
        const int nq = flat ? bx * by * bz : bx * by;
        for (int kz = 0; kz < nz; ++kz)
          for (int q = tid; q < nq; q += 1024) {
            const int i = lo3[0] + q % bx;
            const int j = lo3[1] + (q / bx) % by;
            const int k = lo3[2] + (flat ? q / (bx * by) : kz);
            const double d2 =
                dist2_rounded((double)L.axis[i] - cx, (double)L.axis[j] - cy, (double)L.axis[k] - cz);
            if (d2 <= r2) {
              const uint32_t g = off + ((uint32_t)k * (uint32_t)n + (uint32_t)j) * (uint32_t)n + (uint32_t)i;
              atomicAnd(&mask[g >> 5], ~(1u << (g & 31u)));
            }
          }
      }
      off += (uint32_t)L.npts;
    }
  }
  __syncthreads();
  // candidates still uncovered (non-zero only when the limit stopped the rounds)
  uint32_t c = 0u;
  for (uint32_t w = (uint32_t)tid; w < nw; w += 1024u) c += (uint32_t)__popc(load_word(&mask[w]));
  c = wave_sum(c);
  if (lane == 0) left_sh[wv] = c;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0u;
    for (int q = 0; q < 16; ++q) t += left_sh[q];
    res[0] = (uint32_t)m;
    res[1] = t;
    m_dev[shape] = m;
  }
}

// eq. 3-12 for every centre; clears the shape's Adam moments
__global__ __launch_bounds__(256) void k_init_scale(Dev D, int shape, float gamma, float* __restrict__ p,
                                                    const int32_t* __restrict__ m_dev, float* __restrict__ m1,
                                                    float* __restrict__ m2) {
  __shared__ float sx[256], sy[256], sz[256];
  const ShapeDev S = D.shapes[shape];
  const int C = D.cap_total;
  const int M = min(max(m_dev[shape], 0), S.cap);
  const int j = blockIdx.x * 256 + threadIdx.x;
  float xj = 0.f, yj = 0.f, zj = 0.f;
  if (j < M) {
    xj = p[C + S.kbase + j];
    yj = p[2 * C + S.kbase + j];
    zj = p[3 * C + S.kbase + j];
  }
  double nearest = INFINITY;
  for (int t0 = 0; t0 < M; t0 += 256) {
    const int q = t0 + threadIdx.x;
    if (q < M) {
      sx[threadIdx.x] = p[C + S.kbase + q];
      sy[threadIdx.x] = p[2 * C + S.kbase + q];
      sz[threadIdx.x] = p[3 * C + S.kbase + q];
    }
    __syncthreads();
    const int nq = min(256, M - t0);
    for (int u = 0; u < nq; ++u) {
      if (t0 + u == j) continue;
      const double dx = (double)sx[u] - xj, dy = (double)sy[u] - yj, dz = (double)sz[u] - zj;
      nearest = fmin(nearest, dx * dx + dy * dy + dz * dz);
    }
    __syncthreads();
  }
  if (j < M) {
    const double dhat = M > 1 ? sqrt(nearest) : 2.0;
    const double w = (double)p[S.kbase + j];
    const float s = (float)log(2.0 * sqrt(-log((double)gamma / (w * w))) / dhat);
    p[4 * C + S.kbase + j] = s;
    p[5 * C + S.kbase + j] = s;
    p[6 * C + S.kbase + j] = s;
  }
  if (j < S.cap)
    for (int seg = 0; seg < 11; ++seg) {
      if (m1) m1[seg * C + S.kbase + j] = 0.f;
      if (m2) m2[seg * C + S.kbase + j] = 0.f;
    }
}

}  // namespace

hipError_t launch_init_inscribed(const Dev& D, int shape, uint32_t npts, bool samples, int m_max, int cap, float gamma,
                                 float* p, int32_t* m_dev, float* m1, float* m2, hipStream_t s) {
  const uint32_t nw = (npts + 31u) / 32u;
  const unsigned gm = (unsigned)std::max<uint32_t>(1u, std::min<uint32_t>((nw + 255u) / 256u, 4096u));
  hipLaunchKernelGGL(k_init_mark, dim3(gm), dim3(256), 0, s, D, shape, npts, nw);
  if (samples) hipLaunchKernelGGL(k_init_nearest, dim3((npts + 255u) / 256u), dim3(256), 0, s, D, shape, npts);
  hipLaunchKernelGGL(k_init_greedy, dim3(1), dim3(1024), 0, s, D, shape, nw, samples ? 1 : 0, m_max, p, m_dev);
  hipLaunchKernelGGL(k_init_scale, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, D, shape, gamma, p, m_dev,
                     m1, m2);
  return hipGetLastError();
}

int init_results(const Dev& D, int32_t* n_centres, int64_t* n_left, hipStream_t s) {
  uint32_t r[2];
  const uint32_t* res = D.init_scratch + 2 * D.init_cand_cap + D.init_words + 2 * D.init_cand_cap;
  if (hipMemcpyAsync(r, res, sizeof(r), hipMemcpyDeviceToHost, s) != hipSuccess)
    return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  *n_centres = (int32_t)r[0];
  *n_left = (int64_t)r[1];
  return 0;
}

}  // namespace erbf
