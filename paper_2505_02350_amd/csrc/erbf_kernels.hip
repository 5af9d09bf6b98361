// HIP kernels of the ERBF-fit step for gfx950 (CDNA4, wave64).
//
//   record     per-kernel record: centre, squared cull radius, log2(e)-scaled
//              quadric A = R^T diag(d^2) R, amplitude (eq. 3-7, 3-26, 3-15),
//              formed by the bucket count pass
//   bucket     tile -> kernel lists: per-kernel count, scan, kernel-major emit,
//              stable radix sort by tile slot (no atomics)
//   forward    point-centric gather over the tile's kernel list staged in LDS,
//              fused residual / id_all mask / loss partials (eq. 3-9, 3-15-1,
//              3-18, 3-19)
//   backward   tile-centric moments: lanes own the tile's kernels and walk the
//              tile's points with non-zero upstream gradient; a second pass
//              sums each kernel's per-tile moments in a fixed order in FP64
//              and forms the gradients (Appendix A, quaternion chain rule);
//              no float atomics
//   stats      per-shape loss statistics, eq. 3-21 weights, gradient combine
//   adam       fused bias-corrected Adam over the packed parameters
//
// Every reduction runs in a fixed order, so results are bitwise reproducible.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "erbf_device.h"
#include "erbf_internal.h"
#include "erbf_launch.h"

namespace erbf {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Conservative index range of the points whose coordinate may lie in
// [c0, c1] on a level (the exact predicate is applied afterwards).
__device__ __forceinline__ void index_range(const LevelDev& L, float c0, float c1, int& i0, int& i1) {
  float f0 = (c0 - L.lo) / L.h;
  float f1 = (c1 - L.lo) / L.h;
  f0 = fminf(fmaxf(f0, -2.0f), (float)L.n + 2.0f);
  f1 = fminf(fmaxf(f1, -2.0f), (float)L.n + 2.0f);
  i0 = max(0, (int)floorf(f0) - 1);
  i1 = min(L.n - 1, (int)ceilf(f1) + 1);
}

__device__ __forceinline__ float tile_lo(const LevelDev& L, int t) {
  return fmaf((float)(t * kTile), L.h, L.lo) - L.pad;
}
__device__ __forceinline__ float tile_hi(const LevelDev& L, int t) {
  return fmaf((float)min(t * kTile + kTile - 1, L.n - 1), L.h, L.lo) + L.pad;
}

__device__ __forceinline__ bool point_active(const uint32_t* bits, int64_t local) {
  if (bits == nullptr) return true;
  return (bits[local >> 5] >> (local & 31)) & 1u;
}

// Number of set bits of `bits` in [b0, b1] (inclusive), b0 <= b1.
__device__ __forceinline__ int popcount_range(const uint32_t* bits, int64_t b0, int64_t b1) {
  int64_t w0 = b0 >> 5, w1 = b1 >> 5;
  int c = 0;
  for (int64_t w = w0; w <= w1; ++w) {
    uint32_t v = bits[w];
    if (w == w0) v &= 0xffffffffu << (b0 & 31);
    if (w == w1) v &= 0xffffffffu >> (31 - (b1 & 31));
    c += __popc(v);
  }
  return c;
}

// ---------------------------------------------------------------------------
// per-kernel record (formed by the bucket count pass, one wave per kernel slot)
// record: r0 = {cx, cy, cz, r^2}  (r^2 < 0 marks a dead slot)
//         r1 = {A00, A11, A22, 2 A01}  r2 = {2 A02, 2 A12, a, 0}, A scaled by log2(e)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void kernel_record(const float* __restrict__ p, const int32_t* __restrict__ m_dev,
                                              const Dev& D, const int j, float4& r0_out, float4& r1_out,
                                              float4& r2_out) {
  const int b = D.kshape[j];
  const ShapeDev S = D.shapes[b];
  const int m = min(max(m_dev[b], 0), S.cap);
  float4 r0 = make_float4(0.f, 0.f, 0.f, -1.f);
  float4 r1 = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 r2 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (j - S.kbase < m) {
    const int C = D.cap_total;
    const float w = p[j];
    const float cx = p[C + j], cy = p[2 * C + j], cz = p[3 * C + j];
    const float s0 = p[4 * C + j], s1 = p[5 * C + j], s2 = p[6 * C + j];
    float R[3][3];
    if (D.orientation == ERBF_ORIENT_EULER) {
      // eq. 3-6: R = Rz(theta_z) Ry(theta_y) Rx(theta_x), angles in the
      // first three orientation slots
      float sx, cx_, sy, cy_, sz, cz_;
      sincosf(p[7 * C + j], &sx, &cx_);
      sincosf(p[8 * C + j], &sy, &cy_);
      sincosf(p[9 * C + j], &sz, &cz_);
      R[0][0] = cz_ * cy_; R[0][1] = cz_ * sy * sx - sz * cx_; R[0][2] = cz_ * sy * cx_ + sz * sx;
      R[1][0] = sz * cy_;  R[1][1] = sz * sy * sx + cz_ * cx_; R[1][2] = sz * sy * cx_ - cz_ * sx;
      R[2][0] = -sy;       R[2][1] = cy_ * sx;                 R[2][2] = cy_ * cx_;
    } else {
      float qw = p[7 * C + j], qx = p[8 * C + j], qy = p[9 * C + j], qz = p[10 * C + j];
      const float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
      if (qn2 > 0.f) {
        const float inv = 1.0f / sqrtf(qn2);
        qw *= inv; qx *= inv; qy *= inv; qz *= inv;
      } else {
        qw = 1.f; qx = qy = qz = 0.f;
      }
      R[0][0] = 1.f - 2.f * (qy * qy + qz * qz);
      R[0][1] = 2.f * (qx * qy - qw * qz);
      R[0][2] = 2.f * (qx * qz + qw * qy);
      R[1][0] = 2.f * (qx * qy + qw * qz);
      R[1][1] = 1.f - 2.f * (qx * qx + qz * qz);
      R[1][2] = 2.f * (qy * qz - qw * qx);
      R[2][0] = 2.f * (qx * qz - qw * qy);
      R[2][1] = 2.f * (qy * qz + qw * qx);
      R[2][2] = 1.f - 2.f * (qx * qx + qy * qy);
    }
    const float d2[3] = {expf(2.f * s0), expf(2.f * s1), expf(2.f * s2)};
    float A[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        A[a][c] = R[0][a] * d2[0] * R[0][c] + R[1][a] * d2[1] * R[1][c] + R[2][a] * d2[2] * R[2][c];
    const float smin = fminf(s0, fminf(s1, s2));
    const float r = D.cull_k / expf(smin);
    const float amp = D.weight_map == ERBF_WEIGHT_SIGNED_SQUARE ? w * fabsf(w) : w;
    r0 = make_float4(cx, cy, cz, r * r);
    r1 = make_float4(A[0][0] * kLog2e, A[1][1] * kLog2e, A[2][2] * kLog2e, 2.f * A[0][1] * kLog2e);
    r2 = make_float4(2.f * A[0][2] * kLog2e, 2.f * A[1][2] * kLog2e, amp, 0.f);
  }
  r0_out = r0;
  r1_out = r1;
  r2_out = r2;
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts (three passes, 1024 elements per block)
// ---------------------------------------------------------------------------


// T: the type of the block sums and of the output (int32 when every prefix
// fits, int64 for the bucket-entry offsets, whose total may pass 2^31 before
// it is compared with the list capacity)
template <typename T>
__global__ __launch_bounds__(1024) void k_scan_reduce(const int32_t* __restrict__ in, int n, T* __restrict__ blocks) {
  __shared__ T sh[32];
  const int i = blockIdx.x * 1024 + threadIdx.x;
  T total;
  block_excl_scan_1024<T>(i < n ? (T)in[i] : (T)0, sh, total);
  if (threadIdx.x == 0) blocks[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_blocks(T* __restrict__ blocks, int nb, int64_t* __restrict__ total_out) {
  __shared__ T sh[32];
  T carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const T v = i < nb ? blocks[i] : (T)0;
    T total;
    const T e = block_excl_scan_1024<T>(v, sh, total);
    if (i < nb) blocks[i] = carry + e;
    carry += total;
  }
  if (threadIdx.x == 0 && total_out) *total_out = (int64_t)carry;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_down(const int32_t* __restrict__ in, int n, const T* __restrict__ blocks,
                                                    T* __restrict__ out) {
  __shared__ T sh[32];
  const int i = blockIdx.x * 1024 + threadIdx.x;
  T total;
  const T e = block_excl_scan_1024<T>(i < n ? (T)in[i] : (T)0, sh, total);
  if (i <= n) out[i] = blocks[blockIdx.x] + e;  // out has n + 1 entries
}

// Single-block exclusive scan of n <= 1024 * PER values; out[n] = total.
// Each thread owns PER consecutive values, read with independent loads.
template <int PER, typename T>
__global__ __launch_bounds__(1024) void k_scan_single(const int32_t* __restrict__ in, int n, T* __restrict__ out,
                                                      int64_t* __restrict__ total_out) {
  __shared__ T sh[32];
  const int t = threadIdx.x;
  const int lo = t * PER;
  T v[PER];
  T sum = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    v[u] = lo + u < n ? (T)in[lo + u] : (T)0;
    sum += v[u];
  }
  T total;
  T run = block_excl_scan_1024<T>(sum, sh, total);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (lo + u < n) out[lo + u] = run;
    run += v[u];
  }
  if (t == 0) {
    out[n] = total;
    if (total_out) *total_out = (int64_t)total;
  }
}

// exclusive scan of n values into out[0..n], the total also to *total_out
template <typename T>
hipError_t launch_scan_any(const int32_t* in, int n, T* blocks, T* out, int64_t* total, hipStream_t s);

// ---------------------------------------------------------------------------
// Tile buckets.  One wave per kernel slot; lanes test the tiles of the
// ball's tile box.  A kernel's tiles are numbered in a fixed order (level,
// z, y, x): the visit index.  The count pass counts each kernel's tiles and
// keeps their slots (up to hit_cap per kernel); the emit pass writes the
// entries kernel-major, entry e = kstart[j] + visit, with the tile slot as
// the sort key, copying the kept slots (walking again only for a kernel
// with more tiles than were kept).  A stable sort of the kernel-major
// list by slot then gives every tile's kernels in ascending order, with no
// atomics and the same result on every run.
// ---------------------------------------------------------------------------

// A tile is hit when the ball, widened slightly, reaches the tile's point box
// (a fixed expression, so a walk in the count pass and one in the emit pass
// take the same decisions) and the tile is in use.
__device__ __forceinline__ float ball_box_e2(const LevelDev& L, const float4& r0, int ty, int tz) {
  const float ey = fmaxf(fmaxf(tile_lo(L, ty) - r0.y, r0.y - tile_hi(L, ty)), 0.f);
  const float ez = fmaxf(fmaxf(tile_lo(L, tz) - r0.z, r0.z - tile_hi(L, tz)), 0.f);
  return fmaf(ey, ey, ez * ez);
}
__device__ __forceinline__ bool ball_box_hit(const LevelDev& L, const float4& r0, float e2, int tx, float rc2) {
  const float ex = fmaxf(fmaxf(tile_lo(L, tx) - r0.x, r0.x - tile_hi(L, tx)), 0.f);
  return fmaf(ex, ex, e2) < rc2;
}

// a slot the bucket lists cover: an active tile, selected when a selection
// is given (mini-batches list only the tiles holding batch points)
__device__ __forceinline__ bool tile_listed(const Dev& D, int slot) {
  return slot >= 0 && (D.tile_sel == nullptr || D.tile_sel[slot] != 0);
}

struct BallBox {
  float rc2;
  int tx0, tx1, ty0, nty, tz0, ntz;
};

__device__ __forceinline__ bool ball_box(const LevelDev& L, const float4& r0, BallBox& B) {
  const float rr = sqrtf(r0.w) * (1.0f + 1e-5f) + 1e-6f;
  B.rc2 = rr * rr;
  int ix0, ix1, iy0, iy1, iz0, iz1;
  index_range(L, r0.x - rr, r0.x + rr, ix0, ix1);
  index_range(L, r0.y - rr, r0.y + rr, iy0, iy1);
  index_range(L, r0.z - rr, r0.z + rr, iz0, iz1);
  if (ix0 > ix1 || iy0 > iy1 || iz0 > iz1) return false;
  B.tx0 = ix0 / kTile;
  B.tx1 = ix1 / kTile;
  B.ty0 = iy0 / kTile;
  B.nty = iy1 / kTile - B.ty0 + 1;
  B.tz0 = iz0 / kTile;
  B.ntz = iz1 / kTile - B.tz0 + 1;
  return true;
}

// slot of tile t (index in the level's tile grid): arithmetic on a level
// whose tiles are all active, the tile map otherwise
__device__ __forceinline__ int tile_slot_of(const Dev& D, const LevelDev& L, int t) {
  return L.dense ? L.slot0 + t : D.tile_map[L.tmap0 + t];
}

// Box walk: lanes own consecutive tiles of the ball's tile box, so a ballot
// numbers the hits in visit order; hit(v, slot) is called for the tile of
// visit index v.  Returns the kernel's tile count.
template <class F>
__device__ __forceinline__ int bucket_box_walk(const Dev& D, const float4 r0, const int j, const int lane, F&& hit) {
  if (r0.w < 0.f) return 0;
  int vbase = 0;
  const ShapeDev S = D.shapes[D.kshape[j]];
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  for (int li = 0; li < S.n_active; ++li) {
    const LevelDev L = D.levels[S.lvl0 + li];
    BallBox B;
    if (!ball_box(L, r0, B)) continue;
    const int ntx = B.tx1 - B.tx0 + 1, nxy = ntx * B.nty, total = nxy * B.ntz;
    // box index -> (x, y, z) by a float reciprocal: exact while
    // (quotient + 1) * divisor < 2^21, which keeps the rounding error
    // below the 0.5 / divisor gap to the next integer; larger boxes take
    // the integer division
    const bool small_box = total + nxy < (1 << 21);
    const float inv_x = 1.0f / (float)ntx, inv_xy = 1.0f / (float)nxy;
    for (int base = 0; base < total; base += 64) {
      const int idx = base + lane;
      int slot = -1;
      if (idx < total) {
        int qz, qy, qx;
        if (small_box) {
          qz = (int)(((float)idx + 0.5f) * inv_xy);
          const int rem = idx - qz * nxy;
          qy = (int)(((float)rem + 0.5f) * inv_x);
          qx = rem - qy * ntx;
        } else {
          qz = idx / nxy;
          qy = (idx % nxy) / ntx;
          qx = idx % ntx;
        }
        const int tx = B.tx0 + qx, ty = B.ty0 + qy, tz = B.tz0 + qz;
        const float e2 = ball_box_e2(L, r0, ty, tz);
        if (e2 < B.rc2 && ball_box_hit(L, r0, e2, tx, B.rc2)) {
          const int sl = tile_slot_of(D, L, (tz * L.nt + ty) * L.nt + tx);
          slot = tile_listed(D, sl) ? sl : -1;
        }
      }
      const unsigned long long bal = __ballot(slot >= 0);
      if (slot >= 0) hit(vbase + __popcll(bal & lt_mask), slot);
      vbase += __popcll(bal);
    }
  }
  return vbase;
}

// Entry v of kernel j (of cnt_j, starting at e0), for tile slot `slot`.
__device__ __forceinline__ void bucket_place(const Dev& D, const int j, const int64_t e0, const int v, const int cnt_j,
                                             const int slot) {
  if (v >= cnt_j) return;
  const int64_t at = e0 + v;
  if (D.bucket_rank) {
    // the tile's count runs back down to 0 as its entries are placed (ready
    // for the next build); the order within the tile is fixed afterwards by
    // k_tile_rank
    const int64_t pos = D.tile_start64[slot] + (int64_t)(atomicSub(&D.tile_cnt[slot], 1) - 1);
    if (pos < D.pair_cap) {
      D.sort_j[0][pos] = j;
      D.sort_vals[0][pos] = at < D.pair_cap ? (int)at : -1;
    }
  } else if (at >= 0 && at < D.pair_cap) {
    if (D.packed_keys) {
      D.kslot[at] = (int32_t)(((uint32_t)slot << 16) | (uint32_t)j);
    } else {
      D.kslot[at] = slot;
      D.kj[at] = j;
    }
  }
}

// Count pass: the kernel's record (every lane forms the same one, lane 0
// stores it), kcnt per kernel (one wave each), its first hit_cap tile slots
// in visit order, and the sum of each block's four kernels.
__global__ __launch_bounds__(256) void k_bucket_count(Dev D, const float* __restrict__ p,
                                                      const int32_t* __restrict__ m_dev) {
  __shared__ int wc[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + w);
  int c = 0;
  if (j < D.cap_total) {
    float4 r0, r1, r2;
    kernel_record(p, m_dev, D, j, r0, r1, r2);
    if (lane == 0) {
      D.rec[3 * j + 0] = r0;
      D.rec[3 * j + 1] = r1;
      D.rec[3 * j + 2] = r2;
    }
    int32_t* hj = D.hits + (int64_t)j * D.hit_cap;
    c = bucket_box_walk(D, r0, j, lane, [&](int v, int sl) {
      if (v < D.hit_cap) hj[v] = sl;
      if (D.bucket_rank) atomicAdd(&D.tile_cnt[sl], 1);
    });
  }
  if (lane == 0) {
    if (j < D.cap_total) D.kcnt[j] = c;
    wc[w] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) D.kblock[blockIdx.x] = (wc[0] + wc[1]) + (wc[2] + wc[3]);
}

// Emit pass: kstart from the scanned block sums, then the entries, copied
// from the count pass's slots when they were all kept, else by the same walk.
__global__ __launch_bounds__(256) void k_bucket_emit(Dev D) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + w);
  if (j >= D.cap_total) return;
  int64_t e0 = D.kblock_ex[blockIdx.x];
  for (int k = 0; k < w; ++k) e0 += D.kcnt[4 * blockIdx.x + k];
  if (lane == 0) D.kstart[j] = e0;
  const int cnt_j = D.kcnt[j];
  int done;
  if (cnt_j <= D.hit_cap) {
    const int32_t* hj = D.hits + (int64_t)j * D.hit_cap;
    for (int v0 = 0; v0 < cnt_j; v0 += 256) {
      // four loads in flight per lane (indices clamped into the kept slots)
      int sl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) sl[i] = hj[min(v0 + 64 * i + lane, cnt_j - 1)];
#pragma unroll
      for (int i = 0; i < 4; ++i) bucket_place(D, j, e0, v0 + 64 * i + lane, cnt_j, sl[i]);
    }
    done = cnt_j;
  } else {
    done = bucket_box_walk(D, D.rec[3 * j], j, lane,
                           [&](int v, int sl) { bucket_place(D, j, e0, v, cnt_j, sl); });
  }
  // both walks take the same decisions; should they ever differ, the
  // counted range is still filled, with a slot past every real tile
  for (int v = done + lane; v < cnt_j; v += 64) {
    const int64_t at = e0 + v;
    if (at >= 0 && at < D.pair_cap) {
      if (!D.bucket_rank) {
        if (D.packed_keys) {
          D.kslot[at] = (int32_t)(((uint32_t)D.tiles_total << 16) | (uint32_t)j);
        } else {
          D.kslot[at] = D.tiles_total;
          D.kj[at] = j;
        }
      }
      float2* o = D.partials + 5 * at;   // no tile writes this entry's moments
#pragma unroll
      for (int i = 0; i < 5; ++i) o[i] = make_float2(0.f, 0.f);
    }
  }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of the (slot, entry) pairs, up to 8 key bits per
// pass.  A fixed grid of radix_nb blocks; block b owns one contiguous
// segment of the entries.  Pass = digit counts per block, an exclusive scan
// over (digit, block), then a stable scatter: within a block, the rank of an
// entry among equal digits comes from wave ballots (lanes in entry order)
// and per-wave running counts, so equal keys keep their order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t bucket_entries(const Dev& D) { return min(D.counters[0], D.pair_cap); }

__device__ __forceinline__ void radix_segment(int64_t n, int nb, int b, int64_t& lo, int64_t& hi) {
  const int64_t per = (n + nb - 1) / nb;
  lo = min(n, per * b);
  hi = min(n, lo + per);
}

constexpr int kRadixHistPer = 8;   // keys per thread per block iteration of the count

__global__ __launch_bounds__(256) void k_radix_hist(Dev D, const int32_t* __restrict__ keys, int shift, int mask) {
  __shared__ int cnt[256];
  const int t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  int64_t lo, hi;
  radix_segment(bucket_entries(D), D.radix_nb, blockIdx.x, lo, hi);
  for (int64_t base = lo; base < hi; base += 256 * kRadixHistPer) {
    // all loads first (indices clamped into the segment), then the counts
    int k[kRadixHistPer];
#pragma unroll
    for (int i = 0; i < kRadixHistPer; ++i) {
      const int64_t idx = base + 256 * i + t;
      k[i] = keys[idx < hi ? idx : lo];
    }
#pragma unroll
    for (int i = 0; i < kRadixHistPer; ++i)
      if (base + 256 * i + t < hi) atomicAdd(&cnt[(k[i] >> shift) & mask], 1);
  }
  __syncthreads();
  D.rhist[t * D.radix_nb + blockIdx.x] = cnt[t];
}

// Row d of the digit counts (one value per sort block) -> exclusive prefix
// within the row; the row totals go after the rows.
__global__ __launch_bounds__(1024) void k_radix_rowscan(Dev D) {
  __shared__ int sh[32];
  const int d = blockIdx.x, b = threadIdx.x, nb = D.radix_nb;
  int total;
  const int e = block_excl_scan_1024(b < nb ? D.rhist[d * nb + b] : 0, sh, total);
  if (b < nb) D.rhist_ex[d * nb + b] = e;
  if (b == 0) D.rhist_ex[256 * nb + d] = total;
}

// exclusive scan over a 256-thread block
__device__ __forceinline__ int block_excl_scan_256(int v, int* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  int base = 0;
  for (int k = 0; k < w; ++k) base += sh[k];
  __syncthreads();
  return base + x - v;
}

constexpr int kRadixPerLane = 8;                     // entries per lane per block iteration
constexpr int kRadixWaveSpan = 64 * kRadixPerLane;   // consecutive entries of one wave
constexpr int kRadixSpan = 4 * kRadixWaveSpan;       // entries per block iteration

// Moves (key, entry, kernel) triples; vin == nullptr means entry = index.
// STAGE: each iteration's entries are first placed in LDS in (digit, wave,
// rank) order, so that the global stores of one digit's run are contiguous
// (worth it when neighbouring entries hold different digits, as in the
// kernel-major input of the first pass).  PACKED: the key is slot << 16 | j
// and no kernel array is read; the last pass (last = 1) writes the slot and
// the kernel apart.
template <bool STAGE, bool PACKED>
__global__ __launch_bounds__(256) void k_radix_scatter(Dev D, const int32_t* __restrict__ kin,
                                                       const int32_t* __restrict__ vin,
                                                       const int32_t* __restrict__ jin, int32_t* __restrict__ kout,
                                                       int32_t* __restrict__ vout, int32_t* __restrict__ jout,
                                                       int shift, int mask, int dbits, int last) {
  __shared__ int run[256];
  __shared__ int wcnt[4][256];   // per-wave digit counts, then global starts
  __shared__ int lcnt[4][256];   // starts within this iteration's staged run
  __shared__ int run_off[STAGE ? 256 : 1];   // output index minus stage index, per digit
  __shared__ int sws[4];
  // staged (key, entry, kernel); an entry's destination is its digit's
  // global start plus its place in the digit's staged run
  __shared__ int stage_k[STAGE ? kRadixSpan : 1], stage_v[STAGE ? kRadixSpan : 1],
      stage_j[STAGE && !PACKED ? kRadixSpan : 1];
  // one sorted entry out: (slot, entry, kernel)
  auto put = [&](int64_t pos, int k, int v, int j) {
    if (PACKED) {
      kout[pos] = last ? (int)((uint32_t)k >> 16) : k;
      if (last) jout[pos] = k & 0xffff;
    } else {
      kout[pos] = k;
      jout[pos] = j;
    }
    vout[pos] = v;
  };
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  int64_t lo, hi;
  radix_segment(bucket_entries(D), D.radix_nb, blockIdx.x, lo, hi);
  // digit t starts after all smaller digits, then after digit t of the
  // earlier blocks
  const int dbase = block_excl_scan_256(D.rhist_ex[256 * D.radix_nb + t], sws);
  run[t] = dbase + D.rhist_ex[t * D.radix_nb + blockIdx.x];
  for (int64_t base = lo; base < hi; base += kRadixSpan) {
    for (int k = lane; k < 256; k += 64) wcnt[w][k] = 0;
    __syncthreads();
    int key[kRadixPerLane], val[kRadixPerLane], kid[kRadixPerLane], rank[kRadixPerLane];
    bool ok[kRadixPerLane];
    // all loads first, from indices clamped into the segment (lo < hi), so
    // that they are in flight together; entries past the segment are
    // masked by ok
#pragma unroll
    for (int i = 0; i < kRadixPerLane; ++i) {
      const int64_t idx = base + w * kRadixWaveSpan + i * 64 + lane;
      ok[i] = idx < hi;
      const int64_t ci = ok[i] ? idx : lo;
      key[i] = kin[ci];
      kid[i] = PACKED ? 0 : jin[ci];
      val[i] = (int)idx;
    }
    if (vin) {
#pragma unroll
      for (int i = 0; i < kRadixPerLane; ++i) {
        const int64_t idx = base + w * kRadixWaveSpan + i * 64 + lane;
        val[i] = vin[idx < hi ? idx : lo];
      }
    }
#pragma unroll
    for (int i = 0; i < kRadixPerLane; ++i) {
      const int d = (key[i] >> shift) & mask;
      // lanes of this wave holding the same digit
      unsigned long long same = __ballot(ok[i]);
      for (int b = 0; b < dbits; ++b) {
        const bool bit = (d >> b) & 1;
        const unsigned long long bb = __ballot(bit);
        same &= bit ? bb : ~bb;
      }
      const int before = wcnt[w][d];
      rank[i] = before + __popcll(same & lt);
      if (ok[i] && (same & lt) == 0) wcnt[w][d] = before + __popcll(same);
    }
    __syncthreads();
    {  // digit t: where each wave's run starts, globally and in the stage
      int c[4], tot = 0;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        c[ww] = wcnt[ww][t];
        tot += c[ww];
      }
      int l = STAGE ? block_excl_scan_256(tot, sws) : 0;
      int g = run[t];
      // the waves' runs of digit t are consecutive both in the stage and in
      // the output, so a stage index maps to the output by one offset
      if (STAGE) run_off[t] = g - l;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        wcnt[ww][t] = g;
        if (STAGE) lcnt[ww][t] = l;
        g += c[ww];
        l += c[ww];
      }
      run[t] = g;
    }
    __syncthreads();
    if (STAGE) {
#pragma unroll
      for (int i = 0; i < kRadixPerLane; ++i) {
        if (ok[i]) {
          const int d = (key[i] >> shift) & mask;
          const int q = lcnt[w][d] + rank[i];
          stage_k[q] = key[i];
          stage_v[q] = val[i];
          if (!PACKED) stage_j[q] = kid[i];
        }
      }
      __syncthreads();
      const int nit = (int)min((int64_t)kRadixSpan, hi - base);
      for (int q = t; q < nit; q += 256) {
        const int k = stage_k[q];
        const int pos = run_off[(k >> shift) & mask] + q;
        put(pos, k, stage_v[q], PACKED ? 0 : stage_j[q]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < kRadixPerLane; ++i) {
        if (ok[i]) {
          const int pos = wcnt[w][(key[i] >> shift) & mask] + rank[i];
          put(pos, key[i], val[i], kid[i]);
        }
      }
    }
    __syncthreads();
  }
}

// class of a list of len entries in the launch order (0: longest)
__device__ __forceinline__ int order_class(int len) {
  return kOrderClasses - 1 - min(len >> 4, kOrderClasses - 1);
}

// tile_start[s] = first sorted entry whose slot is >= s (s = 0 .. n_slots),
// by a lower-bound search over the sorted keys; with the launch
// order switched on, also the class counts of the block's 256 slots
// (order_hist row blockIdx.x).
__global__ __launch_bounds__(256) void k_tile_starts(Dev D, const int32_t* __restrict__ keys, int n_slots) {
  __shared__ int st[257];
  __shared__ int cnt[kOrderClasses];
  const int t = threadIdx.x, s = blockIdx.x * 256 + t;
  const int64_t n_e = bucket_entries(D);
  auto lower = [&](int v) {
    int64_t lo = 0, hi = n_e;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    return (int)lo;
  };
  int v = 0;
  if (s <= n_slots) {
    v = lower(s);
    D.tile_start[s] = v;
  }
  if (!D.tile_order_on) return;   // uniform over the launch
  st[t] = v;
  if (t == 0) {
    const int s1 = blockIdx.x * 256 + 256;
    st[256] = s1 <= n_slots ? lower(s1) : 0;
  }
  if (t < kOrderClasses) cnt[t] = 0;
  __syncthreads();
  if (s < n_slots) atomicAdd(&cnt[order_class(st[t + 1] - st[t])], 1);
  __syncthreads();
  if (t < kOrderClasses) D.order_hist[blockIdx.x * kOrderClasses + t] = cnt[t];
}

// Launch order of the tile kernels: the active slots by the length of their
// kernel lists, longest first, in kOrderClasses classes of 16 entries (the
// last class takes every list of 1008 entries or more).  A tile's work grows
// with its list, so the long tiles start first instead of finishing last.
// Each block of 256 slots has its class counts in order_hist (from
// k_tile_starts, or k_order_count when the lists are ranked); k_order_place
// gives the block's slots of class c the places after every slot of a
// longer class and after the class-c slots of the blocks before it.  The
// order inside a block's run follows the LDS atomics and is not fixed; no
// result depends on it (every tile writes only its own outputs).
__global__ __launch_bounds__(256) void k_order_count(Dev D, int n_slots) {
  __shared__ int cnt[kOrderClasses];
  const int t = threadIdx.x, s = blockIdx.x * 256 + t;
  if (t < kOrderClasses) cnt[t] = 0;
  __syncthreads();
  if (s < n_slots) atomicAdd(&cnt[order_class(D.tile_start[s + 1] - D.tile_start[s])], 1);
  __syncthreads();
  if (t < kOrderClasses) D.order_hist[blockIdx.x * kOrderClasses + t] = cnt[t];
}

__global__ __launch_bounds__(256) void k_order_place(Dev D, int n_slots, int nb) {
  constexpr int kRows = 64;   // blocks' counts staged per round
  __shared__ int hbuf[kRows * kOrderClasses];
  __shared__ int base[kOrderClasses], pre[kOrderClasses];
  const int t = threadIdx.x, s = blockIdx.x * 256 + t;
  const bool have = s < n_slots;
  const int lo = have ? D.tile_start[s] : 0, hi = have ? D.tile_start[s + 1] : 0;
  int tot = 0, pr = 0;   // thread t < kOrderClasses: class t over all blocks, and over the blocks before this one
  for (int b0 = 0; b0 < nb; b0 += kRows) {
    const int nr = min(kRows, nb - b0);
    int v[kRows * kOrderClasses / 256];
#pragma unroll
    for (int i = 0; i < kRows * kOrderClasses / 256; ++i) {
      const int idx = t + 256 * i;
      v[i] = idx / kOrderClasses < nr ? D.order_hist[(int64_t)b0 * kOrderClasses + idx] : 0;
    }
#pragma unroll
    for (int i = 0; i < kRows * kOrderClasses / 256; ++i) hbuf[t + 256 * i] = v[i];
    __syncthreads();
    if (t < kOrderClasses) {
      for (int r = 0; r < nr; ++r) {
        const int x = hbuf[r * kOrderClasses + t];
        tot += x;
        pr += b0 + r < (int)blockIdx.x ? x : 0;
      }
    }
    __syncthreads();
  }
  if (t < kOrderClasses) {
    base[t] = tot;
    pre[t] = pr;
  }
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int c = 0; c < kOrderClasses; ++c) {
      const int n = base[c];
      base[c] = run + pre[c];
      run += n;
    }
  }
  __syncthreads();
  if (have) D.tile_order[atomicAdd(&base[order_class(hi - lo)], 1)] = s;
}

// Tile lists without a sort (rank mode): the emit pass has placed every
// tile's entries in its range [start, end) in arbitrary order (sort_j[0],
// sort_vals[0]).  One wave per tile marks the tile's kernels in a bitmap over
// its shape's kernel slots (LDS), forms the prefix counts of the bitmap's
// words, and writes each entry at start + (number of the tile's kernels with
// a lower slot): the tile's kernels in ascending order, as the stable sort
// gives them, whatever order the atomics placed them in.

__global__ __launch_bounds__(256) void k_tile_rank(Dev D, int n_slots) {
  extern __shared__ uint32_t rank_lds[];   // per wave: bitmap words, then their prefix counts
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int s = blockIdx.x * 4 + wv;
  const bool have = s < n_slots;
  int kbase = 0, W = 0;
  int64_t beg = 0, end = 0;
  if (have) {
    const ShapeDev S = D.shapes[D.levels[D.slot_tile[s].x].shape];
    kbase = S.kbase;
    W = (S.cap + 31) >> 5;
    beg = min(D.tile_start64[s], D.pair_cap);
    end = min(D.tile_start64[s + 1], D.pair_cap);
  }
  const int wmax = D.rank_words;
  uint32_t* bm = rank_lds + (size_t)wv * 2 * wmax;
  uint32_t* pre = bm + wmax;
  for (int w = lane; w < W; w += 64) bm[w] = 0u;
  __syncthreads();
  for (int64_t c = beg + lane; c < end; c += 64) {
    const int loc = D.sort_j[0][c] - kbase;
    atomicOr(&bm[loc >> 5], 1u << (loc & 31));
  }
  __syncthreads();
  {
    // prefix counts of the words: lane l sums its run of words, a wave scan
    // gives each run's start
    const int per = (W + 63) >> 6;
    const int w0 = min(W, lane * per), w1 = min(W, w0 + per);
    int cnt = 0;
    for (int w = w0; w < w1; ++w) cnt += __popc(bm[w]);
    int x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    int run = x - cnt;
    for (int w = w0; w < w1; ++w) {
      pre[w] = run;
      run += __popc(bm[w]);
    }
  }
  __syncthreads();
  for (int64_t c = beg + lane; c < end; c += 64) {
    const int j = D.sort_j[0][c];
    const int e = D.sort_vals[0][c];
    const int loc = j - kbase;
    const int rk = (int)pre[loc >> 5] + __popc(bm[loc >> 5] & ((1u << (loc & 31)) - 1u));
    D.items[beg + rk] = j;
    D.tile_e[beg + rk] = e;
  }
  if (have && lane == 0) {
    D.tile_start[s] = (int)beg;
    if (s == n_slots - 1) D.tile_start[n_slots] = (int)min(D.tile_start64[n_slots], D.pair_cap);
  }
}

// ---------------------------------------------------------------------------
// forward: one workgroup (4 waves) per active tile of 8^3 points
//   wave w covers x in [0,8), y in 4*(w&1)+[0,4), z in 4*(w>>1)+[0,4);
//   lane l covers points x = 2*(l&3)+{0,1}, y += (l>>2)&3, z += l>>4,
//   so the four lanes of a quad share one row (y, z).
// Each wave's list holds the kernels of the tile's list whose (padded) ball
// meets the bounding box of the wave's training points.
// A wave walks its kernel list four kernels at a time: lane l of a quad forms
// the row terms (|dyz|^2 and the y/z parts of the quadric) of kernel k + (l&3)
// for the quad's row, and each of the four kernels then takes its row terms
// from the quad lane that formed them, passed through LDS (DPP quad
// broadcasts in the fused step kernel, which has no registers to spare for
// the LDS reads).  The row work is done once per (row, kernel) instead of
// once per lane, and every value is the same float expression as in a
// one-kernel-at-a-time walk.
// ---------------------------------------------------------------------------

constexpr int kFwdChunk = 256;

// v broadcast from lane I of each quad to the four lanes of the quad
template <int I>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), I * 0x55, 0xf, 0xf, false));
}

// staged kernel record (LDS): U = {cx, A00, r^2, a} is read by the whole wave
// for one kernel, V0 = {cy, cz, A11, A22} and V1 = {2 A01, 2 A02, 2 A12, 0} by
// the quad lane that forms that kernel's row terms
struct FwdRowTerms {
  float syz, bl, cc;
};

__device__ __forceinline__ FwdRowTerms fwd_row_terms(const float4 V0, const float4 V1, float py, float pz) {
  const float dy = py - V0.x, dz = pz - V0.y;
  FwdRowTerms t;
  t.syz = fmaf(dy, dy, dz * dz);
  t.bl = fmaf(V1.x, dy, V1.y * dz);
  t.cc = fmaf(dy, fmaf(V0.z, dy, V1.z * dz), V0.w * dz * dz);
  return t;
}

// one kernel of a step of four at the lane's two points, with the kernel's
// row terms RT = (syz, bl, cc) at the lane's row
__device__ __forceinline__ void fwd_eval_pair(const float4 U, const float4 RT, float px0, float px1,
                                              unsigned long long act_mask0, unsigned long long act_mask1,
                                              float& acc0, float& acc1, uint32_t& pf) {
  const float syz = RT.x, bl = RT.y, cc = RT.z;
  const float dx0 = px0 - U.x, dx1 = px1 - U.x;
  float q0 = fmaf(dx0, fmaf(U.y, dx0, bl), cc);
  float q1 = fmaf(dx1, fmaf(U.y, dx1, bl), cc);
  const bool in0 = fmaf(dx0, dx0, syz) < U.z;
  const bool in1 = fmaf(dx1, dx1, syz) < U.z;
  q0 = in0 ? q0 : INFINITY;
  q1 = in1 ? q1 : INFINITY;
  acc0 = fmaf(U.w, fast_exp2(-q0), acc0);
  acc1 = fmaf(U.w, fast_exp2(-q1), acc1);
  pf += __popcll(__ballot(in0) & act_mask0) + __popcll(__ballot(in1) & act_mask1);
}

// LDS of the forward tile body for chunks of C kernel records
template <int C>
struct FwdLdsT {
  // records of the chunk, plus an inert record (r^2 < 0, a = 0) at index
  // C that pads each wave's list to a multiple of four.  Each wave's list
  // holds the byte offsets of its records, entry i at slist[i % 4][wave][i / 4]
  // (the four entries of a step in four arrays, read without unpacking).
  float4 srec[C * 3 + 3];
  uint16_t slist[4][4][C / 4 + 1];
  // row terms (syz, bl, cc) of the step's four kernels at each quad's row,
  // twelve floats a quad: every lane writes its kernel's three, every lane
  // reads its quad's twelve (three 16-byte reads)
  float4 sxch[4][16][3];
  int scnt[4][4];
  float sbox[4][6];
  double red_d[4];
  float red_f[4];
  int red_i[4];
  int64_t red_p[4];
};
using FwdLds = FwdLdsT<kFwdChunk>;

// backward tile: a workgroup of W waves (2, 4 or 8; four in the fused step
// kernel), 512 points (512 / (64 W) per thread)
constexpr int kBwdThreads = 256;

// LDS of the backward tile body: the tile's points with a non-zero upstream
// gradient (x, G, G x', G x'^2), row r's points at spx[8 r ...], padded to an
// even count with an inert point (far away, G = 0), and the rows in use
template <int W>
struct BwdLdsT {
  float4 spx[kTile * kTile * kTile];
  float4 srow[kTile * kTile];   // (y, z, first point, point count) of the rows in use
  int swr[kTile * kTile * kTile / (64 * W)][W];
  int64_t spb[W];
  uint32_t wrows[4];            // fused staging (four waves): rows in use of each wave's 16 rows
};
using BwdLds = BwdLdsT<4>;

template <int N>
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kTileLdsBytes = cmax<0>((int)sizeof(FwdLds), (int)sizeof(BwdLds));

// The active slot handled by workgroup b of a grid launch over n slots.
// chunk 0: slot b.  chunk C > 0: the slots are cut into runs of C
// consecutive slots (neighbouring tiles, sharing most of their kernels),
// dealt to the eight XCDs round-robin, since workgroup b runs on XCD b % 8;
// each XCD then works on a few runs at a time and finds their kernel records
// in its own L2.  The grid is padded to a multiple of 8 C; padding
// workgroups get -1.  A bijection of [0, padded grid) onto the slots and -1.
__device__ __forceinline__ int tile_slot(int b, int n, int chunk) {
  if (chunk <= 0) return b;
  const int x = b & 7, k = b >> 3;
  const int slot = ((k / chunk) * 8 + x) * chunk + (k % chunk);
  return slot < n ? slot : -1;
}

// The slot at launch position pos (-1: none): the pos-th entry of the launch
// order (the active tiles, longest list first) or, without it, slot pos.
__device__ __forceinline__ int ordered_slot(const Dev& D, int pos) {
  return pos < 0 ? -1 : (D.tile_order_on ? D.tile_order[pos] : pos);
}

__device__ void bwd_stage_from_registers(const Dev& D, const LevelDev& L, int slot, int tx, int ty, int tz,
                                         const float g[2], BwdLds& B, int64_t beg, int64_t end);

template <bool LOSS, bool BWD, int C>
__device__ __forceinline__ void forward_tile(const Dev& D, const int slot, float* __restrict__ f_out,
                                             float tau1, float tau2, char* lds) {
  FwdLdsT<C>& F = *reinterpret_cast<FwdLdsT<C>*>(lds);
  float4* srec = F.srec;
  auto& slist = F.slist;
  auto& scnt = F.scnt;
  auto& sbox = F.sbox;
  double* red_d = F.red_d;
  float* red_f = F.red_f;
  int* red_i = F.red_i;
  int64_t* red_p = F.red_p;

  const int2 lt = D.slot_tile[slot];
  const LevelDev L = D.levels[lt.x];
  if (L.kind != kLevelGrid) return;   // sample tiles: k_sample_forward
  const int n = L.n, nt = L.nt;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int tz = lt.y / (nt * nt), ty = (lt.y / nt) % nt, tx = lt.y % nt;

  const int xi0 = tx * kTile + 2 * (lane & 3);
  const int yi = ty * kTile + 4 * (wv & 1) + ((lane >> 2) & 3);
  const int zi = tz * kTile + 4 * (wv >> 1) + (lane >> 4);
  const float px0 = L.axis[min(xi0, n - 1)];
  const float px1 = L.axis[min(xi0 + 1, n - 1)];
  const float py = L.axis[min(yi, n - 1)];
  const float pz = L.axis[min(zi, n - 1)];

  // training points of this lane (inside the grid and the level's mask)
  const bool vyz = yi < n && zi < n;
  const int64_t local0 = ((int64_t)min(zi, n - 1) * n + min(yi, n - 1)) * n + min(xi0, n - 1);
  const bool act0 = vyz && xi0 < n && point_active(L.bits, local0);
  const bool act1 = vyz && xi0 + 1 < n && point_active(L.bits, local0 + 1);
  const unsigned long long act_mask0 = __ballot(act0), act_mask1 = __ballot(act1);
  int64_t pfw = 0;   // in-ball pairs at this wave's training points (wave-uniform)

  // the first chunk's records, read while the boxes below are formed
  const int64_t beg = min((int64_t)D.tile_start[slot], D.pair_cap);
  const int64_t end = min((int64_t)D.tile_start[slot + 1], D.pair_cap);
  float4 f0 = make_float4(0.f, 0.f, 0.f, 0.f), f1 = f0, f2 = f0;
  if (tid < end - beg && tid < C) {
    const int j = D.items[beg + tid];
    f0 = D.rec[3 * j];
    f1 = D.rec[3 * j + 1];
    f2 = D.rec[3 * j + 2];
  }

  // bounding box of each wave's training points (its list holds the kernels
  // whose ball meets it; a wave without training points walks nothing)
  {
    const bool any = act0 || act1;
    const int xlo = act0 ? xi0 : (act1 ? xi0 + 1 : INT_MAX), xhi = act1 ? xi0 + 1 : (act0 ? xi0 : -1);
    const int bxlo = -wave_max_i(-xlo), bxhi = wave_max_i(xhi);
    const int bylo = -wave_max_i(any ? -yi : -INT_MAX), byhi = wave_max_i(any ? yi : -1);
    const int bzlo = -wave_max_i(any ? -zi : -INT_MAX), bzhi = wave_max_i(any ? zi : -1);
    if (lane == 0 && (act_mask0 | act_mask1) != 0ull) {
      sbox[wv][0] = L.axis[bxlo]; sbox[wv][1] = L.axis[bxhi];
      sbox[wv][2] = L.axis[bylo]; sbox[wv][3] = L.axis[byhi];
      sbox[wv][4] = L.axis[bzlo]; sbox[wv][5] = L.axis[bzhi];
    } else if (lane == 0) {
      // no training point: an empty box (every distance test fails)
      sbox[wv][0] = INFINITY; sbox[wv][1] = -INFINITY;
      sbox[wv][2] = INFINITY; sbox[wv][3] = -INFINITY;
      sbox[wv][4] = INFINITY; sbox[wv][5] = -INFINITY;
    }
  }
  __syncthreads();

  float acc0 = 0.f, acc1 = 0.f;
  if (tid < 3) srec[3 * C + tid] = make_float4(0.f, 0.f, tid == 0 ? -1.f : 0.f, 0.f);
  // a record into the chunk's LDS (the first chunk's before the loop, so
  // that its registers are free again)
  auto stage = [&](const float4 a0, const float4 a1, const float4 a2) {
    srec[3 * tid] = make_float4(a0.x, a1.x, a0.w, a2.z);
    srec[3 * tid + 1] = make_float4(a0.y, a0.z, a1.y, a1.z);
    srec[3 * tid + 2] = make_float4(a1.w, a2.x, a2.y, 0.f);
  };
  if (tid < end - beg && tid < C) stage(f0, f1, f2);

  for (int64_t c0 = beg; c0 < end; c0 += C) {
    const int cnt = (int)min((int64_t)C, end - c0);
    uint32_t mybits = 0;
    if (tid < cnt) {
      if (c0 != beg) {
        const int j = D.items[c0 + tid];
        stage(D.rec[3 * j], D.rec[3 * j + 1], D.rec[3 * j + 2]);
      }
      // the waves whose box the record's padded ball meets (this thread's
      // own LDS entries: c, r^2)
      const float4 u = srec[3 * tid], v = srec[3 * tid + 1];
      const float cx = u.x, cy = v.x, cz = v.y;
      const float rr = sqrtf(u.z) * (1.0f + 1e-5f) + 1e-6f;
      const float rc2 = rr * rr;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const float ex = fmaxf(fmaxf(sbox[w][0] - cx, cx - sbox[w][1]), 0.f);
        const float ey = fmaxf(fmaxf(sbox[w][2] - cy, cy - sbox[w][3]), 0.f);
        const float ez = fmaxf(fmaxf(sbox[w][4] - cz, cz - sbox[w][5]), 0.f);
        if (ex * ex + ey * ey + ez * ez < rc2) mybits |= 1u << w;
      }
    }
    // compact per-wave lists in chunk order
    int prefix[4];
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const unsigned long long bal = __ballot((mybits >> w) & 1u);
      prefix[w] = __popcll(bal & lt_mask);
      if (lane == 0) scnt[w][wv] = __popcll(bal);
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if ((mybits >> w) & 1u) {
        int off = prefix[w];
        for (int v = 0; v < wv; ++v) off += scnt[w][v];
        slist[off & 3][w][off >> 2] = (uint16_t)(tid * (int)sizeof(float4) * 3);   // byte offset of the record
      }
    }
    const int len = __builtin_amdgcn_readfirstlane(scnt[wv][0] + scnt[wv][1] + scnt[wv][2] + scnt[wv][3]);
    const int len4 = (len + 3) & ~3;
    // the wave pads its own list (entries [len, len4), written by no other wave)
    if (lane < len4 - len) slist[(len + lane) & 3][wv][(len + lane) >> 2] = (uint16_t)(C * (int)sizeof(float4) * 3);
    __syncthreads();
    const char* srec_b = reinterpret_cast<const char*>(srec);
    uint32_t pf = 0;
    float4* xq = F.sxch[wv][lane >> 2];   // this lane's quad's row terms
    float* xw = reinterpret_cast<float*>(xq) + 3 * (lane & 3);
    for (int k = 0; k < len4; k += 4) {
      const int q = k >> 2;
      const float4* own = reinterpret_cast<const float4*>(srec_b + slist[lane & 3][wv][q]);
      const FwdRowTerms t = fwd_row_terms(own[1], own[2], py, pz);
      float4 T0, T1, T2, T3;
      if (BWD) {
        // (the fused step kernel, short of registers: DPP quad broadcasts)
        T0 = make_float4(quad_bcast<0>(t.syz), quad_bcast<0>(t.bl), quad_bcast<0>(t.cc), 0.f);
        T1 = make_float4(quad_bcast<1>(t.syz), quad_bcast<1>(t.bl), quad_bcast<1>(t.cc), 0.f);
        T2 = make_float4(quad_bcast<2>(t.syz), quad_bcast<2>(t.bl), quad_bcast<2>(t.cc), 0.f);
        T3 = make_float4(quad_bcast<3>(t.syz), quad_bcast<3>(t.bl), quad_bcast<3>(t.cc), 0.f);
      } else {
        // the quad's four row terms pass through LDS (no VALU work): the LDS
        // operations of one wave complete in order, so the reads return this
        // step's writes
        xw[0] = t.syz;
        xw[1] = t.bl;
        xw[2] = t.cc;
        __builtin_amdgcn_wave_barrier();
        const float4 X0 = xq[0], X1 = xq[1], X2 = xq[2];
        T0 = make_float4(X0.x, X0.y, X0.z, 0.f);
        T1 = make_float4(X0.w, X1.x, X1.y, 0.f);
        T2 = make_float4(X1.z, X1.w, X2.x, 0.f);
        T3 = make_float4(X2.y, X2.z, X2.w, 0.f);
      }
      const float4 U0 = *reinterpret_cast<const float4*>(srec_b + slist[0][wv][q]);
      const float4 U1 = *reinterpret_cast<const float4*>(srec_b + slist[1][wv][q]);
      const float4 U2 = *reinterpret_cast<const float4*>(srec_b + slist[2][wv][q]);
      const float4 U3 = *reinterpret_cast<const float4*>(srec_b + slist[3][wv][q]);
      fwd_eval_pair(U0, T0, px0, px1, act_mask0, act_mask1, acc0, acc1, pf);
      fwd_eval_pair(U1, T1, px0, px1, act_mask0, act_mask1, acc0, acc1, pf);
      fwd_eval_pair(U2, T2, px0, px1, act_mask0, act_mask1, acc0, acc1, pf);
      fwd_eval_pair(U3, T3, px0, px1, act_mask0, act_mask1, acc0, acc1, pf);
      __builtin_amdgcn_wave_barrier();   // the next step's writes come after these reads
    }
    pfw += pf;
    __syncthreads();
  }

  // epilogue
  double l2 = 0.0;
  float mxe = 0.f;
  int cnt_id = 0;
  float gv[2] = {0.f, 0.f};   // G = 2E at the lane's two points (0 outside id_all or the grid)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int xi = xi0 + h;
    if (!(vyz && xi < n)) continue;
    const int64_t local = ((int64_t)zi * n + yi) * n + xi;
    const int64_t idx = L.pt_base + local;
    const bool act = point_active(L.bits, local);
    const float f = act ? (h ? acc1 : acc0) : 0.f;
    if (f_out) f_out[idx] = f;
    if (LOSS) {
      const float t = L.target[local];
      const bool id0 = tau1 < t && t < tau2;
      const bool id1 = t <= tau1 && f > tau1;
      const bool id2 = t >= tau2 && f < tau2;
      const bool in = act && (id0 || id1 || id2);
      const float E = in ? f - t : 0.f;
      gv[h] = 2.f * E;
      D.G[idx] = gv[h];
      l2 += (double)E * (double)E;
      mxe = fmaxf(mxe, fabsf(E));
      cnt_id += in ? 1 : 0;
    }
  }
  if (LOSS) {
    l2 = wave_sum(l2);
    mxe = wave_max_f(mxe);
    cnt_id = wave_sum(cnt_id);
  }
  if (lane == 0) { red_d[wv] = l2; red_f[wv] = mxe; red_i[wv] = cnt_id; red_p[wv] = pfw; }
  __syncthreads();
  if (tid == 0) {
    TileStat ts;
    ts.l2 = (red_d[0] + red_d[1]) + (red_d[2] + red_d[3]);
    ts.max_abs_e = fmaxf(fmaxf(red_f[0], red_f[1]), fmaxf(red_f[2], red_f[3]));
    ts.n_idall = red_i[0] + red_i[1] + red_i[2] + red_i[3];
    ts.p_fwd = (red_p[0] + red_p[1]) + (red_p[2] + red_p[3]);
    D.tstat[slot] = ts;
  }
  if (BWD) {
    // the backward of the same tile: G of its points is in registers, and
    // the list's records were just read (L2)
    __syncthreads();   // the forward's LDS is no longer read
    bwd_stage_from_registers(D, L, slot, tx, ty, tz, gv, *reinterpret_cast<BwdLds*>(lds), beg, end);
  }
}

// one workgroup per tile (grid launch) ...  Eight waves per SIMD (at most 64
// VGPRs) keep the exp / LDS latencies of the walk hidden.
template <bool LOSS, int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_forward(Dev D, float* __restrict__ f_out, float tau1, float tau2, int n_slots) {
  __shared__ __align__(16) char lds[sizeof(FwdLdsT<C>)];
  const int slot = ordered_slot(D, tile_slot(blockIdx.x, n_slots, D.slot_chunk));
  if (slot < 0) return;
  forward_tile<LOSS, false, C>(D, slot, f_out, tau1, tau2, lds);
}

// ... or a persistent grid: each workgroup walks the tiles round-robin
// (slot = blockIdx.x, blockIdx.x + gridDim.x, ...).  The walk depends only on
// blockIdx and gridDim, so every branch of the loop is uniform and every
// barrier inside the tile body is reached by the whole workgroup.
template <bool LOSS, int C>
__global__ __launch_bounds__(256) void k_forward_persistent(Dev D, float* __restrict__ f_out, float tau1,
                                                            float tau2, int n_slots) {
  __shared__ __align__(16) char lds[sizeof(FwdLdsT<C>)];
  for (int pos = blockIdx.x; pos < n_slots; pos += gridDim.x) {
    forward_tile<LOSS, false, C>(D, ordered_slot(D, pos), f_out, tau1, tau2, lds);
    __syncthreads();
  }
}

// The step's tile kernel: forward and loss, then the backward moments of the
// same tile (the two bodies of k_forward<true> and k_bwd_tiles, with the
// backward's points staged from the forward's registers; results equal those
// of the two kernels bit for bit).  The LDS of the two bodies overlaps.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void k_step_tiles(Dev D, float* __restrict__ f_out, float tau1, float tau2, int n_slots) {
  __shared__ __align__(16) char lds[kTileLdsBytes];
  const int slot = ordered_slot(D, tile_slot(blockIdx.x, n_slots, D.slot_chunk));
  if (slot < 0) return;
  forward_tile<true, true, kFwdChunk>(D, slot, f_out, tau1, tau2, lds);
}

__global__ __launch_bounds__(256) void k_step_tiles_persistent(Dev D, float* __restrict__ f_out, float tau1,
                                                               float tau2, int n_slots) {
  __shared__ __align__(16) char lds[kTileLdsBytes];
  for (int pos = blockIdx.x; pos < n_slots; pos += gridDim.x) {
    forward_tile<true, true, kFwdChunk>(D, ordered_slot(D, pos), f_out, tau1, tau2, lds);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// mini-batch forward: one wave per batch point walks the kernel list of the
// point's tile (lanes strided over the list, then a fixed butterfly), then
// forms E and G = 2E at the point and its loss records (eq. 3-9, 3-15-1,
// 3-18, 3-19 restricted to the batch)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_batch_forward(Dev D, const int64_t* __restrict__ pts, int n_pts,
                                                       float* __restrict__ f_out, float tau1, float tau2) {
  const int lane = threadIdx.x & 63;
  const int k = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (k >= n_pts) return;
  const int64_t gi = pts[k];
  // the level holding point gi (levels are ordered by pt_base)
  int li = 0;
  for (int a = 1; a < D.n_levels_total; ++a)
    if (D.levels[a].pt_base <= gi) li = a;
  const LevelDev L = D.levels[li];
  const int n = L.n, nt = L.nt;
  const int64_t local = gi - L.pt_base;
  const bool samples = L.kind == kLevelSamples;
  bool valid;
  if (samples)
    valid = gi >= 0 && L.sxyz != nullptr && local >= 0 && local < (int64_t)L.n_samples;
  else
    valid = gi >= 0 && L.axis != nullptr && local >= 0 && local < (int64_t)n * n * n && point_active(L.bits, local);
  int slot = -1;
  float px = 0.f, py = 0.f, pz = 0.f;
  if (valid && samples) {
    slot = L.sslot[local];
    px = L.sxyz[3 * local];
    py = L.sxyz[3 * local + 1];
    pz = L.sxyz[3 * local + 2];
  } else if (valid) {
    const int xi = (int)(local % n);
    const int yi = (int)((local / n) % n);
    const int zi = (int)(local / ((int64_t)n * n));
    slot = D.tile_map[L.tmap0 + ((zi / kTile) * nt + yi / kTile) * nt + xi / kTile];
    px = L.axis[xi];
    py = L.axis[yi];
    pz = L.axis[zi];
  }
  float acc = 0.f;
  int cnt = 0;
  if (slot >= 0) {
    const int64_t beg = min((int64_t)D.tile_start[slot], D.pair_cap);
    const int64_t end = min((int64_t)D.tile_start[slot + 1], D.pair_cap);
    for (int64_t e = beg + lane; e < end; e += 64) {
      const int j = D.items[e];
      const float4 a0 = D.rec[3 * j], a1 = D.rec[3 * j + 1], a2 = D.rec[3 * j + 2];
      const float dx = px - a0.x, dy = py - a0.y, dz = pz - a0.z;
      const bool in = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < a0.w;
      float q = fmaf(dx, fmaf(a1.x, dx, fmaf(a1.w, dy, a2.x * dz)), fmaf(dy, fmaf(a1.y, dy, a2.y * dz), a1.z * dz * dz));
      q = in ? q : INFINITY;
      acc = fmaf(a2.z, fast_exp2(-q), acc);
      cnt += in ? 1 : 0;
    }
  }
  const float f = wave_sum(acc);
  const int pf = wave_sum(cnt);
  if (lane != 0) return;
  float E = 0.f;
  bool id = false;
  if (valid && (samples || L.target)) {
    const float t = samples ? 1.f : L.target[local];   // surface samples carry label 1
    id = (tau1 < t && t < tau2) || (t <= tau1 && f > tau1) || (t >= tau2 && f < tau2);
    E = id ? f - t : 0.f;
  }
  if (valid) D.G[gi] = 2.f * E;
  if (f_out) f_out[k] = valid ? f : 0.f;
  D.b_l2[k] = (double)E * (double)E;
  D.b_abs[k] = fabsf(E);
  D.b_id[k] = id ? 1 : 0;
  D.b_pf[k] = valid ? pf : 0;
  D.b_shape[k] = valid ? L.shape : -1;
}

// tiles holding batch points (the mini-batch's bucket selection)
__global__ __launch_bounds__(256) void k_batch_tiles(Dev D, const int64_t* __restrict__ pts, int n_pts,
                                                     int32_t* __restrict__ sel) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n_pts) return;
  const int64_t gi = pts[k];
  int li = 0;
  for (int a = 1; a < D.n_levels_total; ++a)
    if (D.levels[a].pt_base <= gi) li = a;
  const LevelDev& L = D.levels[li];
  const int64_t local = gi - L.pt_base;
  int slot = -1;
  if (L.kind == kLevelSamples) {
    if (gi >= 0 && L.sxyz != nullptr && local >= 0 && local < (int64_t)L.n_samples) slot = L.sslot[local];
  } else if (gi >= 0 && L.axis != nullptr && local >= 0 && local < (int64_t)L.n * L.n * L.n) {
    const int n = L.n, nt = L.nt;
    const int xi = (int)(local % n), yi = (int)((local / n) % n), zi = (int)(local / ((int64_t)n * n));
    slot = D.tile_map[L.tmap0 + ((zi / kTile) * nt + yi / kTile) * nt + xi / kTile];
  }
  if (slot >= 0) sel[slot] = 1;
}

// Zero moments for entries [c_lo, c_hi) of the tile-major lists (tiles whose
// points all have G = 0), so that every entry's partial is written each step
// and the reduce reads them without checks.
__device__ __forceinline__ void zero_partials(const Dev& D, int64_t c_lo, int64_t c_hi, int tid, int nthreads) {
  for (int64_t c = c_lo + tid; c < c_hi; c += nthreads) {
    const int eo = D.tile_e[c];
    if (eo < 0) continue;   // past the list capacity (overflow)
    float2* o = D.partials + 5 * (int64_t)eo;
#pragma unroll
    for (int i = 0; i < 5; ++i) o[i] = make_float2(0.f, 0.f);
  }
}

// ---------------------------------------------------------------------------
// surface samples (label 1, eq. 3-10 on the surface).  A sample level bins
// its samples into the 8^3-cell tiles of an n^3-cell grid; a tile's box is
// its cells (the level's pad is half a cell), so every sample lies in its
// tile's box and the tile's kernel list, built like a grid tile's, holds
// every kernel whose ball reaches it.  One workgroup per active sample tile;
// the pair arithmetic is the grid kernels' expression for expression.
// ---------------------------------------------------------------------------

// Each active sample tile's kernel list is cut into samp_split contiguous
// parts (in the backward, whole rounds of 256 kernels), one workgroup each.  Forward: the part's kernel records are staged
// in LDS and every lane takes one sample of the tile, so a record serves
// 256 samples; each (sample, part) sum goes to a scratch slot, and a second
// pass adds a sample's parts in order, forms E and G and the tile's
// statistics.  Backward: every lane takes one kernel of the part and walks
// the tile's samples, staged in LDS with their G.
__global__ __launch_bounds__(256) void k_sample_forward(Dev D) {
  __shared__ float4 srec[kFwdChunk * 3];
  const int slot = D.samp_slots[blockIdx.x];
  const int2 lt = D.slot_tile[slot];
  const LevelDev L = D.levels[lt.x];
  const int tid = threadIdx.x;
  const int s0 = L.sstart[slot - L.slot0], s1 = L.sstart[slot - L.slot0 + 1];
  const int64_t beg = min((int64_t)D.tile_start[slot], D.pair_cap);
  const int64_t end = min((int64_t)D.tile_start[slot + 1], D.pair_cap);
  const int64_t part = (end - beg + D.samp_split - 1) / D.samp_split;
  const int64_t rb = min(end, beg + part * blockIdx.y), re = min(end, rb + part);
  const int64_t gbase = L.spos - D.samp_pos;   // this level's first entry of the sorted sample arrays
  for (int sb = s0; sb < s1; sb += 256) {
    const int si = sb + tid;
    const bool valid = si < s1;
    const float4 P = valid ? L.spos[si] : make_float4(1e30f, 1e30f, 1e30f, 0.f);
    float acc = 0.f;
    int cnt = 0;
    for (int64_t c0 = rb; c0 < re; c0 += kFwdChunk) {
      const int nc = (int)min((int64_t)kFwdChunk, re - c0);
      __syncthreads();   // the previous chunk's records are no longer read
      if (tid < nc) {
        const int j = D.items[c0 + tid];
        srec[3 * tid] = D.rec[3 * j];
        srec[3 * tid + 1] = D.rec[3 * j + 1];
        srec[3 * tid + 2] = D.rec[3 * j + 2];
      }
      __syncthreads();
      for (int k = 0; k < nc; ++k) {
        const float4 a0 = srec[3 * k], a1 = srec[3 * k + 1], a2 = srec[3 * k + 2];
        const float dx = P.x - a0.x, dy = P.y - a0.y, dz = P.z - a0.z;
        const bool in = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < a0.w;
        float q = fmaf(dx, fmaf(a1.x, dx, fmaf(a1.w, dy, a2.x * dz)), fmaf(dy, fmaf(a1.y, dy, a2.y * dz), a1.z * dz * dz));
        q = in ? q : INFINITY;
        acc = fmaf(a2.z, fast_exp2(-q), acc);
        cnt += in ? 1 : 0;
      }
    }
    if (valid) {
      const int64_t o = (gbase + si) * kSampSplitMax + blockIdx.y;
      D.samp_f[o] = acc;
      D.samp_c[o] = cnt;
    }
  }
}

// per sample tile: each sample's parts added in order, f, E = f - 1 and
// G = 2E, and the tile's statistics
template <bool LOSS>
__global__ __launch_bounds__(256) void k_sample_fwd_final(Dev D, float* __restrict__ f_out, float tau1, float tau2) {
  __shared__ double red_d[4];
  __shared__ float red_f[4];
  __shared__ int red_i[4];
  __shared__ int64_t red_p[4];
  const int slot = D.samp_slots[blockIdx.x];
  const int2 lt = D.slot_tile[slot];
  const LevelDev L = D.levels[lt.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int s0 = L.sstart[slot - L.slot0], s1 = L.sstart[slot - L.slot0 + 1];
  const int64_t gbase = L.spos - D.samp_pos;
  double l2 = 0.0;
  float mxe = 0.f;
  int cnt_id = 0;
  int64_t pfw = 0;
  for (int si = s0 + tid; si < s1; si += 256) {
    float f = 0.f;
    int pf = 0;
    const int64_t o = (gbase + si) * kSampSplitMax;
    for (int y = 0; y < D.samp_split; ++y) {
      f += D.samp_f[o + y];
      pf += D.samp_c[o + y];
    }
    const int64_t idx = L.pt_base + __float_as_int(L.spos[si].w);
    if (f_out) f_out[idx] = f;
    if (LOSS) {
      const float t = 1.f;   // surface samples carry label 1
      const bool id = (tau1 < t && t < tau2) || (t <= tau1 && f > tau1) || (t >= tau2 && f < tau2);
      const float E = id ? f - t : 0.f;
      D.G[idx] = 2.f * E;
      l2 += (double)E * (double)E;
      mxe = fmaxf(mxe, fabsf(E));
      cnt_id += id ? 1 : 0;
    }
    pfw += pf;
  }
  l2 = wave_sum(l2);
  mxe = wave_max_f(mxe);
  cnt_id = wave_sum(cnt_id);
  pfw = wave_sum(pfw);
  if (lane == 0) { red_d[wv] = l2; red_f[wv] = mxe; red_i[wv] = cnt_id; red_p[wv] = pfw; }
  __syncthreads();
  if (tid == 0) {
    TileStat ts;
    ts.l2 = (red_d[0] + red_d[1]) + (red_d[2] + red_d[3]);
    ts.max_abs_e = fmaxf(fmaxf(red_f[0], red_f[1]), fmaxf(red_f[2], red_f[3]));
    ts.n_idall = red_i[0] + red_i[1] + red_i[2] + red_i[3];
    ts.p_fwd = (red_p[0] + red_p[1]) + (red_p[2] + red_p[3]);
    D.tstat[slot] = ts;
  }
}

__global__ __launch_bounds__(256) void k_sample_bwd(Dev D, const float* __restrict__ Gsrc) {
  constexpr int kStage = 1024;
  __shared__ float4 sp[kStage];
  __shared__ int64_t spb[4];
  const int slot = D.samp_slots[blockIdx.x];
  const int2 lt = D.slot_tile[slot];
  const LevelDev L = D.levels[lt.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int s0 = L.sstart[slot - L.slot0], s1 = L.sstart[slot - L.slot0 + 1];
  const int64_t beg = min((int64_t)D.tile_start[slot], D.pair_cap);
  const int64_t end = min((int64_t)D.tile_start[slot + 1], D.pair_cap);
  // parts of whole rounds of 256 kernels, so that every lane has one
  const int64_t part = (((end - beg + D.samp_split - 1) / D.samp_split + 255) / 256) * 256;
  const int64_t rb = min(end, beg + part * blockIdx.y), re = min(end, rb + part);
  int nz = 0;
  for (int si = s0 + tid; si < s1; si += 256) nz |= Gsrc[L.pt_base + __float_as_int(L.spos[si].w)] != 0.f ? 1 : 0;
  if (!__syncthreads_or(nz)) {
    zero_partials(D, rb, re, tid, 256);
    if (tid == 0) D.samp_pb[(int64_t)blockIdx.x * kSampSplitMax + blockIdx.y] = 0;
    return;
  }
  int64_t pb = 0;
  for (int64_t c0 = rb; c0 < re; c0 += 256) {
    const int64_t e = c0 + tid;
    const bool have = e < re;
    float4 r0 = make_float4(0.f, 0.f, 0.f, -1.f), r1 = make_float4(0.f, 0.f, 0.f, 0.f),
           r2 = make_float4(0.f, 0.f, 0.f, 0.f);
    int e_out = 0;
    if (have) {
      const int j = D.items[e];
      e_out = D.tile_e[e];
      r0 = D.rec[3 * j];
      r1 = D.rec[3 * j + 1];
      r2 = D.rec[3 * j + 2];
    }
    float T[10];
#pragma unroll
    for (int i = 0; i < 10; ++i) T[i] = 0.f;
    uint32_t pbg = 0;
    for (int sb = s0; sb < s1; sb += kStage) {
      const int ns = min(kStage, s1 - sb);
      __syncthreads();   // the previous stage is no longer read
      for (int q = tid; q < ns; q += 256) {
        const float4 P = L.spos[sb + q];
        sp[q] = make_float4(P.x, P.y, P.z, Gsrc[L.pt_base + __float_as_int(P.w)]);
      }
      __syncthreads();
      for (int k = 0; k < ns; ++k) {
        const float4 P = sp[k];
        const float dx = P.x - r0.x, dy = P.y - r0.y, dz = P.z - r0.z;
        const bool in = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < r0.w;
        float q = fmaf(dx, fmaf(r1.x, dx, fmaf(r1.w, dy, r2.x * dz)), fmaf(dy, fmaf(r1.y, dy, r2.y * dz), r1.z * dz * dz));
        q = in ? q : INFINITY;
        const float g = P.w * fast_exp2(-q);
        const float gx = g * dx, gy = g * dy, gz = g * dz;
        T[0] += g;
        T[1] += gx;
        T[2] += gy;
        T[3] += gz;
        T[4] = fmaf(gx, dx, T[4]);
        T[5] = fmaf(gx, dy, T[5]);
        T[6] = fmaf(gx, dz, T[6]);
        T[7] = fmaf(gy, dy, T[7]);
        T[8] = fmaf(gy, dz, T[8]);
        T[9] = fmaf(gz, dz, T[9]);
        pbg += (in && P.w != 0.f) ? 1u : 0u;
      }
    }
    pb += pbg;
    if (have && e_out >= 0) {
      float2* o = D.partials + 5 * (int64_t)e_out;
#pragma unroll
      for (int i = 0; i < 5; ++i) o[i] = make_float2(T[2 * i], T[2 * i + 1]);
    }
  }
  pb = wave_sum(pb);
  if (lane == 0) spb[wv] = pb;
  __syncthreads();
  if (tid == 0) D.samp_pb[(int64_t)blockIdx.x * kSampSplitMax + blockIdx.y] = (spb[0] + spb[1]) + (spb[2] + spb[3]);
}

// per sample tile: in-ball pairs with G != 0 of its samp_split workgroups
__global__ __launch_bounds__(64) void k_sample_bwd_sum(Dev D) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= D.n_samp_slots) return;
  int64_t t = 0;
  for (int y = 0; y < D.samp_split; ++y) t += D.samp_pb[(int64_t)i * kSampSplitMax + y];
  D.tile_pbwd[D.samp_slots[i]] = t;
}

// ---------------------------------------------------------------------------
// backward, stage 1: one workgroup per active tile.  The tile's points with a
// non-zero upstream gradient are staged in LDS in (z, y, x) order; each lane
// owns one kernel of the tile's list and walks those points, so every branch
// of the walk (row changes, empty tiles) is uniform across the wave.  Per
// row the lane keeps three sums over x (sum g, sum g dx, sum g dx^2) and folds
// them into the ten moments with the row's dy, dz:
//   T0 = sum g, T1 = sum g D, T2 = sum g D D^T,  g = G exp(-D^T A D)
// A point is staged with G, G x' and G x'^2, x' its offset from the tile's
// first x, so the row sums cost three FMAs per point: with c' the kernel's
// offset from that x, sum g dx = sum G e x' - c' sum G e and
// sum g dx^2 = sum G e x'^2 - 2 c' sum G e x' + c'^2 sum G e (e = exp(...)).
// The moments of each (tile, kernel) entry go to `partials`.
// ---------------------------------------------------------------------------

// (Four waves per workgroup share a tile's kernel groups of 64; two or eight
// waves measured slower on the 256^3 snapshot.)

// The walk over the staged rows, once the tile's R rows are in B: each wave
// takes its own groups of 64 kernels of the list [beg, end) (waves past the
// end of the list do no work); the first group's kernel of each lane (jf, ef,
// record f0..f2) was read while the points were staged.
template <int W>
__device__ __forceinline__ void bwd_walk(const Dev& D, const int slot, BwdLdsT<W>& B, const int R, const float xref,
                                         const int64_t end, const int64_t cf, const int ef, const float4 f0,
                                         const float4 f1, const float4 f2) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  int64_t pb = 0;   // in-ball pairs at non-zero points (wave-uniform)
  for (int64_t c0 = cf; c0 < end; c0 += 64 * W) {
    const bool have = c0 + lane < end;
    float4 r0 = f0, r1 = f1, r2 = f2;   // the first group's, read during staging
    int e_out = ef;
    if (c0 != cf) {
      r0 = make_float4(0.f, 0.f, 0.f, -1.f);
      r1 = r2 = make_float4(0.f, 0.f, 0.f, 0.f);
      e_out = 0;
      if (have) {
        const int j = D.items[c0 + lane];
        e_out = D.tile_e[c0 + lane];
        r0 = D.rec[3 * j];
        r1 = D.rec[3 * j + 1];
        r2 = D.rec[3 * j + 2];
      }
    }
    const float cx = r0.x, cy = r0.y, cz = r0.z, rad2 = r0.w;
    const float A00 = r1.x, A11 = r1.y, A22 = r1.z, A01x2 = r1.w, A02x2 = r2.x, A12x2 = r2.y;
    const float co = cx - xref, m2co = -2.f * co, co2 = co * co;
    float T[10];
#pragma unroll
    for (int i = 0; i < 10; ++i) T[i] = 0.f;
    uint32_t pbg = 0;
    // Per row the point sums (s0, t1, t2) = sums of (G e, G e x', G e x'^2)
    // are turned into sums of (g, g dx, g dx^2) about the kernel's centre and
    // folded with the row's dy, dz into the moments.  Rows come in ascending
    // (z, y), so the dz terms of the quadric are formed once per z plane (the
    // same values as per row: the results do not change).
    int plane = -1;
    float dz = 0.f, dz2 = 0.f, A02dz = 0.f, A12dz = 0.f, A22dzz = 0.f;
    for (int r = 0; r < R; ++r) {
      const float4 RW = B.srow[r];
      const int k0 = __builtin_amdgcn_readfirstlane(__float_as_int(RW.z));
      const int kn = __builtin_amdgcn_readfirstlane(__float_as_int(RW.w)) >> 1;
      const int pl = k0 >> 6;   // the row's z within the tile (row index 8 z + y, 8 points each)
      if (pl != plane) {        // wave-uniform
        plane = pl;
        dz = RW.y - cz;
        dz2 = dz * dz;
        A02dz = A02x2 * dz;
        A12dz = A12x2 * dz;
        A22dzz = A22 * dz * dz;
      }
      const float dy = RW.x - cy;
      const float syz = fmaf(dy, dy, dz2);
      const float bl = fmaf(A01x2, dy, A02dz);
      const float cc = fmaf(dy, fmaf(A11, dy, A12dz), A22dzz);
      // sums of G e, G e x', G e x'^2 over the row (s0, t1, t2); the row's
      // first point starts them (every row in use holds at least one pair)
      float s0, t1, t2;
      auto point = [&](const float4 PP, bool first) {
        const float dx = PP.x - cx;
        const bool in = fmaf(dx, dx, syz) < rad2;
        float q = fmaf(dx, fmaf(A00, dx, bl), cc);
        q = in ? q : INFINITY;
        const float e = fast_exp2(-q);
        s0 = first ? PP.y * e : fmaf(PP.y, e, s0);
        t1 = first ? PP.z * e : fmaf(PP.z, e, t1);
        t2 = first ? PP.w * e : fmaf(PP.w, e, t2);
        pbg += __popcll(__ballot(in));
      };
      // a row holds one to four point pairs (kn, wave-uniform); the pairs
      // are unrolled so their LDS reads take fixed offsets from the row
      const float4* rp = B.spx + k0;
      point(rp[0], true);
      point(rp[1], false);
      if (kn >= 2) {
        point(rp[2], false);
        point(rp[3], false);
      }
      if (kn >= 3) {
        point(rp[4], false);
        point(rp[5], false);
      }
      if (kn >= 4) {
        point(rp[6], false);
        point(rp[7], false);
      }
      // sum g dx and sum g dx^2 about the kernel's centre
      const float s1 = fmaf(-co, s0, t1);
      const float s2 = fmaf(co2, s0, fmaf(m2co, t1, t2));
      T[0] += s0; T[1] += s1; T[2] = fmaf(dy, s0, T[2]); T[3] = fmaf(dz, s0, T[3]);
      T[4] += s2; T[5] = fmaf(dy, s1, T[5]); T[6] = fmaf(dz, s1, T[6]);
      T[7] = fmaf(dy * dy, s0, T[7]); T[8] = fmaf(dy * dz, s0, T[8]); T[9] = fmaf(dz2, s0, T[9]);
    }
    pb += pbg;
    if (have && e_out >= 0) {
      float2* o = D.partials + 5 * (int64_t)e_out;   // kernel-major: the reduce reads it in order
#pragma unroll
      for (int i = 0; i < 5; ++i) o[i] = make_float2(T[2 * i], T[2 * i + 1]);
    }
  }
  if (lane == 0) B.spb[wv] = pb;
  __syncthreads();
  if (tid == 0) {
    int64_t t = 0;
    for (int v = 0; v < W; ++v) t += B.spb[v];
    D.tile_pbwd[slot] = t;
  }
}

// The kernel each lane owns in its wave's first group of the list, read
// while the points are staged.
struct BwdFirst {
  int64_t cf;
  int ef;
  float4 f0, f1, f2;
};

__device__ __forceinline__ BwdFirst bwd_first_group(const Dev& D, int64_t beg, int64_t end) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  BwdFirst F;
  F.cf = beg + 64 * wv;
  F.ef = 0;
  F.f0 = make_float4(0.f, 0.f, 0.f, -1.f);
  F.f1 = F.f2 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (F.cf + lane < end) {
    const int jf = D.items[F.cf + lane];
    F.ef = D.tile_e[F.cf + lane];
    F.f0 = D.rec[3 * jf];
    F.f1 = D.rec[3 * jf + 1];
    F.f2 = D.rec[3 * jf + 2];
  }
  return F;
}

template <int W>
__device__ __forceinline__ void bwd_tile(const Dev& D, const int slot, const float* __restrict__ Gsrc, BwdLdsT<W>& B) {
  constexpr int kThreads = 64 * W, kRounds = kTile * kTile * kTile / kThreads;
  const int2 lt = D.slot_tile[slot];
  const LevelDev L = D.levels[lt.x];
  if (L.kind != kLevelGrid) return;   // sample tiles: k_sample_bwd
  const int tid = threadIdx.x;
  const int64_t beg = min((int64_t)D.tile_start[slot], D.pair_cap);
  const int64_t end = min((int64_t)D.tile_start[slot + 1], D.pair_cap);
  if (beg == end) {
    // no kernel reaches the tile (or, in a mini-batch, no batch point is in it)
    if (tid == 0) D.tile_pbwd[slot] = 0;
    return;
  }
  const int n = L.n, nt = L.nt;
  const int lane = tid & 63, wv = tid >> 6;
  const int tz = lt.y / (nt * nt), ty = (lt.y / nt) % nt, tx = lt.y % nt;
  const float* __restrict__ G = Gsrc + L.pt_base;

  // thread p = tid + kThreads h holds point (x, y, z) = (p & 7, (p >> 3) & 7, p >> 6)
  // of the tile: eight consecutive lanes hold one row
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  const int rl = lane & ~7;                       // first lane of this lane's row
  const float xref = L.axis[tx * kTile];         // x' = x - xref
  const BwdFirst F = bwd_first_group(D, beg, end);
  bool row_used[kRounds];
  int row_cnt[kRounds], row_pos[kRounds];
#pragma unroll
  for (int h = 0; h < kRounds; ++h) {
    const int p = tid + kThreads * h;
    const int xi = tx * kTile + (p & 7), yi = ty * kTile + ((p >> 3) & 7), zi = tz * kTile + (p >> 6);
    float g = 0.f;
    if (xi < n && yi < n && zi < n) g = G[((int64_t)zi * n + yi) * n + xi];
    const bool nz = g != 0.f;
    const unsigned long long bal = __ballot(nz);
    const unsigned row_bits = (unsigned)(bal >> rl) & 0xffu;
    const int r = p >> 3;
    if (nz) {
      const float px = L.axis[xi], xo = px - xref, gx = g * xo;
      B.spx[8 * r + __popc(row_bits & ((1u << (lane & 7)) - 1u))] = make_float4(px, g, gx, gx * xo);
    }
    const int c = __popc(row_bits);
    row_cnt[h] = c;
    row_used[h] = c > 0;
    if ((lane & 7) == 0 && (c & 1)) B.spx[8 * r + c] = make_float4(1e30f, 0.f, 0.f, 0.f);
    const unsigned long long rb = __ballot((lane & 7) == 0 && c > 0);
    row_pos[h] = __popcll(rb & lt_mask);
    if (lane == 0) B.swr[h][wv] = __popcll(rb);
  }
  __syncthreads();
  int tot = 0;
  int base_h[kRounds];
#pragma unroll
  for (int h = 0; h < kRounds; ++h) {
    for (int v = 0; v < W; ++v) {
      if (v == wv) base_h[h] = tot;
      tot += B.swr[h][v];
    }
  }
#pragma unroll
  for (int h = 0; h < kRounds; ++h) {
    if ((lane & 7) == 0 && row_used[h]) {
      const int p = tid + kThreads * h;
      const int yi = ty * kTile + ((p >> 3) & 7), zi = tz * kTile + (p >> 6);
      B.srow[base_h[h] + row_pos[h]] =
          make_float4(L.axis[yi], L.axis[zi], __int_as_float(8 * (p >> 3)), __int_as_float((row_cnt[h] + 1) & ~1));
    }
  }
  // workgroup-uniform (all threads read the same LDS counts); readfirstlane
  // makes that visible, so the early exit below is a scalar branch
  const int R = __builtin_amdgcn_readfirstlane(tot);
  if (R == 0) {
    zero_partials(D, beg, end, tid, kThreads);
    if (tid == 0) D.tile_pbwd[slot] = 0;
    return;
  }
  __syncthreads();
  bwd_walk<W>(D, slot, B, R, xref, end, F.cf, F.ef, F.f0, F.f1, F.f2);
}

// Staging from the forward's registers (the fused step kernel): thread
// (wave w, lane l) holds the points x = 2 (l & 3) + {0, 1}, y = 4 (w & 1) +
// ((l >> 2) & 3), z = 4 (w >> 1) + (l >> 4) of the tile, so the four lanes of
// a quad hold one row (y, z).  Rows are numbered r = 8 z + y and placed in
// ascending r, points in ascending x, exactly as bwd_tile places them.
__device__ void bwd_stage_from_registers(const Dev& D, const LevelDev& L, int slot, int tx, int ty, int tz,
                                         const float g[2], BwdLds& B, int64_t beg, int64_t end) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (beg == end) {
    if (tid == 0) D.tile_pbwd[slot] = 0;
    return;
  }
  const int n = L.n;
  const float xref = L.axis[tx * kTile];
  const BwdFirst F = bwd_first_group(D, beg, end);
  const int q = lane & 3, qb = lane & ~3;
  const int yl = 4 * (wv & 1) + ((lane >> 2) & 3), zl = 4 * (wv >> 1) + (lane >> 4);
  const int r = 8 * zl + yl;
  const bool nz0 = g[0] != 0.f, nz1 = g[1] != 0.f;
  const unsigned long long b0 = __ballot(nz0), b1 = __ballot(nz1);
  const unsigned long long below = ((1ull << q) - 1ull) << qb, quad = 0xfull << qb;
  const int pos0 = __popcll(b0 & below) + __popcll(b1 & below);
  const int c = __popcll(b0 & quad) + __popcll(b1 & quad);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h ? nz1 : nz0) {
      const int xi = tx * kTile + 2 * q + h;
      const float px = L.axis[min(xi, n - 1)], xo = px - xref, gx = g[h] * xo;
      B.spx[8 * r + pos0 + (h ? (nz0 ? 1 : 0) : 0)] = make_float4(px, g[h], gx, gx * xo);
    }
  }
  if (q == 0 && (c & 1)) B.spx[8 * r + c] = make_float4(1e30f, 0.f, 0.f, 0.f);
  // this wave's 16 rows in use (quad i of the wave is row bit i)
  const unsigned long long lead = __ballot(q == 0 && c > 0);
  if (lane == 0) {
    uint32_t m = 0;
    for (int i = 0; i < 16; ++i) m |= (uint32_t)((lead >> (4 * i)) & 1ull) << i;
    B.wrows[wv] = m;
  }
  __syncthreads();
  // the 64-bit mask of rows in use, bit r = 8 z + y
  unsigned long long used = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t m = B.wrows[w];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int rr = 8 * (4 * (w >> 1) + (i >> 2)) + 4 * (w & 1) + (i & 3);
      used |= (unsigned long long)((m >> i) & 1u) << rr;
    }
  }
  if (q == 0 && c > 0) {
    const int yi = ty * kTile + yl, zi = tz * kTile + zl;
    B.srow[__popcll(used & ((1ull << r) - 1ull))] =
        make_float4(L.axis[min(yi, n - 1)], L.axis[min(zi, n - 1)], __int_as_float(8 * r), __int_as_float((c + 1) & ~1));
  }
  const int R = __builtin_amdgcn_readfirstlane(__popcll(used));
  if (R == 0) {
    zero_partials(D, beg, end, tid, kBwdThreads);
    if (tid == 0) D.tile_pbwd[slot] = 0;
    return;
  }
  __syncthreads();
  bwd_walk<4>(D, slot, B, R, xref, end, F.cf, F.ef, F.f0, F.f1, F.f2);
}

template <int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(8))) void k_bwd_tiles(
    Dev D, const float* __restrict__ Gsrc, int n_slots) {
  __shared__ BwdLdsT<W> B;
  const int slot = ordered_slot(D, tile_slot(blockIdx.x, n_slots, D.slot_chunk));
  if (slot < 0) return;
  bwd_tile<W>(D, slot, Gsrc, B);
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_bwd_tiles_persistent(Dev D, const float* __restrict__ Gsrc,
                                                                  int n_slots) {
  __shared__ BwdLdsT<W> B;
  for (int pos = blockIdx.x; pos < n_slots; pos += gridDim.x) {
    bwd_tile<W>(D, ordered_slot(D, pos), Gsrc, B);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// backward, stage 2: sixteen lanes per kernel slot.  Sums the kernel's
// per-tile moments in a fixed order (lane-strided, then a fixed butterfly)
// in float64 and turns them into gradients (Appendix A; quaternion or Euler
// chain rule).
// ---------------------------------------------------------------------------

// Rotation about axis k (0 = x, 1 = y, 2 = z) by angle t and its derivative
// in t (the standard right-handed matrices).
__device__ __forceinline__ void axis_rotation(int k, double t, double M[3][3], double dM[3][3]) {
  const double c = cos(t), s = sin(t);
  const int i = k == 0 ? 1 : (k == 1 ? 2 : 0), jj = k == 0 ? 2 : (k == 1 ? 0 : 1);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      M[a][b] = 0.0;
      dM[a][b] = 0.0;
    }
  M[k][k] = 1.0;
  M[i][i] = c; M[jj][jj] = c; M[i][jj] = -s; M[jj][i] = s;
  dM[i][i] = -s; dM[jj][jj] = -s; dM[i][jj] = -c; dM[jj][i] = c;
}

__device__ __forceinline__ void mat3_mul(const double A[3][3], const double B[3][3], double Cm[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Cm[a][b] = A[a][0] * B[0][b] + A[a][1] * B[1][b] + A[a][2] * B[2][b];
}

__device__ __forceinline__ double mat3_dot(const double A[3][3], const double B[3][3]) {
  double r = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) r += A[a][b] * B[a][b];
  return r;
}

// A kernel's gradients from its ten summed moments (Appendix A; the
// quaternion or Euler chain rule), written to its slot of grad.
__device__ void reduce_epilogue(const Dev& D, const float* __restrict__ p, float* __restrict__ grad, const int j,
                                const double v[10]) {
  const int C = D.cap_total;
  const double w = p[j];
  const double s[3] = {p[4 * C + j], p[5 * C + j], p[6 * C + j]};
  const double q4[4] = {p[7 * C + j], p[8 * C + j], p[9 * C + j], p[10 * C + j]};
  const bool euler = D.orientation == ERBF_ORIENT_EULER;
  double qn = 1.0;
  double qh[4] = {1.0, 0.0, 0.0, 0.0};
  double R[3][3], Rx[3][3], Ry[3][3], Rz[3][3], dRx[3][3], dRy[3][3], dRz[3][3];
  if (euler) {
    axis_rotation(0, q4[0], Rx, dRx);
    axis_rotation(1, q4[1], Ry, dRy);
    axis_rotation(2, q4[2], Rz, dRz);
    double RyRx[3][3];
    mat3_mul(Ry, Rx, RyRx);
    mat3_mul(Rz, RyRx, R);
  } else {
    qn = sqrt(q4[0] * q4[0] + q4[1] * q4[1] + q4[2] * q4[2] + q4[3] * q4[3]);
    if (qn > 0.0) {
      for (int k = 0; k < 4; ++k) qh[k] = q4[k] / qn;
    } else {
      qn = 1.0;
    }
    const double qw = qh[0], qx = qh[1], qy = qh[2], qz = qh[3];
    R[0][0] = 1 - 2 * (qy * qy + qz * qz); R[0][1] = 2 * (qx * qy - qw * qz); R[0][2] = 2 * (qx * qz + qw * qy);
    R[1][0] = 2 * (qx * qy + qw * qz); R[1][1] = 1 - 2 * (qx * qx + qz * qz); R[1][2] = 2 * (qy * qz - qw * qx);
    R[2][0] = 2 * (qx * qz - qw * qy); R[2][1] = 2 * (qy * qz + qw * qx); R[2][2] = 1 - 2 * (qx * qx + qy * qy);
  }
  double d2[3];
  for (int k = 0; k < 3; ++k) d2[k] = exp(2.0 * s[k]);
  const double amp = D.weight_map == ERBF_WEIGHT_SIGNED_SQUARE ? w * fabs(w) : w;
  const double dadw = D.weight_map == ERBF_WEIGHT_SIGNED_SQUARE ? 2.0 * fabs(w) : 1.0;
  const double T1[3] = {v[1], v[2], v[3]};
  const double T2[3][3] = {{v[4], v[5], v[6]}, {v[5], v[7], v[8]}, {v[6], v[8], v[9]}};
  // dL/dw
  const double gw = v[0] * dadw;
  // dL/dc = 2 a A T1, A = R^T D^2 R
  double u1[3];
  for (int k = 0; k < 3; ++k) u1[k] = d2[k] * (R[k][0] * T1[0] + R[k][1] * T1[1] + R[k][2] * T1[2]);
  double gc[3];
  for (int l = 0; l < 3; ++l) gc[l] = 2.0 * amp * (R[0][l] * u1[0] + R[1][l] * u1[1] + R[2][l] * u1[2]);
  // RT2 = R T2
  double RT2[3][3];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) RT2[k][l] = R[k][0] * T2[0][l] + R[k][1] * T2[1][l] + R[k][2] * T2[2][l];
  // dL/ds_k = -2 a d_k^2 r_k^T T2 r_k
  double gs[3];
  for (int k = 0; k < 3; ++k)
    gs[k] = -2.0 * amp * d2[k] * (RT2[k][0] * R[k][0] + RT2[k][1] * R[k][1] + RT2[k][2] * R[k][2]);
  // dL/dR = -2 a D^2 R T2
  double gR[3][3];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) gR[k][l] = -2.0 * amp * d2[k] * RT2[k][l];
  grad[j] = (float)gw;
  for (int l = 0; l < 3; ++l) grad[(1 + l) * C + j] = (float)gc[l];
  for (int k = 0; k < 3; ++k) grad[(4 + k) * C + j] = (float)gs[k];
  if (euler) {
    // dL/dtheta_k = <dL/dR, dR/dtheta_k>: Rz Ry dRx, Rz dRy Rx, dRz Ry Rx
    double T[3][3], U[3][3], dR[3][3];
    mat3_mul(Ry, dRx, T);
    mat3_mul(Rz, T, dR);
    grad[7 * C + j] = (float)mat3_dot(gR, dR);
    mat3_mul(dRy, Rx, T);
    mat3_mul(Rz, T, dR);
    grad[8 * C + j] = (float)mat3_dot(gR, dR);
    mat3_mul(Ry, Rx, U);
    mat3_mul(dRz, U, dR);
    grad[9 * C + j] = (float)mat3_dot(gR, dR);
    grad[10 * C + j] = 0.f;
    return;
  }
  // dL/dqhat through dR/dqhat, then the projection through q / |q|
  const double qw = qh[0], qx = qh[1], qy = qh[2], qz = qh[3];
  double gq[4];
  gq[0] = 2 * (-qz * gR[0][1] + qy * gR[0][2] + qz * gR[1][0] - qx * gR[1][2] - qy * gR[2][0] + qx * gR[2][1]);
  gq[1] = 2 * (qy * gR[0][1] + qz * gR[0][2] + qy * gR[1][0] - 2 * qx * gR[1][1] - qw * gR[1][2] + qz * gR[2][0] +
               qw * gR[2][1] - 2 * qx * gR[2][2]);
  gq[2] = 2 * (-2 * qy * gR[0][0] + qx * gR[0][1] + qw * gR[0][2] + qx * gR[1][0] + qz * gR[1][2] - qw * gR[2][0] +
               qz * gR[2][1] - 2 * qy * gR[2][2]);
  gq[3] = 2 * (-2 * qz * gR[0][0] - qw * gR[0][1] + qx * gR[0][2] + qw * gR[1][0] - 2 * qz * gR[1][1] +
               qy * gR[1][2] + qx * gR[2][0] + qy * gR[2][1]);
  const double dot = qh[0] * gq[0] + qh[1] * gq[1] + qh[2] * gq[2] + qh[3] * gq[3];
  for (int k = 0; k < 4; ++k) grad[(7 + k) * C + j] = (float)((gq[k] - qh[k] * dot) / qn);
}

// Sixteen lanes per kernel, four kernels per wave, sixteen per block: a
// lane group sums its kernel's partials (contiguous, entries strided by 16)
// in float64, folds them over the group in a fixed order, and the group's
// first lane forms the gradients.
__global__ __launch_bounds__(256) void k_bwd_reduce(Dev D, const float* __restrict__ p,
                                                    float* __restrict__ grad) {
  const int lane = threadIdx.x & 63, sl = lane & 15;
  const int j = blockIdx.x * 16 + (threadIdx.x >> 6) * 4 + (lane >> 4);
  const int C = D.cap_total;
  if (j >= C) return;   // the whole lane group leaves together
  const float4 r0 = D.rec[3 * j];
  if (r0.w < 0.f) {
    if (sl < 11) grad[sl * C + j] = 0.f;
    return;
  }
  double v[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) v[i] = 0.0;
  const int64_t base = D.kstart[j];
  const int c = D.kcnt[j];
  // every entry's moments are written each step (zero for tiles without a
  // non-zero G, and for the filler entries of the emit pass)
  const int cc = (int)min((int64_t)c, max((int64_t)0, D.pair_cap - base));
  for (int e = sl; e < cc; e += 16) {
    const float2* q = D.partials + 5 * (base + e);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const float2 a = q[i];
      v[2 * i] += a.x;
      v[2 * i + 1] += a.y;
    }
  }
#pragma unroll
  for (int i = 0; i < 10; ++i) {
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o, 16);
  }
  if (sl != 0) return;
  reduce_epilogue(D, p, grad, j, v);
}

// ---------------------------------------------------------------------------
// Step statistics and the loss weights of eq. 3-21.  Per shape: kStatParts
// blocks each sum a fixed slice of the shape's tiles and kernels; one wave
// then sums the slices in a fixed order, decides alpha and beta and writes
// the statistics; a grid-wide pass applies the weights to the gradient.
// ---------------------------------------------------------------------------

// MODE 0: forward statistics; 1: backward pair count only; 2: both, plus
// the sums of eq. 3-21 and L1 over the weights.
// BATCH: the forward part comes from the mini-batch records (n_pts of them)
// instead of the tile statistics.
template <int MODE, bool BATCH>
__device__ __forceinline__ void stats_part_body(const Dev& D, const float* __restrict__ p,
                                                const int32_t* __restrict__ m_dev, const float* __restrict__ grad,
                                                int n_pts) {
  __shared__ double shd[4][7];
  __shared__ float shf[4];
  const int part = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const ShapeDev S = D.shapes[b];
  const int m = min(max(m_dev[b], 0), S.cap);
  double l2 = 0.0, nid = 0.0, pf = 0.0, pb = 0.0, l1 = 0.0, num = 0.0, den = 0.0;
  float mx = 0.f;
  // this block's slice of the shape's tiles (levels in order)
  int tot = 0;
  for (int li = 0; li < S.n_active; ++li) tot += D.levels[S.lvl0 + li].n_slots;
  const int per = (tot + kStatParts - 1) / kStatParts;
  const int lo = part * per, hi = min(tot, lo + per);
  int acc = 0;
  for (int li = 0; li < S.n_active; ++li) {
    const LevelDev L = D.levels[S.lvl0 + li];
    const int a0 = max(lo, acc), a1 = min(hi, acc + L.n_slots);
    for (int x = a0 + tid; x < a1; x += 256) {
      const int sl = L.slot0 + (x - acc);
      if (MODE != 1 && !BATCH) {
        const TileStat ts = D.tstat[sl];
        l2 += ts.l2;
        nid += (double)ts.n_idall;
        mx = fmaxf(mx, ts.max_abs_e);
        pf += (double)ts.p_fwd;
      }
      if (MODE >= 1) pb += (double)D.tile_pbwd[sl];
    }
    acc += L.n_slots;
  }
  if (BATCH) {
    // this block's slice of the batch, the shape's points only
    const int bper = (n_pts + kStatParts - 1) / kStatParts;
    const int b0 = part * bper, b1 = min(n_pts, b0 + bper);
    for (int k = b0 + tid; k < b1; k += 256) {
      if (D.b_shape[k] != b) continue;
      l2 += D.b_l2[k];
      nid += (double)D.b_id[k];
      mx = fmaxf(mx, D.b_abs[k]);
      pf += (double)D.b_pf[k];
    }
  }
  if (MODE == 2) {
    const int kper = (m + kStatParts - 1) / kStatParts;
    const int k0 = part * kper, k1 = min(m, k0 + kper);
    for (int k = k0 + tid; k < k1; k += 256) {
      const float w = p[S.kbase + k];
      const double g1 = w > 0.f ? 1.0 : (w < 0.f ? -1.0 : 0.0);
      const double g2 = grad[S.kbase + k];
      l1 += fabs((double)w);
      num += (g1 - g2) * g1;
      den += (g2 - g1) * (g2 - g1);
    }
  }
  // wave sums, then the four waves' sums in a fixed order, all behind one
  // barrier
  double v[7] = {l2, nid, pf, pb, l1, num, den};
#pragma unroll
  for (int i = 0; i < 7; ++i) v[i] = wave_sum(v[i]);
  mx = wave_max_f(mx);
  const int lane = tid & 63, wv = tid >> 6;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 7; ++i) shd[wv][i] = v[i];
    shf[wv] = mx;
  }
  __syncthreads();
  if (tid == 0) {
    double r[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) r[i] = (shd[0][i] + shd[1][i]) + (shd[2][i] + shd[3][i]);
    StatPart sp;
    sp.l2 = r[0];
    sp.nid = r[1];
    sp.pf = r[2];
    sp.pb = r[3];
    sp.l1 = r[4];
    sp.num = r[5];
    sp.den = r[6];
    sp.mx = fmaxf(fmaxf(shf[0], shf[1]), fmaxf(shf[2], shf[3]));
    sp.pad = 0;
    D.stat_part[b * kStatParts + part] = sp;
  }
}

template <int MODE, bool BATCH>
__global__ __launch_bounds__(256) void k_stats_part(Dev D, const float* __restrict__ p,
                                                    const int32_t* __restrict__ m_dev,
                                                    const float* __restrict__ grad, int n_pts) {
  stats_part_body<MODE, BATCH>(D, p, m_dev, grad, n_pts);
}

// One wave: the shape's slices in a fixed order, the weights of eq. 3-21 and
// the statistics.
template <int MODE>
__device__ __forceinline__ void stats_final_wave(const Dev& D, const int b, const int lane,
                                                 const int32_t* __restrict__ m_dev, erbf_stats* __restrict__ out,
                                                 const StatsArgs& a) {
  const ShapeDev S = D.shapes[b];
  const int m = min(max(m_dev[b], 0), S.cap);
  StatPart sp = {};
  if (lane < kStatParts) sp = D.stat_part[b * kStatParts + lane];
  const double l2 = wave_sum(sp.l2), nid = wave_sum(sp.nid), pf = wave_sum(sp.pf), pb = wave_sum(sp.pb);
  const double l1 = wave_sum(sp.l1), num = wave_sum(sp.num), den = wave_sum(sp.den);
  const float mx = wave_max_f(sp.mx);
  if (lane != 0) return;
  double alpha = 1.0, beta = 0.0;
  if (MODE == 2) {
    if (a.mode == ERBF_MODE_FIXED) {
      beta = a.lambda_dev ? (double)a.lambda_dev[b] : (double)a.lambda;
    } else if (a.mode == ERBF_MODE_DYNAMIC && (a.l1_active_dev ? a.l1_active_dev[b] : a.l1_active) &&
               mx < a.tau_m) {
      alpha = den > 0.0 ? fmin(fmax(num / den, 0.0), 1.0) : 1.0;
      beta = 1.0 - alpha;
    }
  }
  D.stat_ab[b] = make_double2(alpha, beta);
  // the step's Adam pass follows (erbf_train_step); a held step counts nothing
  if (a.step_inc && !(a.hold && *a.hold != 0)) a.step_inc[b] += 1;
  if (out) {
    const int64_t nb = D.counters[0];
    erbf_stats st;
    st.L2 = l2;
    st.L1 = MODE == 2 ? l1 : 0.0;
    st.loss = alpha * l2 + beta * st.L1;
    st.alpha = alpha;
    st.beta = beta;
    st.n_idall = (int64_t)nid;
    st.P_fwd = (int64_t)pf;
    st.P_bwd = (int64_t)pb;
    st.n_bucket_pairs = nb;
    st.max_abs_E = mx;
    st.m = m;
    st.flags = nb > D.pair_cap ? ERBF_FLAG_BUCKET_OVERFLOW : 0;
    st.reserved = 0;
    st.P_fwd_total = out[b].P_fwd_total + st.P_fwd;
    st.P_bwd_total = out[b].P_bwd_total + st.P_bwd;
    st.calls = out[b].calls + 1;
    out[b] = st;
  }
}

template <int MODE>
__global__ __launch_bounds__(64) void k_stats_final(Dev D, const int32_t* __restrict__ m_dev,
                                                    erbf_stats* __restrict__ out, StatsArgs a) {
  stats_final_wave<MODE>(D, blockIdx.x, threadIdx.x, m_dev, out, a);
}

// The slices and the final in one launch: every block writes its slice,
// then takes a ticket; the block holding the shape's last ticket has seen
// every slice written (each block fences its slice before its ticket) and
// forms the statistics and the weights in the same fixed order as
// k_stats_final, then resets the ticket for the next call.
template <int MODE, bool BATCH>
__global__ __launch_bounds__(256) void k_stats_fused(Dev D, const float* __restrict__ p,
                                                     const int32_t* __restrict__ m_dev,
                                                     const float* __restrict__ grad, int n_pts,
                                                     erbf_stats* __restrict__ out, StatsArgs a) {
  __shared__ int last;
  stats_part_body<MODE, BATCH>(D, p, m_dev, grad, n_pts);
  const int b = blockIdx.y;
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned t = atomicAdd(&D.tickets[b], 1u);
    last = t == (unsigned)(kStatParts - 1);
    if (last) __threadfence();
  }
  __syncthreads();
  if (!last) return;
  if (threadIdx.x < 64) stats_final_wave<MODE>(D, b, threadIdx.x, m_dev, out, a);
  if (threadIdx.x == 0) D.tickets[b] = 0u;
}

// combine: alpha * dL2 + beta * sign(w) on w; alpha * dL2 on the rest
__global__ __launch_bounds__(256) void k_stats_apply(Dev D, const float* __restrict__ p,
                                                     const int32_t* __restrict__ m_dev, float* __restrict__ grad) {
  const int jj = blockIdx.x * 256 + threadIdx.x;
  if (jj >= D.cap_total) return;
  const int b = D.kshape[jj];
  const ShapeDev S = D.shapes[b];
  const int m = min(max(m_dev[b], 0), S.cap);
  if (jj - S.kbase >= m) return;
  const double2 ab = D.stat_ab[b];
  const int C = D.cap_total;
  const float w = p[jj];
  const double sg = w > 0.f ? 1.0 : (w < 0.f ? -1.0 : 0.0);
  grad[jj] = (float)(ab.x * (double)grad[jj] + ab.y * sg);
  if (ab.x != 1.0) {
    for (int seg = 1; seg < 11; ++seg) grad[seg * C + jj] = (float)(ab.x * (double)grad[seg * C + jj]);
  }
}

// ---------------------------------------------------------------------------
// Adam
// ---------------------------------------------------------------------------

__global__ void k_step_inc(int32_t* step, int n, const int32_t* hold) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(hold && *hold != 0)) step[i] += 1;
}

// Bias-corrected Adam over the packed parameters, at step t = step[b] of
// each shape (already incremented for this step).  COMBINE: the gradient is
// the L2 gradient as the backward left it, combined here with the step's loss
// weights (alpha dL2 + beta sign(w) on w, alpha dL2 elsewhere, eq. 3-21) and
// written back, so the loss call needs no pass of its own for it.  While
// the hold word is non-zero the pass changes nothing.
template <bool COMBINE>
__global__ __launch_bounds__(256) void k_adam(Dev D, float* __restrict__ p, const int32_t* __restrict__ m_dev,
                                              float* __restrict__ g, float* __restrict__ m1, float* __restrict__ m2,
                                              const int32_t* __restrict__ step, AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int C = D.cap_total;
  if (i >= (int64_t)11 * C) return;
  if (a.hold && *a.hold != 0) return;
  const int j = (int)(i % C);
  const int b = D.kshape[j];
  const ShapeDev S = D.shapes[b];
  if (j - S.kbase >= min(max(m_dev[b], 0), S.cap)) return;
  const float lr = a.lr_dev ? a.lr_dev[b] : a.lr;
  const int t = step[b];
  float gi = g[i];
  if (COMBINE) {
    const double2 ab = D.stat_ab[b];
    if (i < C) {
      const float w = p[i];
      const double sg = w > 0.f ? 1.0 : (w < 0.f ? -1.0 : 0.0);
      gi = (float)(ab.x * (double)gi + ab.y * sg);
      g[i] = gi;
    } else if (ab.x != 1.0) {
      gi = (float)(ab.x * (double)gi);
      g[i] = gi;
    }
  }
  const float mm = a.beta1 * m1[i] + (1.f - a.beta1) * gi;
  const float vv = a.beta2 * m2[i] + (1.f - a.beta2) * gi * gi;
  m1[i] = mm;
  m2[i] = vv;
  const float bc1 = 1.f - powf(a.beta1, (float)t);
  const float bc2 = 1.f - powf(a.beta2, (float)t);
  const float denom = sqrtf(vv) / sqrtf(bc2) + a.eps;
  p[i] -= (lr / bc1) * mm / denom;
}

// ---------------------------------------------------------------------------
// misc elementwise
// ---------------------------------------------------------------------------

// G[idx] = src[idx] * active(idx) over every point of the active levels.
__global__ __launch_bounds__(256) void k_mask_copy(Dev D, int li, const float* __restrict__ src) {
  const LevelDev L = D.levels[li];
  const int64_t npts = L.npts;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npts;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx = L.pt_base + k;
    const bool act = L.kind == kLevelSamples ? k < (int64_t)L.n_samples : point_active(L.bits, k);
    D.G[idx] = act ? src[idx] : 0.f;
  }
}

__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ x, int64_t n, float v) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    x[k] = v;
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* __restrict__ x, int64_t n, int32_t v) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    x[k] = v;
}

// eq. 3-10 in double, rounded once
__global__ __launch_bounds__(256) void k_targets(const float* __restrict__ S, int64_t n, float m,
                                                 float* __restrict__ t) {
  const double md = m;
  const double h = 0.69314718055994530942 / (md * md);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)S[k] - md;
    t[k] = (float)(2.0 * exp(-h * d * d));
  }
}

__global__ __launch_bounds__(256) void k_band_bits(const float* __restrict__ S, int64_t n, float band,
                                                   uint32_t* __restrict__ bits) {
  const int64_t nw = (n + 31) >> 5;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (int64_t)gridDim.x * blockDim.x) {
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) {
      const int64_t k = w * 32 + b;
      if (k < n && fabsf(S[k]) < band) v |= 1u << b;
    }
    bits[w] = v;
  }
}

// octree layer below a level of np points per axis: child point (i, j, k)
// of the 2np level is kept iff its parent cell (i/2, j/2, k/2) is present
// (parent bit, or every cell when pbits is null) and |S(parent)| <= thr
__global__ __launch_bounds__(256) void k_octree_bits(const float* __restrict__ Sp, const uint32_t* __restrict__ pbits,
                                                     int np, double thr, uint32_t* __restrict__ bits) {
  const int nc = 2 * np;
  const int64_t n = (int64_t)nc * nc * nc;
  const int64_t nw = (n + 31) >> 5;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (int64_t)gridDim.x * blockDim.x) {
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) {
      const int64_t g = w * 32 + b;
      if (g >= n) break;
      const int i = (int)(g % nc), j = (int)((g / nc) % nc), k = (int)(g / ((int64_t)nc * nc));
      const int64_t pg = ((int64_t)(k >> 1) * np + (j >> 1)) * np + (i >> 1);
      const bool present = !pbits || ((pbits[pg >> 5] >> (pg & 31)) & 1u);
      if (present && (double)fabsf(Sp[pg]) <= thr) v |= 1u << b;
    }
    bits[w] = v;
  }
}

// order-preserving float -> int key
__device__ __forceinline__ int fkey(float f) {
  const int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float fkey_inv(int k) {
  return __int_as_float(k >= 0 ? k : k ^ 0x7fffffff);
}

__global__ __launch_bounds__(256) void k_sdf_min(const float* __restrict__ S, int64_t n, int* __restrict__ key) {
  int best = INT32_MAX;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    best = min(best, fkey(S[k]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMin(key, best);
}

__global__ void k_sdf_min_init(int* key, const float* prev, int accumulate) {
  *key = accumulate ? fkey(*prev) : INT32_MAX;
}

__global__ void k_sdf_min_fin(const int* key, float* out) { *out = fkey_inv(*key); }

// ---------------------------------------------------------------------------
// refine: tile occupancy of a new level
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_tile_flags(Dev D, int li, int32_t* __restrict__ flags) {
  const LevelDev L = D.levels[li];
  const int nt = L.nt, n = L.n;
  const int ntt = nt * nt * nt;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntt) return;
  const int tz = t / (nt * nt), ty = (t / nt) % nt, tx = t % nt;
  int any = 0;
  if (L.bits == nullptr) {
    any = 1;
  } else {
    for (int z = tz * kTile; z < min(tz * kTile + kTile, n) && !any; ++z)
      for (int y = ty * kTile; y < min(ty * kTile + kTile, n) && !any; ++y) {
        const int64_t row = ((int64_t)z * n + y) * n;
        const int x0 = tx * kTile, x1 = min(tx * kTile + kTile, n) - 1;
        any = popcount_range(L.bits, row + x0, row + x1) > 0;
      }
  }
  flags[t] = any;
}

__global__ __launch_bounds__(256) void k_tile_assign(Dev D, int li, const int32_t* __restrict__ flags,
                                                     const int32_t* __restrict__ excl, int slot0) {
  const LevelDev L = D.levels[li];
  const int ntt = L.nt * L.nt * L.nt;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntt) return;
  if (flags[t]) {
    const int s = slot0 + excl[t];
    D.tile_map[L.tmap0 + t] = s;
    D.slot_tile[s] = make_int2(li, t);
  } else {
    D.tile_map[L.tmap0 + t] = -1;
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
static inline unsigned gridstride(int64_t n) { return (unsigned)std::min<int64_t>(nblk(n, 256), 4096); }

template <typename T>
hipError_t launch_scan_t(const int32_t* in, int n, T* blocks, T* out, int64_t* total, hipStream_t s) {
  const int nb = (int)nblk(n + 1, 1024);
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(1024), 0, s, in, n, blocks);
  hipLaunchKernelGGL(k_scan_blocks<T>, dim3(1), dim3(1024), 0, s, blocks, nb, total);
  hipLaunchKernelGGL(k_scan_down<T>, dim3(nb), dim3(1024), 0, s, in, n, blocks, out);
  return hipGetLastError();
}

hipError_t launch_scan(const int32_t* in, int n, int32_t* blocks, int32_t* out, int64_t* total,
                       hipStream_t s) {
  return launch_scan_t<int32_t>(in, n, blocks, out, total, s);
}

template <typename T>
hipError_t launch_scan_any(const int32_t* in, int n, T* blocks, T* out, int64_t* total, hipStream_t s) {
  if (n <= 1024 * 4)
    hipLaunchKernelGGL((k_scan_single<4, T>), dim3(1), dim3(1024), 0, s, in, n, out, total);
  else if (n <= 1024 * 16)
    hipLaunchKernelGGL((k_scan_single<16, T>), dim3(1), dim3(1024), 0, s, in, n, out, total);
  else
    return launch_scan_t<T>(in, n, blocks, out, total, s);
  return hipGetLastError();
}

// the launch order of the tile kernels (when switched on), after tile_start
// and the class counts (counted = false: count them here)
static void launch_tile_order(const Dev& D, int n_slots, bool counted, hipStream_t s) {
  if (!D.tile_order_on || n_slots <= 0) return;
  const int nb = (int)nblk(n_slots, 256);
  if (!counted) hipLaunchKernelGGL(k_order_count, dim3(nb), dim3(256), 0, s, D, n_slots);
  hipLaunchKernelGGL(k_order_place, dim3(nb), dim3(256), 0, s, D, n_slots, nb);
}

hipError_t launch_buckets(const Dev& D, const float* p, const int32_t* m_dev, int n_slots, hipStream_t s) {
  const int nkb = (int)nblk(D.cap_total, 4);   // count/emit blocks, four kernels each
  // the count pass also forms every kernel's record, which the forward and
  // backward read even when no tile is active
  hipLaunchKernelGGL(k_bucket_count, dim3(nkb), dim3(256), 0, s, D, p, m_dev);
  if (n_slots <= 0) return hipGetLastError();
  {
    // 64-bit offsets: the entry total may pass 2^31 (then it exceeds the
    // list capacity, no entry past it is written, and the overflow flag is
    // raised from counters[0])
    const hipError_t e = launch_scan_any<int64_t>(D.kblock, nkb, reinterpret_cast<int64_t*>(D.scan_blocks),
                                                  D.kblock_ex, D.counters, s);
    if (e != hipSuccess) return e;
  }
  if (D.bucket_rank) {
    // tile starts from the per-tile counts, entries placed in their tiles,
    // then ordered within each tile
    hipError_t e = launch_scan_any<int64_t>(D.tile_cnt, n_slots, reinterpret_cast<int64_t*>(D.scan_blocks),
                                            D.tile_start64, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bucket_emit, dim3(nkb), dim3(256), 0, s, D);
    const size_t lds = sizeof(uint32_t) * 4 * 2 * (size_t)D.rank_words;
    hipLaunchKernelGGL(k_tile_rank, dim3(nblk(n_slots, 4)), dim3(256), lds, s, D, n_slots);
    launch_tile_order(D, n_slots, false, s);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_bucket_emit, dim3(nkb), dim3(256), 0, s, D);
  // keys are slots (< n_slots) or the filler tiles_total: sort on just
  // enough bits, at most 8 per pass
  int bits = 0;
  while ((1ll << bits) <= (int64_t)D.tiles_total) ++bits;
  const int passes = (bits + 7) / 8;
  const int dbits = passes ? (bits + passes - 1) / passes : 0;
  // pass 0 reads the kernel-major entries (kept for the backward reduce);
  // the last pass writes the tile lists
  // packed keys: the slot sits in the upper 16 bits, the kernel rides along
  // in the lower 16
  const bool packed = D.packed_keys != 0;
  const int32_t* kin = D.kslot;
  const int32_t* vin = nullptr;     // identity: entry e holds value e
  const int32_t* jin = packed ? nullptr : D.kj;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = (packed ? 16 : 0) + pass * dbits, mask = (1 << dbits) - 1;
    const bool last = pass == passes - 1;
    int32_t* kout = last ? D.tile_keys : D.sort_keys[pass & 1];
    int32_t* vout = last ? D.tile_e : D.sort_vals[pass & 1];
    int32_t* jout = last ? D.items : (packed ? nullptr : D.sort_j[pass & 1]);
    hipLaunchKernelGGL(k_radix_hist, dim3(D.radix_nb), dim3(256), 0, s, D, kin, shift, mask);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(1024), 0, s, D);
    using Scatter = void (*)(Dev, const int32_t*, const int32_t*, const int32_t*, int32_t*, int32_t*, int32_t*, int,
                             int, int, int);
    const Scatter sc = pass == 0 ? (packed ? k_radix_scatter<true, true> : k_radix_scatter<true, false>)
                                 : (packed ? k_radix_scatter<false, true> : k_radix_scatter<false, false>);
    hipLaunchKernelGGL(sc, dim3(D.radix_nb), dim3(256), 0, s, D, kin, vin, jin, kout, vout, jout, shift, mask, dbits,
                       last ? 1 : 0);
    kin = kout;
    vin = vout;
    jin = jout;
  }
  hipLaunchKernelGGL(k_tile_starts, dim3(nblk(n_slots + 1, 256)), dim3(256), 0, s, D, D.tile_keys, n_slots);
  launch_tile_order(D, n_slots, true, s);
  return hipGetLastError();
}

// grid of a one-workgroup-per-tile launch (padded for the XCD runs)
static inline int tile_grid(const Dev& D, int n_slots) {
  if (D.slot_chunk <= 0) return n_slots;
  const int per = 8 * D.slot_chunk;
  return (n_slots + per - 1) / per * per;
}

// Launch with start/stop events taken at the kernel's own start and end when
// timing is requested, otherwise as an ordinary launch (graph-capturable).
template <typename... Args>
inline void launch_timed(void (*kernel)(Args...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

hipError_t launch_forward(const Dev& D, int n_slots, bool loss, float* f_out, float tau1, float tau2,
                          const hipEvent_t* ev, hipStream_t s, bool with_bwd) {
  if (n_slots > 0) {
    hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
    const bool pers = (D.variant & kVariantFwdPersistent) != 0;
    const int grid = pers ? std::min(n_slots, D.persistent_wgs) : tile_grid(D, n_slots);
    if (with_bwd) {
      if (pers)
        launch_timed(k_step_tiles_persistent, dim3(grid), dim3(256), s, e0, e1, D, f_out, tau1, tau2, n_slots);
      else
        launch_timed(k_step_tiles, dim3(grid), dim3(256), s, e0, e1, D, f_out, tau1, tau2, n_slots);
    } else {
      // the chunk of kernel records staged at a time (64, 128 or 256)
      using FwdKernel = void (*)(Dev, float*, float, float, int);
      const int ci = D.fwd_chunk == 64 ? 0 : (D.fwd_chunk == 128 ? 1 : 2);
      static const FwdKernel grid_k[2][3] = {{k_forward<false, 64>, k_forward<false, 128>, k_forward<false, 256>},
                                             {k_forward<true, 64>, k_forward<true, 128>, k_forward<true, 256>}};
      static const FwdKernel pers_k[2][3] = {
          {k_forward_persistent<false, 64>, k_forward_persistent<false, 128>, k_forward_persistent<false, 256>},
          {k_forward_persistent<true, 64>, k_forward_persistent<true, 128>, k_forward_persistent<true, 256>}};
      launch_timed((pers ? pers_k : grid_k)[loss ? 1 : 0][ci], dim3(grid), dim3(256), s, e0, e1, D, f_out, tau1,
                   tau2, n_slots);
    }
  }
  if (D.n_samp_slots > 0) {
    hipLaunchKernelGGL(k_sample_forward, dim3(D.n_samp_slots, D.samp_split), dim3(256), 0, s, D);
    if (loss)
      hipLaunchKernelGGL(k_sample_fwd_final<true>, dim3(D.n_samp_slots), dim3(256), 0, s, D, f_out, tau1, tau2);
    else
      hipLaunchKernelGGL(k_sample_fwd_final<false>, dim3(D.n_samp_slots), dim3(256), 0, s, D, f_out, tau1, tau2);
  }
  return hipGetLastError();
}

hipError_t launch_backward(const Dev& D, int n_slots, const float* p, const float* G, float* grad,
                           const hipEvent_t* ev, hipStream_t s, bool tiles_done, hipEvent_t fwd_stop,
                           uint8_t* shared) {
  uint8_t sh = 0;
  bool tiles_timed = false;   // the tile kernel was launched with ev[1] as its stop
  if (tiles_done) {
    // the grid tiles' moments came with the forward (the fused step kernel):
    // a zero-length interval for the backward-tile events
    if (ev && ev[0]) {
      const hipError_t e = hipEventRecord(ev[0], s);
      if (e != hipSuccess) return e;
    }
    if (ev && ev[1]) {
      const hipError_t e = hipEventRecord(ev[1], s);
      if (e != hipSuccess) return e;
    }
  } else if (n_slots > 0) {
    // W waves per tile workgroup (2, 4 or 8)
    using BwdKernel = void (*)(Dev, const float*, int);
    const int wi = D.bwd_waves == 2 ? 0 : (D.bwd_waves == 8 ? 2 : 1);
    static const BwdKernel grid_k[3] = {k_bwd_tiles<2>, k_bwd_tiles<4>, k_bwd_tiles<8>};
    static const BwdKernel pers_k[3] = {k_bwd_tiles_persistent<2>, k_bwd_tiles_persistent<4>,
                                        k_bwd_tiles_persistent<8>};
    const int threads = 64 * (wi == 0 ? 2 : (wi == 2 ? 8 : 4));
    // the tiles follow the forward directly unless sample-level forward
    // kernels ran in between
    hipEvent_t e0 = ev ? ev[0] : nullptr;
    if (ev && fwd_stop && D.n_samp_slots == 0) {
      e0 = nullptr;
      sh |= 1;
    }
    if (D.variant & kVariantBwdPersistent) {
      // the same number of resident waves whatever W
      const int grid = std::min(n_slots, D.persistent_wgs * 256 / threads);
      launch_timed(pers_k[wi], dim3(grid), dim3(threads), s, e0, ev ? ev[1] : nullptr, D, G, n_slots);
    } else {
      launch_timed(grid_k[wi], dim3(tile_grid(D, n_slots)), dim3(threads), s, e0, ev ? ev[1] : nullptr, D, G,
                   n_slots);
    }
    tiles_timed = ev != nullptr;
  } else if (ev && ev[0]) {
    // no tile at all: a zero-length interval
    hipError_t e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e != hipSuccess) return e;
  }
  if (D.n_samp_slots > 0) {
    hipLaunchKernelGGL(k_sample_bwd, dim3(D.n_samp_slots, D.samp_split), dim3(256), 0, s, D, G);
    hipLaunchKernelGGL(k_sample_bwd_sum, dim3(nblk(D.n_samp_slots, 64)), dim3(64), 0, s, D);
  }
  // the reduce follows the tiles directly unless sample-level kernels ran
  // in between
  hipEvent_t r0 = ev ? ev[2] : nullptr;
  if (tiles_timed && D.n_samp_slots == 0) {
    r0 = nullptr;
    sh |= 2;
  }
  launch_timed(k_bwd_reduce, dim3(nblk(D.cap_total, 16)), dim3(256), s, r0, ev ? ev[3] : nullptr, D, p, grad);
  if (shared) *shared = sh;
  return hipGetLastError();
}

hipError_t launch_stats(const Dev& D, int mode, const float* p, const int32_t* m_dev, float* grad,
                        erbf_stats* out, const StatsArgs& a, hipStream_t s, bool apply) {
  const dim3 parts(kStatParts, D.n_shapes);
  if (mode == 0) {
    hipLaunchKernelGGL((k_stats_fused<0, false>), parts, dim3(256), 0, s, D, p, m_dev, grad, 0, out, a);
  } else if (mode == 1) {
    hipLaunchKernelGGL((k_stats_fused<1, false>), parts, dim3(256), 0, s, D, p, m_dev, grad, 0, out, a);
  } else {
    hipLaunchKernelGGL((k_stats_fused<2, false>), parts, dim3(256), 0, s, D, p, m_dev, grad, 0, out, a);
    if (apply) hipLaunchKernelGGL(k_stats_apply, dim3(nblk(D.cap_total, 256)), dim3(256), 0, s, D, p, m_dev, grad);
  }
  return hipGetLastError();
}

hipError_t launch_batch_tiles(const Dev& D, int n_slots, const int64_t* pts, int n_pts, int32_t* sel, hipStream_t s) {
  hipError_t e = launch_fill_i32(sel, std::max(n_slots, 1), 0, s);
  if (e != hipSuccess) return e;
  if (n_pts > 0) hipLaunchKernelGGL(k_batch_tiles, dim3(nblk(n_pts, 256)), dim3(256), 0, s, D, pts, n_pts, sel);
  return hipGetLastError();
}

hipError_t launch_batch_step(const Dev& D, int n_slots, const int64_t* pts, int n_pts, const float* p,
                             const int32_t* m_dev, float* grad, float* f_out, erbf_stats* out, float tau1, float tau2,
                             const StatsArgs& a, hipStream_t s) {
  if (n_pts > 0)
    hipLaunchKernelGGL(k_batch_forward, dim3(nblk(n_pts, 4)), dim3(256), 0, s, D, pts, n_pts, f_out, tau1, tau2);
  hipError_t e = launch_backward(D, n_slots, p, D.G, grad, nullptr, s, false);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stats_fused<2, true>), dim3(kStatParts, D.n_shapes), dim3(256), 0, s, D, p, m_dev, grad,
                     n_pts, out, a);
  hipLaunchKernelGGL(k_stats_apply, dim3(nblk(D.cap_total, 256)), dim3(256), 0, s, D, p, m_dev, grad);
  return hipGetLastError();
}

hipError_t launch_adam(const Dev& D, float* p, const int32_t* m_dev, float* g, float* m1, float* m2,
                       int32_t* step, const AdamArgs& a, bool combine, hipStream_t s) {
  const dim3 grid(nblk((int64_t)11 * D.cap_total, 256));
  if (combine) {
    // the step counters were incremented by the loss call's statistics
    hipLaunchKernelGGL(k_adam<true>, grid, dim3(256), 0, s, D, p, m_dev, g, m1, m2, step, a);
  } else {
    hipLaunchKernelGGL(k_step_inc, dim3(nblk(D.n_shapes, 256)), dim3(256), 0, s, step, D.n_shapes, a.hold);
    hipLaunchKernelGGL(k_adam<false>, grid, dim3(256), 0, s, D, p, m_dev, g, m1, m2, step, a);
  }
  return hipGetLastError();
}

hipError_t launch_mask_copy(const Dev& D, int li, int64_t npts, const float* src, hipStream_t s) {
  hipLaunchKernelGGL(k_mask_copy, dim3(gridstride(npts)), dim3(256), 0, s, D, li, src);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* x, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(gridstride(n)), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(gridstride(n)), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

hipError_t launch_targets(const float* S, int64_t n, float m, float* t, hipStream_t s) {
  hipLaunchKernelGGL(k_targets, dim3(gridstride(n)), dim3(256), 0, s, S, n, m, t);
  return hipGetLastError();
}

hipError_t launch_band_bits(const float* S, int64_t n, float band, uint32_t* bits, hipStream_t s) {
  hipLaunchKernelGGL(k_band_bits, dim3(gridstride((n + 31) / 32)), dim3(256), 0, s, S, n, band, bits);
  return hipGetLastError();
}

hipError_t launch_octree_bits(const float* Sp, const uint32_t* pbits, int np, uint32_t* bits, hipStream_t s) {
  const int64_t nc = 2 * (int64_t)np;
  // half-diagonal of a parent cell (width 2/np), in double
  const double thr = std::sqrt(3.0) / (double)np;
  hipLaunchKernelGGL(k_octree_bits, dim3(gridstride((nc * nc * nc + 31) / 32)), dim3(256), 0, s, Sp, pbits, np, thr,
                     bits);
  return hipGetLastError();
}

hipError_t launch_sdf_min(const float* S, int64_t n, float* out, int accumulate, int* key_scratch,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_sdf_min_init, dim3(1), dim3(1), 0, s, key_scratch, out, accumulate);
  hipLaunchKernelGGL(k_sdf_min, dim3(gridstride(n)), dim3(256), 0, s, S, n, key_scratch);
  hipLaunchKernelGGL(k_sdf_min_fin, dim3(1), dim3(1), 0, s, key_scratch, out);
  return hipGetLastError();
}

hipError_t launch_tile_flags(const Dev& D, int li, int ntt, int32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_tile_flags, dim3(nblk(ntt, 256)), dim3(256), 0, s, D, li, flags);
  return hipGetLastError();
}

hipError_t launch_tile_assign(const Dev& D, int li, int ntt, const int32_t* flags, const int32_t* excl,
                              int slot0, hipStream_t s) {
  hipLaunchKernelGGL(k_tile_assign, dim3(nblk(ntt, 256)), dim3(256), 0, s, D, li, flags, excl, slot0);
  return hipGetLastError();
}

}  // namespace erbf
