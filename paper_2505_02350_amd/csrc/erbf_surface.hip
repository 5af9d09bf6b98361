// Surface evaluation of Section 4 (Evaluation Metric): the zero-level
// surface of a grid field by marching tetrahedra, points sampled uniformly by
// area on it, and the Hausdorff, Chamfer and normal cosine-similarity metrics
// between two sampled surfaces.
//
// Extraction: each cube of eight neighbouring grid points is split into six
// tetrahedra around its main diagonal (corner 0 to corner 7; corner c sits at
// offsets (c & 1, c >> 1 & 1, c >> 2)).  A tetrahedron whose corners straddle
// the iso value (inside: value < iso) gives one triangle (one corner apart)
// or two (two and two), with vertices interpolated linearly along the
// straddling edges.  A count pass and a scan give every cube its first
// triangle, so triangles come out in cube order (x fastest), then
// tetrahedron, then case order, on every run.
//
// Sampling: triangle areas in double, their running sum (a blocked scan in a
// fixed order), then per sample the first triangle
// whose running sum exceeds u0 times the total and the point
// (1 - sqrt(u1)) A + sqrt(u1) (1 - u2) B + sqrt(u1) u2 C, all in double; the
// uniforms are the caller's.
//
// Metrics: for every point of either set, the closest point of the other
// (brute force, the other set streamed through LDS, ties to the lower
// index), its distance and |n . n_closest|; one block then forms HD (the
// largest distance), CD (half the mean distance each way) and CS (half the
// mean |cos| each way) in a fixed order.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "erbf_device.h"
#include "erbf_internal.h"
#include "erbf_launch.h"

namespace erbf {

namespace {

__constant__ int kTet[6][4] = {{0, 1, 3, 7}, {0, 3, 2, 7}, {0, 2, 6, 7}, {0, 6, 4, 7}, {0, 4, 5, 7}, {0, 5, 1, 7}};

__device__ __forceinline__ int tet_tris(const float v[4], float iso) {
  int ins = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) ins += v[q] < iso ? 1 : 0;
  return (ins == 0 || ins == 4) ? 0 : (ins == 2 ? 2 : 1);
}

__device__ __forceinline__ void load_cube(const float* __restrict__ F, const float* __restrict__ ax, int n, int64_t c,
                                          float cv[8], float cp[8][3]) {
  const int m = n - 1;
  const int i = (int)(c % m), j = (int)((c / m) % m), k = (int)(c / ((int64_t)m * m));
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ii = i + (q & 1), jj = j + ((q >> 1) & 1), kk = k + (q >> 2);
    cv[q] = F[((int64_t)kk * n + jj) * n + ii];
    cp[q][0] = ax[ii];
    cp[q][1] = ax[jj];
    cp[q][2] = ax[kk];
  }
}

__global__ __launch_bounds__(256) void k_mt_count(const float* __restrict__ F, const float* __restrict__ ax, int n,
                                                  float iso, int32_t* __restrict__ cnt) {
  const int64_t m3 = (int64_t)(n - 1) * (n - 1) * (n - 1);
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < m3; c += (int64_t)gridDim.x * blockDim.x) {
    float cv[8], cp[8][3];
    load_cube(F, ax, n, c, cv, cp);
    int t = 0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const float v[4] = {cv[kTet[q][0]], cv[kTet[q][1]], cv[kTet[q][2]], cv[kTet[q][3]]};
      t += tet_tris(v, iso);
    }
    cnt[c] = t;
  }
}

// 64-bit total of the per-cube counts (integer atomics: the sum does not
// depend on their order)
__global__ __launch_bounds__(256) void k_count_total(const int32_t* __restrict__ cnt, int64_t m3,
                                                     unsigned long long* __restrict__ total) {
  unsigned long long acc = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < m3; c += (int64_t)gridDim.x * blockDim.x)
    acc += (unsigned long long)cnt[c];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0 && acc) atomicAdd(total, acc);
}

__device__ __forceinline__ void edge_point(const float cp[8][3], const float cv[8], int a, int b, float iso,
                                           float* out) {
  // an infinite corner value (eq. 3-10 inverted where the network gives
  // t <= 0) is infinitely far outside: the vertex sits on the other corner
  const float t = isinf(cv[b]) ? 0.f : (isinf(cv[a]) ? 1.f : (iso - cv[a]) / (cv[b] - cv[a]));
#pragma unroll
  for (int d = 0; d < 3; ++d) out[d] = cp[a][d] + t * (cp[b][d] - cp[a][d]);
}

__global__ __launch_bounds__(256) void k_mt_emit(const float* __restrict__ F, const float* __restrict__ ax, int n,
                                                 float iso, const int32_t* __restrict__ off, float* __restrict__ tris,
                                                 int64_t cap) {
  const int64_t m3 = (int64_t)(n - 1) * (n - 1) * (n - 1);
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < m3; c += (int64_t)gridDim.x * blockDim.x) {
    int64_t w = off[c];
    if (off[c + 1] == w) continue;
    float cv[8], cp[8][3];
    load_cube(F, ax, n, c, cv, cp);
    for (int q = 0; q < 6; ++q) {
      int ins[4], outs[4], ni = 0, no = 0;
      for (int r = 0; r < 4; ++r) {
        const int corner = kTet[q][r];
        if (cv[corner] < iso) ins[ni++] = corner;
        else outs[no++] = corner;
      }
      if (ni == 0 || ni == 4) continue;
      if (ni == 1 || ni == 3) {
        const int lone = ni == 1 ? ins[0] : outs[0];
        const int* oth = ni == 1 ? outs : ins;
        if (w < cap) {
          float* o = tris + 9 * w;
          edge_point(cp, cv, lone, oth[0], iso, o);
          edge_point(cp, cv, lone, oth[1], iso, o + 3);
          edge_point(cp, cv, lone, oth[2], iso, o + 6);
        }
        w += 1;
      } else {
        float e0[3], e1[3], e2[3], e3[3];
        edge_point(cp, cv, ins[0], outs[0], iso, e0);
        edge_point(cp, cv, ins[0], outs[1], iso, e1);
        edge_point(cp, cv, ins[1], outs[1], iso, e2);
        edge_point(cp, cv, ins[1], outs[0], iso, e3);
        if (w < cap) {
          float* o = tris + 9 * w;
          for (int d = 0; d < 3; ++d) { o[d] = e0[d]; o[3 + d] = e1[d]; o[6 + d] = e2[d]; }
        }
        if (w + 1 < cap) {
          float* o = tris + 9 * (w + 1);
          for (int d = 0; d < 3; ++d) { o[d] = e0[d]; o[3 + d] = e2[d]; o[6 + d] = e3[d]; }
        }
        w += 2;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_tri_area(const float* __restrict__ tris, int64_t nt, double* __restrict__ area) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
    const float* p = tris + 9 * t;
    const double ux = (double)p[3] - p[0], uy = (double)p[4] - p[1], uz = (double)p[5] - p[2];
    const double vx = (double)p[6] - p[0], vy = (double)p[7] - p[1], vz = (double)p[8] - p[2];
    const double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    area[t] = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
  }
}

// running sum of the areas: an inclusive scan of 1024-value blocks (wave
// shuffles, then the 16 wave totals), the block totals scanned by one block,
// and the offsets added back; a fixed order, so every run rounds alike
__device__ __forceinline__ double block_incl_scan_1024(double v, double* sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  double base = 0.0;
  for (int w = 0; w < wv; ++w) base += sh[w];
  __syncthreads();
  return base + x;
}

__global__ __launch_bounds__(1024) void k_dscan_blocks(double* __restrict__ a, int64_t n, double* __restrict__ tot) {
  __shared__ double sh[16];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const double x = block_incl_scan_1024(i < n ? a[i] : 0.0, sh);
  if (i < n) a[i] = x;
  if (threadIdx.x == 1023) tot[blockIdx.x] = x;
}

__global__ __launch_bounds__(1024) void k_dscan_top(double* __restrict__ tot, int64_t nb) {
  __shared__ double sh[16];
  __shared__ double carry;
  if (threadIdx.x == 0) carry = 0.0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const double v = i < nb ? tot[i] : 0.0;
    const double x = block_incl_scan_1024(v, sh);
    const double c = carry;
    if (i < nb) tot[i] = c + x;   // running total up to and including block i
    __syncthreads();
    if (threadIdx.x == 1023) carry = c + x;
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_dscan_add(double* __restrict__ a, int64_t n, const double* __restrict__ tot) {
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i < n && blockIdx.x > 0) a[i] += tot[blockIdx.x - 1];
}

__global__ __launch_bounds__(256) void k_sample_tris(const float* __restrict__ tris, int64_t nt,
                                                     const double* __restrict__ csum, const float* __restrict__ u,
                                                     int64_t ns, float* __restrict__ pts, float* __restrict__ nrm,
                                                     int32_t* __restrict__ which) {
  const double total = csum[nt - 1];
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += (int64_t)gridDim.x * blockDim.x) {
    const double target = (double)u[3 * s] * total;
    // first t with csum[t] > target
    int64_t lo = 0, hi = nt;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (csum[mid] > target) hi = mid;
      else lo = mid + 1;
    }
    const int64_t t = min(lo, nt - 1);
    const float* p = tris + 9 * t;
    const double r1 = sqrt((double)u[3 * s + 1]), r2 = (double)u[3 * s + 2];
    const double wa = 1.0 - r1, wb = r1 * (1.0 - r2), wc = r1 * r2;
#pragma unroll
    for (int d = 0; d < 3; ++d) pts[3 * s + d] = (float)(wa * p[d] + wb * p[3 + d] + wc * p[6 + d]);
    const double ux = (double)p[3] - p[0], uy = (double)p[4] - p[1], uz = (double)p[5] - p[2];
    const double vx = (double)p[6] - p[0], vy = (double)p[7] - p[1], vz = (double)p[8] - p[2];
    const double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    const double inv = 1.0 / sqrt(cx * cx + cy * cy + cz * cz);
    nrm[3 * s] = (float)(cx * inv);
    nrm[3 * s + 1] = (float)(cy * inv);
    nrm[3 * s + 2] = (float)(cz * inv);
    if (which) which[s] = (int32_t)t;
  }
}

// closest point of R for every point of Q: distance and |n_q . n_r|
__global__ __launch_bounds__(256) void k_closest(const float* __restrict__ Q, const float* __restrict__ NQ, int64_t nq,
                                                 const float* __restrict__ R, const float* __restrict__ NR, int64_t nr,
                                                 double* __restrict__ dist, double* __restrict__ cosabs) {
  __shared__ float4 sr[256];
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = q < nq;
  const float qx = valid ? Q[3 * q] : 0.f, qy = valid ? Q[3 * q + 1] : 0.f, qz = valid ? Q[3 * q + 2] : 0.f;
  float best = INFINITY;
  int64_t arg = 0;
  for (int64_t r0 = 0; r0 < nr; r0 += 256) {
    const int64_t r = r0 + threadIdx.x;
    __syncthreads();
    if (r < nr) sr[threadIdx.x] = make_float4(R[3 * r], R[3 * r + 1], R[3 * r + 2], 0.f);
    __syncthreads();
    const int cnt = (int)min((int64_t)256, nr - r0);
    for (int k = 0; k < cnt; ++k) {
      const float4 p = sr[k];
      const float dx = p.x - qx, dy = p.y - qy, dz = p.z - qz;
      const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
      if (d2 < best) {
        best = d2;
        arg = r0 + k;
      }
    }
  }
  if (valid) {
    dist[q] = sqrt((double)best);
    const double c = (double)NQ[3 * q] * NR[3 * arg] + (double)NQ[3 * q + 1] * NR[3 * arg + 1] +
                     (double)NQ[3 * q + 2] * NR[3 * arg + 2];
    cosabs[q] = fabs(c);
  }
}

// HD, CD, CS from the two directions' records, in a fixed order (one block)
__global__ __launch_bounds__(1024) void k_metrics(const double* __restrict__ d_tr, const double* __restrict__ c_tr,
                                                  int64_t nt, const double* __restrict__ d_rt,
                                                  const double* __restrict__ c_rt, int64_t nr,
                                                  double* __restrict__ out) {
  __shared__ double sh[4][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double mx = 0.0, s_tr = 0.0, s_rt = 0.0, k_tr = 0.0, k_rt = 0.0;
  for (int64_t i = tid; i < nt; i += 1024) {
    mx = fmax(mx, d_tr[i]);
    s_tr += d_tr[i];
    k_tr += c_tr[i];
  }
  for (int64_t i = tid; i < nr; i += 1024) {
    mx = fmax(mx, d_rt[i]);
    s_rt += d_rt[i];
    k_rt += c_rt[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  s_tr = wave_sum(s_tr);
  s_rt = wave_sum(s_rt);
  k_tr = wave_sum(k_tr);
  k_rt = wave_sum(k_rt);
  __shared__ double shm[16];
  if (lane == 0) {
    shm[wv] = mx;
    sh[0][wv] = s_tr;
    sh[1][wv] = s_rt;
    sh[2][wv] = k_tr;
    sh[3][wv] = k_rt;
  }
  __syncthreads();
  if (tid == 0) {
    double m = 0.0, a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (int w = 0; w < 16; ++w) {
      m = fmax(m, shm[w]);
      a += sh[0][w];
      b += sh[1][w];
      c += sh[2][w];
      d += sh[3][w];
    }
    out[0] = m;
    out[1] = 0.5 * a / (double)nt + 0.5 * b / (double)nr;
    out[2] = 0.5 * c / (double)nt + 0.5 * d / (double)nr;
  }
}

__global__ __launch_bounds__(256) void k_sdf_from_targets(const float* __restrict__ t, int64_t n, float m,
                                                          float* __restrict__ S) {
  const double md = m;
  const double h = 0.69314718055994530942 / (md * md);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double v = t[k];
    const double arg = v > 0.0 ? log(2.0 / v) : INFINITY;
    S[k] = (float)(md + sqrt(fmax(arg, 0.0) / h));
  }
}

inline unsigned gsz(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

}  // namespace

hipError_t launch_mt_count(const float* F, const float* ax, int n, float iso, int32_t* cnt, int64_t* total64,
                           hipStream_t s) {
  const int64_t m3 = (int64_t)(n - 1) * (n - 1) * (n - 1);
  hipLaunchKernelGGL(k_mt_count, dim3(gsz(m3)), dim3(256), 0, s, F, ax, n, iso, cnt);
  hipLaunchKernelGGL(k_count_total, dim3(gsz(m3)), dim3(256), 0, s, cnt, m3,
                     reinterpret_cast<unsigned long long*>(total64));
  return hipGetLastError();
}

hipError_t launch_mt_emit(const float* F, const float* ax, int n, float iso, const int32_t* off, float* tris,
                          int64_t cap, hipStream_t s) {
  const int64_t m3 = (int64_t)(n - 1) * (n - 1) * (n - 1);
  hipLaunchKernelGGL(k_mt_emit, dim3(gsz(m3)), dim3(256), 0, s, F, ax, n, iso, off, tris, cap);
  return hipGetLastError();
}

hipError_t launch_surface_sample(const float* tris, int64_t nt, const float* u, int64_t ns, double* area, float* pts,
                                 float* nrm, int32_t* which, hipStream_t s) {
  // area holds nt areas followed by one block total per 1024 areas
  const int64_t nb = (nt + 1023) / 1024;
  double* tot = area + nt;
  hipLaunchKernelGGL(k_tri_area, dim3(gsz(nt)), dim3(256), 0, s, tris, nt, area);
  hipLaunchKernelGGL(k_dscan_blocks, dim3((unsigned)nb), dim3(1024), 0, s, area, nt, tot);
  hipLaunchKernelGGL(k_dscan_top, dim3(1), dim3(1024), 0, s, tot, nb);
  hipLaunchKernelGGL(k_dscan_add, dim3((unsigned)nb), dim3(1024), 0, s, area, nt, tot);
  hipLaunchKernelGGL(k_sample_tris, dim3(gsz(ns)), dim3(256), 0, s, tris, nt, area, u, ns, pts, nrm, which);
  return hipGetLastError();
}

hipError_t launch_surface_metrics(const float* Pt, const float* Nt, int64_t nt, const float* Pr, const float* Nr,
                                  int64_t nr, double* scratch, double* out, hipStream_t s) {
  double* d_tr = scratch;
  double* c_tr = scratch + nt;
  double* d_rt = scratch + 2 * nt;
  double* c_rt = scratch + 2 * nt + nr;
  hipLaunchKernelGGL(k_closest, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, Pt, Nt, nt, Pr, Nr, nr, d_tr, c_tr);
  hipLaunchKernelGGL(k_closest, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, Pr, Nr, nr, Pt, Nt, nt, d_rt, c_rt);
  hipLaunchKernelGGL(k_metrics, dim3(1), dim3(1024), 0, s, d_tr, c_tr, nt, d_rt, c_rt, nr, out);
  return hipGetLastError();
}

// Device scratch of the metrics variant that allocates nothing: one copy per
// GPU, held until the process ends.  In host code `scratch` names a host-side
// stand-in; its device address comes from hipGetSymbolAddress, once per
// device, and only that address is handed to kernels.
static __device__ __align__(256) double scratch[2 * kNoallocMetricsPoints];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_metrics_scratch(double** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

hipError_t launch_sdf_from_targets(const float* t, int64_t n, float m, float* S, hipStream_t s) {
  hipLaunchKernelGGL(k_sdf_from_targets, dim3(gsz(n)), dim3(256), 0, s, t, n, m, S);
  return hipGetLastError();
}

}  // namespace erbf
