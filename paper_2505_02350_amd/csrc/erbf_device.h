// Small device helpers shared by the HIP translation units (wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace erbf {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// exclusive scan over a 1024-thread block (16 waves); also returns the total
// (T = int or int64_t; sh holds 32 values of T)
template <typename T>
__device__ __forceinline__ T block_excl_scan_1024(T v, T* sh, T& total) {
  // 1024 threads, 16 waves
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  if (wv == 0) {
    T s = lane < 16 ? sh[lane] : (T)0;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const T y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < 16) sh[16 + lane] = s;
  }
  __syncthreads();
  total = sh[31];
  const T wbase = wv > 0 ? sh[16 + wv - 1] : (T)0;
  const T r = wbase + x - v;
  __syncthreads();
  return r;
}

}  // namespace erbf
