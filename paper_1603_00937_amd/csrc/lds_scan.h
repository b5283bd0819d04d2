// Block-wide exclusive prefix sum of an int32 array held in LDS, shared by the graph and partition
// kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gbi {

// v[0..m) <- exclusive prefix sums of v (in place); returns the total.  All NT threads of the
// block call it; red is an LDS array of NT entries.  Thread t owns the contiguous segment
// [t s, t s + s) of v, s = ceil(m / NT): segment sums, one scan of the NT sums, then each segment
// rewritten from its offset (one scan however long v is).
template <int NT>
__device__ __forceinline__ int32_t lds_exclusive_scan(int32_t* v, int m, int32_t* red) {
  const int seg = (m + NT - 1) / NT;
  const int b = min((int)threadIdx.x * seg, m), e = min(b + seg, m);
  int32_t sum = 0;
  for (int k = b; k < e; ++k) sum += v[k];
  __syncthreads();
  red[threadIdx.x] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan over NT values
  for (int d = 1; d < NT; d <<= 1) {
    const int32_t y = threadIdx.x >= d ? red[threadIdx.x - d] : 0;
    __syncthreads();
    red[threadIdx.x] += y;
    __syncthreads();
  }
  int32_t run = red[threadIdx.x] - sum;
  for (int k = b; k < e; ++k) {
    const int32_t x = v[k];
    v[k] = run;
    run += x;
  }
  const int32_t total = red[NT - 1];
  __syncthreads();
  return total;
}

}  // namespace gbi
