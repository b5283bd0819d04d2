// Exclusive prefix sums of int32 counts (row pointers, subgraph offsets).
// Three launches: per-block totals, one-block scan of the totals, per-block scan + offset.
#include "internal.h"

namespace gbi {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 8;
constexpr int kPerBlock = kThreads * kPerThread;

template <typename T>
__device__ T block_exclusive_scan(T v, T* lds_waves, T* total) {
  // wavefront inclusive scan (64 lanes), then across the 4 waves through LDS
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) lds_waves[wave] = x;
  __syncthreads();
  T base = 0, all = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wave) base += lds_waves[w];
    all += lds_waves[w];
  }
  __syncthreads();
  *total = all;
  return base + x - v;
}

__global__ void k_block_sums(const int32_t* __restrict__ in, int n, int64_t* __restrict__ sums) {
  __shared__ int64_t w[kThreads / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kPerBlock;
  int64_t acc = 0;
  for (int i = 0; i < kPerThread; ++i) {
    int64_t k = b0 + (int64_t)threadIdx.x * kPerThread + i;
    if (k < n) acc += in[k];
  }
  int64_t tot;
  block_exclusive_scan<int64_t>(acc, w, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_sums(int64_t* __restrict__ sums, int nb) {
  __shared__ int64_t w[kThreads / 64];
  int64_t carry = 0;
  for (int base = 0; base < nb; base += kThreads) {
    int k = base + threadIdx.x;
    int64_t v = k < nb ? sums[k] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan<int64_t>(v, w, &tot);
    if (k < nb) sums[k] = carry + ex;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

template <typename TO>
__global__ void k_scan_apply(const int32_t* __restrict__ in, int n, const int64_t* __restrict__ sums,
                             TO* __restrict__ out, int nb) {
  __shared__ int64_t w[kThreads / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kPerBlock;
  const int64_t t0 = b0 + (int64_t)threadIdx.x * kPerThread;
  int64_t vals[kPerThread];
  int64_t acc = 0;
  for (int i = 0; i < kPerThread; ++i) {
    vals[i] = (t0 + i < n) ? in[t0 + i] : 0;
    acc += vals[i];
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan<int64_t>(acc, w, &tot) + sums[blockIdx.x];
  for (int i = 0; i < kPerThread; ++i) {
    if (t0 + i < n) out[t0 + i] = (TO)ex;
    ex += vals[i];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = (TO)sums[nb];
}

template <typename TO>
void scan_impl(const int32_t* in, TO* out, int n, hipStream_t s) {
  if (n == 0) {
    GB_HIP(hipMemsetAsync(out, 0, sizeof(TO), s));
    return;
  }
  const int nb = (n + kPerBlock - 1) / kPerBlock;
  DBuf<int64_t> sums(nb + 1, s);
  hipLaunchKernelGGL(k_block_sums, dim3(nb), dim3(kThreads), 0, s, in, n, sums.get());
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kThreads), 0, s, sums.get(), nb);
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_apply<TO>, dim3(nb), dim3(kThreads), 0, s, in, n, sums.get(), out, nb);
  GB_LAUNCH_CHECK();
}

}  // namespace

void exclusive_scan_i32(const int32_t* in, int32_t* out, int n, hipStream_t s) {
  scan_impl<int32_t>(in, out, n, s);
}
void exclusive_scan_i64(const int32_t* in, int64_t* out, int n, hipStream_t s) {
  scan_impl<int64_t>(in, out, n, s);
}

}  // namespace gbi
