// Rates this device sustains, measured by the library's own kernels (the denominators the
// rooflines of the squaring kernels are read against besides the datasheet figures): matrix-core
// throughput per data type from independent MFMA chains on register operands (no memory
// traffic), and HBM bandwidth from a streaming copy.
#include "internal.h"

#pragma clang fp contract(off)

namespace gbi {

typedef double d4v_p __attribute__((ext_vector_type(4)));
typedef float f4v_p __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v_p __attribute__((ext_vector_type(8)));
typedef _Float16 h8v_p __attribute__((ext_vector_type(8)));

__device__ inline d4v_p peak_mma_f64(double a, double b, d4v_p c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4v_p peak_mma_f32(float a, float b, f4v_p c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f4v_p peak_mma_bf16(bf8v_p a, bf8v_p b, f4v_p c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f4v_p peak_mma_f16(h8v_p a, h8v_p b, f4v_p c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

namespace {

constexpr int kChains = 8;  // independent accumulators per wave

// KIND 0 FP64 (16x16x4), 1 FP32 (16x16x4), 2 bf16 (16x16x32), 3 fp16 (16x16x32)
template <int KIND>
__global__ __launch_bounds__(256) void k_mfma_peak(float* __restrict__ out, int iters) {
  const float seed = 1.0f + 1e-3f * (float)(threadIdx.x & 63);
  float s = 0.f;
  if constexpr (KIND == 0) {
    d4v_p acc[kChains];
    for (int q = 0; q < kChains; ++q) acc[q] = d4v_p{0, 0, 0, 0};
    const double a = seed, b = 1.0 - 1e-3 * seed;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_f64(a, b, acc[q]);
    for (int q = 0; q < kChains; ++q) s += (float)(acc[q][0] + acc[q][3]);
  } else if constexpr (KIND == 1) {
    f4v_p acc[kChains];
    for (int q = 0; q < kChains; ++q) acc[q] = f4v_p{0, 0, 0, 0};
    const float a = seed, b = 1.0f - 1e-3f * seed;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_f32(a, b, acc[q]);
    for (int q = 0; q < kChains; ++q) s += acc[q][0] + acc[q][3];
  } else {
    f4v_p acc[kChains];
    for (int q = 0; q < kChains; ++q) acc[q] = f4v_p{0, 0, 0, 0};
    if constexpr (KIND == 2) {
      bf8v_p a, b;
      for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(seed * (1.0f + 0.01f * e));
        b[e] = (__bf16)(1.0f - 0.01f * e);
      }
      for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_bf16(a, b, acc[q]);
    } else {
      h8v_p a, b;
      for (int e = 0; e < 8; ++e) {
        a[e] = (_Float16)(seed * (1.0f + 0.01f * e));
        b[e] = (_Float16)(1.0f - 0.01f * e);
      }
      for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_f16(a, b, acc[q]);
    }
    for (int q = 0; q < kChains; ++q) s += acc[q][0] + acc[q][3];
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ a,
                                                     float4* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    b[i] = a[i];
}

}  // namespace

// flops of one MFMA instruction per kind (16 x 16 outputs, k = 4 or 32)
static double mfma_flops(int kind) { return kind <= 1 ? 2.0 * 16 * 16 * 4 : 2.0 * 16 * 16 * 32; }

double peak_rate(int kind, hipStream_t s) {
  int dev = 0, cus = 0;
  GB_HIP(hipGetDevice(&dev));
  GB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  hipEvent_t a, b;
  GB_HIP(hipEventCreate(&a));
  GB_HIP(hipEventCreate(&b));
  struct Ev {
    hipEvent_t& a;
    hipEvent_t& b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{a, b};
  float ms = 0.f;
  double work = 0.0;
  if (kind <= 3) {
    const int grid = cus * 8, iters = kind == 0 ? 2048 : kind == 1 ? 4096 : 4096;
    DBuf<float> out((size_t)grid * 256, s);
    auto launch = [&] {
      if (kind == 0) hipLaunchKernelGGL(k_mfma_peak<0>, dim3(grid), dim3(256), 0, s, out.get(), iters);
      else if (kind == 1) hipLaunchKernelGGL(k_mfma_peak<1>, dim3(grid), dim3(256), 0, s, out.get(), iters);
      else if (kind == 2) hipLaunchKernelGGL(k_mfma_peak<2>, dim3(grid), dim3(256), 0, s, out.get(), iters);
      else hipLaunchKernelGGL(k_mfma_peak<3>, dim3(grid), dim3(256), 0, s, out.get(), iters);
      GB_LAUNCH_CHECK();
    };
    launch();  // warm-up (clocks up)
    GB_HIP(hipEventRecord(a, s));
    for (int r = 0; r < 5; ++r) launch();
    GB_HIP(hipEventRecord(b, s));
    GB_HIP(hipEventSynchronize(b));
    GB_HIP(hipEventElapsedTime(&ms, a, b));
    work = 5.0 * grid * 4.0 * iters * kChains * mfma_flops(kind);  // 4 waves per workgroup
    return work / (ms * 1e-3) / 1e12;  // TFLOP/s
  }
  const int64_t n = (int64_t)1 << 27;  // 2 GiB each way
  DBuf<float4> x(n, s), y(n, s);
  hipLaunchKernelGGL(k_stream_copy, dim3(cus * 16), dim3(256), 0, s, x.get(), y.get(), n);
  GB_HIP(hipEventRecord(a, s));
  for (int r = 0; r < 5; ++r)
    hipLaunchKernelGGL(k_stream_copy, dim3(cus * 16), dim3(256), 0, s, x.get(), y.get(), n);
  GB_LAUNCH_CHECK();
  GB_HIP(hipEventRecord(b, s));
  GB_HIP(hipEventSynchronize(b));
  GB_HIP(hipEventElapsedTime(&ms, a, b));
  work = 5.0 * 2.0 * (double)n * 16.0;  // bytes read + written
  return work / (ms * 1e-3) / 1e9;      // GB/s
}

}  // namespace gbi
