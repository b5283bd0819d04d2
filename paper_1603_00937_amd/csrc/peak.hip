// Rates this device sustains, measured by the library's own kernels (the denominators the
// rooflines of the squaring kernels are read against besides the datasheet figures): matrix-core
// throughput per data type from independent MFMA chains on register operands (no memory
// traffic), and HBM bandwidth from a streaming copy.
#include <vector>

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
typedef float f16v_p __attribute__((ext_vector_type(16)));
__device__ inline f16v_p peak_mma_bf16_32(bf8v_p a, bf8v_p b, f16v_p c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f16v_p peak_mma_f16_32(h8v_p a, h8v_p b, f16v_p c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

namespace {

constexpr int kChains = 8;  // independent accumulators per wave

// KIND 0 FP64 (16x16x4), 1 FP32 (16x16x4), 2 bf16 (16x16x32), 3 fp16 (16x16x32),
// 5 bf16 (32x32x16), 6 fp16 (32x32x16)
// Thread 0 of each workgroup also records the core cycles and the constant-rate wall-clock
// ticks its loop took (clk[2 b], clk[2 b + 1]): their ratio is the core clock under this load.
// Every chain has its own operand and starting value, so no two chains compute the same numbers
// (the compiler would otherwise merge them).
template <int KIND>
__global__ __launch_bounds__(256) void k_mfma_peak(float* __restrict__ out,
                                                   long long* __restrict__ clk, int iters) {
  const float seed = 1.0f + 1e-3f * (float)(threadIdx.x & 63);
  const long long c0 = clock64(), w0 = wall_clock64();
  float s = 0.f;
  if constexpr (KIND == 0) {
    d4v_p acc[kChains];
    double a[kChains];
    for (int q = 0; q < kChains; ++q) {
      acc[q] = d4v_p{(double)q, 0, 0, 0};
      a[q] = seed * (1.0 + 0.01 * q);
    }
    const double b = 1.0 - 1e-3 * seed;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_f64(a[q], b, acc[q]);
    for (int q = 0; q < kChains; ++q) s += (float)(acc[q][0] + acc[q][3]);
  } else if constexpr (KIND == 1) {
    f4v_p acc[kChains];
    float a[kChains];
    for (int q = 0; q < kChains; ++q) {
      acc[q] = f4v_p{(float)q, 0, 0, 0};
      a[q] = seed * (1.0f + 0.01f * q);
    }
    const float b = 1.0f - 1e-3f * seed;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_f32(a[q], b, acc[q]);
    for (int q = 0; q < kChains; ++q) s += acc[q][0] + acc[q][3];
  } else if constexpr (KIND >= 5) {
    f16v_p acc[kChains];
    for (int q = 0; q < kChains; ++q) {
      acc[q] = f16v_p{};
      acc[q][0] = (float)q;
    }
    if constexpr (KIND == 5) {
      bf8v_p a[kChains], b;
      for (int e = 0; e < 8; ++e) {
        for (int q = 0; q < kChains; ++q) a[q][e] = (__bf16)(seed * (1.0f + 0.01f * (e + 8 * q)));
        b[e] = (__bf16)(1.0f - 0.01f * e);
      }
      for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_bf16_32(a[q], b, acc[q]);
    } else {
      h8v_p a[kChains], b;
      for (int e = 0; e < 8; ++e) {
        for (int q = 0; q < kChains; ++q)
          a[q][e] = (_Float16)(seed * (1.0f + 0.01f * (e + 8 * q)));
        b[e] = (_Float16)(1.0f - 0.01f * e);
      }
      for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_f16_32(a[q], b, acc[q]);
    }
    for (int q = 0; q < kChains; ++q) s += acc[q][0] + acc[q][15];
  } else {
    f4v_p acc[kChains];
    for (int q = 0; q < kChains; ++q) acc[q] = f4v_p{(float)q, 0, 0, 0};
    if constexpr (KIND == 2) {
      bf8v_p a[kChains], b;
      for (int e = 0; e < 8; ++e) {
        for (int q = 0; q < kChains; ++q) a[q][e] = (__bf16)(seed * (1.0f + 0.01f * (e + 8 * q)));
        b[e] = (__bf16)(1.0f - 0.01f * e);
      }
      for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_bf16(a[q], b, acc[q]);
    } else {
      h8v_p a[kChains], b;
      for (int e = 0; e < 8; ++e) {
        for (int q = 0; q < kChains; ++q)
          a[q][e] = (_Float16)(seed * (1.0f + 0.01f * (e + 8 * q)));
        b[e] = (_Float16)(1.0f - 0.01f * e);
      }
      for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < kChains; ++q) acc[q] = peak_mma_f16(a[q], b, acc[q]);
    }
    for (int q = 0; q < kChains; ++q) s += acc[q][0] + acc[q][3];
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = clock64() - c0;
    clk[2 * blockIdx.x + 1] = wall_clock64() - w0;
  }
}

__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ a,
                                                     float4* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    b[i] = a[i];
}

}  // namespace

// flops of one MFMA instruction per kind (16 x 16 outputs with k = 4 or 32; 32 x 32 with k = 16)
static double mfma_flops(int kind) {
  return kind <= 1 ? 2.0 * 16 * 16 * 4 : kind <= 3 ? 2.0 * 16 * 16 * 32 : 2.0 * 32 * 32 * 16;
}

double peak_rate(int kind, hipStream_t s, double* clock_mhz) {
  if (clock_mhz) *clock_mhz = 0.0;
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
  if (kind != 4) {
    const int grid = cus * 8, iters = kind == 0 ? 2048 : kind >= 5 ? 2048 : 4096;
    DBuf<float> out((size_t)grid * 256, s);
    DBuf<long long> clk((size_t)grid * 2, s);
    auto launch = [&] {
      float* o = out.get();
      long long* c = clk.get();
      if (kind == 0) hipLaunchKernelGGL(k_mfma_peak<0>, dim3(grid), dim3(256), 0, s, o, c, iters);
      else if (kind == 1) hipLaunchKernelGGL(k_mfma_peak<1>, dim3(grid), dim3(256), 0, s, o, c, iters);
      else if (kind == 2) hipLaunchKernelGGL(k_mfma_peak<2>, dim3(grid), dim3(256), 0, s, o, c, iters);
      else if (kind == 3) hipLaunchKernelGGL(k_mfma_peak<3>, dim3(grid), dim3(256), 0, s, o, c, iters);
      else if (kind == 5) hipLaunchKernelGGL(k_mfma_peak<5>, dim3(grid), dim3(256), 0, s, o, c, iters);
      else hipLaunchKernelGGL(k_mfma_peak<6>, dim3(grid), dim3(256), 0, s, o, c, iters);
      GB_LAUNCH_CHECK();
    };
    launch();  // warm-up (clocks up)
    GB_HIP(hipEventRecord(a, s));
    for (int r = 0; r < 5; ++r) launch();
    GB_HIP(hipEventRecord(b, s));
    GB_HIP(hipEventSynchronize(b));
    GB_HIP(hipEventElapsedTime(&ms, a, b));
    work = 5.0 * grid * 4.0 * iters * kChains * mfma_flops(kind);  // 4 waves per workgroup
    if (clock_mhz) {  // the last launch's workgroups: core cycles over wall-clock ticks
      std::vector<long long> h((size_t)grid * 2);
      GB_HIP(hipMemcpy(h.data(), clk.get(), h.size() * sizeof(long long), hipMemcpyDeviceToHost));
      double cyc = 0.0, tick = 0.0;
      for (int b = 0; b < grid; ++b) {
        cyc += (double)h[2 * b];
        tick += (double)h[2 * b + 1];
      }
      int wall_khz = 0;
      GB_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
      if (tick > 0) *clock_mhz = cyc / tick * wall_khz / 1000.0;
    }
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
