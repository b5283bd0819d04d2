// Cores (communities, obs. vi-vii) and core+halo subgraphs (Eq. 6).
// A subgraph lists its core vertices ascending, then its halo -- every vertex outside the
// core adjacent to a core vertex -- ascending.  One workgroup per core builds the halo in an
// LDS bitmap over all vertices, so the lists come out sorted and duplicate-free.
#include "internal.h"

namespace gbi {
namespace {

constexpr int kT = 256;

__device__ int32_t lds_exclusive_scan(int32_t* v, int m, int32_t* red) {
  int32_t carry = 0;
  for (int base = 0; base < m; base += kT) {
    const int k = base + threadIdx.x;
    const int32_t x = k < m ? v[k] : 0;
    __syncthreads();
    red[threadIdx.x] = x;
    __syncthreads();
    for (int d = 1; d < kT; d <<= 1) {
      const int32_t y = threadIdx.x >= d ? red[threadIdx.x - d] : 0;
      __syncthreads();
      red[threadIdx.x] += y;
      __syncthreads();
    }
    if (k < m) v[k] = carry + red[threadIdx.x] - x;
    carry += red[kT - 1];
    __syncthreads();
  }
  return carry;
}

template <int PASS>
__global__ __launch_bounds__(kT) void k_halo(int n, const int32_t* __restrict__ rp,
                                             const int32_t* __restrict__ col,
                                             const int32_t* __restrict__ core_ptr,
                                             const int32_t* __restrict__ core_vtx,
                                             int32_t* __restrict__ cnt,
                                             const int32_t* __restrict__ sub_ptr,
                                             int32_t* __restrict__ sub_idx) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int c = blockIdx.x;
  const int nw = (n + 31) >> 5;
  uint32_t* bits = reinterpret_cast<uint32_t*>(smem);
  int32_t* wc = reinterpret_cast<int32_t*>(bits + nw);
  int32_t* red = wc + nw;
  const int c0 = core_ptr[c], c1 = core_ptr[c + 1];
  for (int q = threadIdx.x; q < nw; q += kT) bits[q] = 0u;
  __syncthreads();
  for (int v = c0; v < c1; ++v) {
    const int u = core_vtx[v];
    for (int p = rp[u] + threadIdx.x; p < rp[u + 1]; p += kT) {
      const int j = col[p];
      atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
  }
  __syncthreads();
  for (int v = c0 + threadIdx.x; v < c1; v += kT) {
    const int u = core_vtx[v];
    atomicAnd(&bits[u >> 5], ~(1u << (u & 31)));
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nw; q += kT) wc[q] = __popc(bits[q]);
  __syncthreads();
  const int32_t halo = lds_exclusive_scan(wc, nw, red);
  if (PASS == 0) {
    if (threadIdx.x == 0) cnt[c] = (c1 - c0) + halo;
    return;
  }
  const int32_t base = sub_ptr[c];
  for (int v = c0 + threadIdx.x; v < c1; v += kT) sub_idx[base + (v - c0)] = core_vtx[v];
  const int32_t hb = base + (c1 - c0);
  for (int q = threadIdx.x; q < nw; q += kT) {
    uint32_t word = bits[q];
    int32_t pos = hb + wc[q];
    while (word) {
      const int b = __ffs(word) - 1;
      sub_idx[pos++] = (q << 5) + b;
      word &= word - 1u;
    }
  }
}

// rank of every subgraph entry in ascending global order: the two sorted runs (core, halo)
// are merged by binary search of each entry in the other run.
__global__ void k_sub_pos(int n_sub, const int32_t* __restrict__ core_ptr,
                          const int32_t* __restrict__ sub_ptr,
                          const int32_t* __restrict__ sub_idx, int32_t* __restrict__ pos) {
  const int s = blockIdx.x;
  const int b = sub_ptr[s], e = sub_ptr[s + 1];
  const int k = core_ptr[s + 1] - core_ptr[s];
  const int32_t* core = sub_idx + b;
  const int32_t* halo = sub_idx + b + k;
  const int nh = e - b - k;
  for (int a = threadIdx.x; a < e - b; a += blockDim.x) {
    const int32_t v = sub_idx[b + a];
    const int32_t* other = a < k ? halo : core;
    int lo = 0, hi = a < k ? nh : k;  // count of entries < v in the other run
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (other[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    pos[b + a] = (a < k ? a : a - k) + lo;
  }
}

// vertex -> (subgraph, local index within the subgraph) for core vertices
__global__ void k_col_map(int n_sub, const int32_t* __restrict__ core_ptr,
                          const int32_t* __restrict__ core_vtx, int32_t* __restrict__ col_sub,
                          int32_t* __restrict__ col_loc) {
  const int s = blockIdx.x;
  for (int v = core_ptr[s] + threadIdx.x; v < core_ptr[s + 1]; v += blockDim.x) {
    const int u = core_vtx[v];
    col_sub[u] = s;
    col_loc[u] = v - core_ptr[s];
  }
}

__global__ void k_iota(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

}  // namespace

void partition_block(const Csr& g, int32_t core_size, Part& P, hipStream_t s) {
  const int n = g.n;
  const int n_sub = (n + core_size - 1) / core_size;
  P.n = n;
  P.n_sub = n_sub;
  P.h_core_ptr.resize(n_sub + 1);
  for (int c = 0; c <= n_sub; ++c)
    P.h_core_ptr[c] = (int32_t)std::min<int64_t>((int64_t)c * core_size, n);
  P.core_ptr = DBuf<int32_t>(n_sub + 1, s);
  GB_HIP(hipMemcpyAsync(P.core_ptr.get(), P.h_core_ptr.data(), (n_sub + 1) * 4,
                        hipMemcpyHostToDevice, s));
  P.core_vtx = DBuf<int32_t>(n, s);
  hipLaunchKernelGGL(k_iota, dim3((n + kT - 1) / kT), dim3(kT), 0, s, P.core_vtx.get(), n);
  GB_LAUNCH_CHECK();

  const int nw = (n + 31) >> 5;
  const size_t lds = (size_t)nw * 8 + kT * 4 + 64;
  if (lds > 160 * 1024) fail(GB_EUNSUPPORTED, "partition: n = %d too large for one LDS bitmap", n);
  DBuf<int32_t> cnt(n_sub, s);
  hipLaunchKernelGGL(k_halo<0>, dim3(n_sub), dim3(kT), lds, s, n, g.row_ptr.get(), g.col.get(),
                     P.core_ptr.get(), P.core_vtx.get(), cnt.get(), nullptr, nullptr);
  GB_LAUNCH_CHECK();
  P.sub_ptr = DBuf<int32_t>(n_sub + 1, s);
  exclusive_scan_i32(cnt.get(), P.sub_ptr.get(), n_sub, s);
  P.h_sub_ptr.resize(n_sub + 1);
  GB_HIP(hipMemcpyAsync(P.h_sub_ptr.data(), P.sub_ptr.get(), (n_sub + 1) * 4,
                        hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  P.total = P.h_sub_ptr[n_sub];
  P.max_sub = 0;
  for (int c = 0; c < n_sub; ++c)
    P.max_sub = std::max(P.max_sub, P.h_sub_ptr[c + 1] - P.h_sub_ptr[c]);
  P.sub_idx = DBuf<int32_t>(P.total, s);
  hipLaunchKernelGGL(k_halo<1>, dim3(n_sub), dim3(kT), lds, s, n, g.row_ptr.get(), g.col.get(),
                     P.core_ptr.get(), P.core_vtx.get(), nullptr, P.sub_ptr.get(),
                     P.sub_idx.get());
  GB_LAUNCH_CHECK();
  P.sub_pos = DBuf<int32_t>(P.total, s);
  hipLaunchKernelGGL(k_sub_pos, dim3(n_sub), dim3(kT), 0, s, n_sub, P.core_ptr.get(),
                     P.sub_ptr.get(), P.sub_idx.get(), P.sub_pos.get());
  GB_LAUNCH_CHECK();
  P.col_sub = DBuf<int32_t>(n, s);
  P.col_loc = DBuf<int32_t>(n, s);
  hipLaunchKernelGGL(k_col_map, dim3(n_sub), dim3(kT), 0, s, n_sub, P.core_ptr.get(),
                     P.core_vtx.get(), P.col_sub.get(), P.col_loc.get());
  GB_LAUNCH_CHECK();
}

}  // namespace gbi
