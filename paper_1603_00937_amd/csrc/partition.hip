// Cores (communities, obs. vi-vii) and core+halo subgraphs (Eq. 6).
// A subgraph lists its core vertices ascending, then its halo -- every vertex outside the
// core adjacent to a core vertex -- ascending.  One workgroup per core builds the halo in an
// LDS bitmap over all vertices, so the lists come out sorted and duplicate-free.
#include "internal.h"
#include "lds_hash.h"
#include "lds_scan.h"

#include <climits>
#include <map>
#include <mutex>

namespace gbi {
namespace {

constexpr int kT = 256;


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
  const int32_t halo = lds_exclusive_scan<kT>(wc, nw, red);
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

// The same subgraph lists for any n: the neighbours of the core vertices go into an LDS hash set
// (2^log2h slots, empty kHashEmpty), the core vertices are dropped while the set is gathered
// (binary search in the ascending core), and the halo is sorted.  Inserts stop past cap
// entries (the set keeps room for kT more); such a core reports its count through `overflow`.
template <int PASS>
__global__ __launch_bounds__(kT) void k_halo_hash(int n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ core_ptr,
                                                  const int32_t* __restrict__ core_vtx,
                                                  int cap, int log2h, int log2u,
                                                  int32_t* __restrict__ cnt,
                                                  const int32_t* __restrict__ sub_ptr,
                                                  int32_t* __restrict__ sub_idx,
                                                  int32_t* __restrict__ overflow) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t count, gathered;
  const int c = blockIdx.x;
  const int H = 1 << log2h, P = 1 << log2u;
  int32_t* keys = reinterpret_cast<int32_t*>(smem);
  int32_t* U = keys + H;
  const int c0 = core_ptr[c], c1 = core_ptr[c + 1];
  for (int q = threadIdx.x; q < H; q += kT) keys[q] = kHashEmpty;
  if (threadIdx.x == 0) {
    count = 0;
    gathered = 0;
  }
  __syncthreads();
  for (int v = c0; v < c1 && *(volatile int32_t*)&count <= cap; ++v) {
    const int u = core_vtx[v];
    for (int p = rp[u] + threadIdx.x; p < rp[u + 1]; p += kT) {
      if (*(volatile int32_t*)&count > cap) break;
      if (hset_insert(keys, log2h, col[p])) atomicAdd(&count, 1);
    }
  }
  __syncthreads();
  if (count > cap) {
    if (threadIdx.x == 0) {
      atomicMax(overflow, count);
      if (PASS == 0) cnt[c] = 0;
    }
    return;
  }
  // gather the set minus the core (ascending: binary search)
  for (int q = threadIdx.x; q < H; q += kT) {
    const int32_t k = keys[q];
    if (k == kHashEmpty) continue;
    int lo = c0, hi = c1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (core_vtx[mid] < k) lo = mid + 1;
      else hi = mid;
    }
    if (lo < c1 && core_vtx[lo] == k) continue;
    U[atomicAdd(&gathered, 1)] = k;
  }
  __syncthreads();
  const int halo = gathered;
  if (PASS == 0) {
    if (threadIdx.x == 0) cnt[c] = (c1 - c0) + halo;
    return;
  }
  for (int r = halo + threadIdx.x; r < P; r += kT) U[r] = INT32_MAX;
  bitonic_sort<kT>(U, P);
  const int32_t base = sub_ptr[c];
  for (int v = c0 + threadIdx.x; v < c1; v += kT) sub_idx[base + (v - c0)] = core_vtx[v];
  for (int r = threadIdx.x; r < halo; r += kT) sub_idx[base + (c1 - c0) + r] = U[r];
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

__global__ void k_zero1(int32_t* p) { *p = 0; }

__global__ void k_iota(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}


// ---- Cuthill-McKee vertex order (one workgroup; the queue order is inherently sequential) ---
// Start at the unvisited vertex of smallest (degree, index); visit the queue in order, append
// each vertex's unvisited neighbours sorted by (degree, index); repeat per component.  The
// visited set is an LDS bitmap; the neighbours of one vertex are filtered, ranked and
// appended by all threads together.
constexpr int kCand = 2048;  // LDS capacity for one vertex's new neighbours

__global__ __launch_bounds__(kT) void k_cm_order(int n, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 int32_t* __restrict__ order,
                                                 int32_t* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nw = (n + 31) >> 5;
  uint32_t* seen = reinterpret_cast<uint32_t*>(smem);
  int64_t* cand = reinterpret_cast<int64_t*>(seen + nw + (nw & 1));
  __shared__ int32_t s_cnt, s_tail, s_head;
  __shared__ int64_t s_best[kT];
  for (int q = threadIdx.x; q < nw; q += kT) seen[q] = 0u;
  if (threadIdx.x == 0) {
    s_tail = 0;
    s_head = 0;
  }
  __syncthreads();
  while (true) {
    // next component: unvisited vertex with the smallest (degree, index)
    int64_t best = INT64_MAX;
    for (int v = threadIdx.x; v < n; v += kT)
      if (!(seen[v >> 5] & (1u << (v & 31)))) {
        const int64_t key = ((int64_t)(rp[v + 1] - rp[v]) << 32) | v;
        best = key < best ? key : best;
      }
    s_best[threadIdx.x] = best;
    __syncthreads();
    for (int h = kT / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h && s_best[threadIdx.x + h] < s_best[threadIdx.x])
        s_best[threadIdx.x] = s_best[threadIdx.x + h];
      __syncthreads();
    }
    if (s_best[0] == INT64_MAX) break;  // every vertex visited
    if (threadIdx.x == 0) {
      const int v = (int)(s_best[0] & 0xffffffff);
      seen[v >> 5] |= 1u << (v & 31);
      order[s_tail] = v;
      s_tail = s_tail + 1;
    }
    __syncthreads();
    while (s_head < s_tail) {
      const int v = order[s_head];
      if (threadIdx.x == 0) s_cnt = 0;
      __syncthreads();
      for (int p = rp[v] + threadIdx.x; p < rp[v + 1]; p += kT) {
        const int u = col[p];
        if (!(seen[u >> 5] & (1u << (u & 31)))) {
          const int slot = atomicAdd(&s_cnt, 1);
          if (slot < kCand) cand[slot] = ((int64_t)(rp[u + 1] - rp[u]) << 32) | u;
        }
      }
      __syncthreads();
      const int c = s_cnt;
      if (c > kCand) {
        if (threadIdx.x == 0) status[0] = c;
        return;  // uniform: every thread read the same count
      }
      // rank by (degree, index) and append; then mark visited
      const int tail = s_tail;
      for (int a = threadIdx.x; a < c; a += kT) {
        const int64_t ka = cand[a];
        int rank = 0;
        for (int b = 0; b < c; ++b) rank += cand[b] < ka;
        order[tail + rank] = (int)(ka & 0xffffffff);
      }
      __syncthreads();
      for (int a = threadIdx.x; a < c; a += kT) {
        const int u = (int)(cand[a] & 0xffffffff);
        atomicOr(&seen[u >> 5], 1u << (u & 31));
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        s_tail = tail + c;
        s_head = s_head + 1;
      }
      __syncthreads();
    }
  }
}

// each core's vertices sorted ascending (cores are blocks of the order)
__global__ void k_sort_cores(const int32_t* __restrict__ order, const int32_t* __restrict__ core_ptr,
                             int32_t* __restrict__ core_vtx) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  (void)c;
  const int cc = blockIdx.x;
  if (threadIdx.x != 0) return;
  const int b = core_ptr[cc], e = core_ptr[cc + 1];
  for (int i = b; i < e; ++i) core_vtx[i] = order[i];
  for (int i = b + 1; i < e; ++i) {
    const int x = core_vtx[i];
    int j = i - 1;
    while (j >= b && core_vtx[j] > x) {
      core_vtx[j + 1] = core_vtx[j];
      --j;
    }
    core_vtx[j + 1] = x;
  }
}

// Common closed neighbours of the ends of every edge: w[e] = |row u ∩ row col[e]| for the rows
// of a symmetric CSR graph that holds its self loops (so each row is the closed neighbourhood).
// One workgroup per vertex u: row u as a bitmap in LDS, then one wave per neighbour v >= u
// counting the entries of row v found in it; the count is symmetric, so the wave also writes
// it at the entry of u in row v, which it meets while scanning row v (each entry has one
// writer).  *missing receives the smallest u whose row lacks u (it is left as it was when
// every row holds its self loop).
__global__ __launch_bounds__(kT) void k_common_nb(int n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  int32_t* __restrict__ w,
                                                  int32_t* __restrict__ missing) {
  extern __shared__ uint32_t bits[];
  const int u = blockIdx.x;
  const int nw = (n + 31) >> 5;
  for (int i = threadIdx.x; i < nw; i += kT) bits[i] = 0u;
  __syncthreads();
  const int b = rp[u], e_end = rp[u + 1];
  for (int e = b + threadIdx.x; e < e_end; e += kT) {
    const int x = col[e];
    atomicOr(&bits[x >> 5], 1u << (x & 31));
  }
  __syncthreads();
  if (threadIdx.x == 0 && !((bits[u >> 5] >> (u & 31)) & 1u)) atomicMin(missing, u);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = b + wave; e < e_end; e += kT / 64) {
    const int v = col[e];
    if (v < u) continue;  // wave-uniform: workgroup v writes this entry
    int c = 0, pos = -1;
    const int f1 = rp[v + 1];
    for (int f = rp[v] + lane; f < f1; f += 4 * 64) {  // four loads in flight per lane
      int x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = f + 64 * i < f1 ? col[f + 64 * i] : -1;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (x[i] >= 0) {
          c += (bits[x[i] >> 5] >> (x[i] & 31)) & 1u;
          if (x[i] == u) pos = f + 64 * i;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
      c += __shfl_down(c, off, 64);
      pos = max(pos, __shfl_down(pos, off, 64));
    }
    if (lane == 0) {
      w[e] = c;
      if (v != u && pos >= 0) w[pos] = c;  // pos >= 0 in a symmetric graph
    }
  }
}

// The kMlTop heaviest neighbours of every vertex by (weight, -index), heaviest first, -1
// padded, the self loop skipped (the candidate lists the matching of the input level walks).
// One wave per vertex: each lane keeps the best kMlTop of its strided share of the row as
// 64-bit keys (weight, ~index), then kMlTop rounds of a wave maximum take the winners in order
// (keys are unique within a row, so one lane wins each round and drops its head).
__global__ __launch_bounds__(kT) void k_top_nb(int n, const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ col,
                                               const int32_t* __restrict__ w,
                                               int32_t* __restrict__ top) {
  const int lane = threadIdx.x & 63;
  const int v = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
  if (v >= n) return;  // wave-uniform
  uint64_t best[kMlTop];
#pragma unroll
  for (int i = 0; i < kMlTop; ++i) best[i] = 0;
  for (int e = rp[v] + lane; e < rp[v + 1]; e += 64) {
    const int u = col[e];
    if (u == v) continue;
    uint64_t x = ((uint64_t)(uint32_t)w[e] << 32) | (uint32_t)(~(uint32_t)u);
    if (x <= best[kMlTop - 1]) continue;
#pragma unroll
    for (int i = 0; i < kMlTop; ++i)
      if (x > best[i]) {
        const uint64_t t = best[i];
        best[i] = x;
        x = t;
      }
  }
  for (int r = 0; r < kMlTop; ++r) {
    uint64_t m = best[0];
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t lo = __shfl_xor((uint32_t)m, off, 64);
      const uint32_t hi = __shfl_xor((uint32_t)(m >> 32), off, 64);
      const uint64_t o = ((uint64_t)hi << 32) | lo;
      m = o > m ? o : m;
    }
    if (m != 0 && best[0] == m) {
#pragma unroll
      for (int i = 0; i + 1 < kMlTop; ++i) best[i] = best[i + 1];
      best[kMlTop - 1] = 0;
    }
    if (lane == 0) top[(int64_t)v * kMlTop + r] = m ? (int32_t)~(uint32_t)m : -1;
  }
}

// The first coarse level of the multilevel partitioner on the device.  Coarse vertex c is the
// pair {lead[c], match[lead[c]]} (one vertex when it is its own match); its row is the set of
// coarse vertices cmap[u] of its members' neighbours u other than c itself, ascending, each
// with the summed weights of the edges that lead to it (integer sums: any order gives the
// same).  One workgroup per coarse vertex, the set as an LDS bitmap over the nc coarse
// vertices; PASS 0 counts the row, PASS 1 writes it (accumulators indexed by rank, at most
// acap = the members' summed degrees).
template <int PASS>
__global__ __launch_bounds__(kT) void k_coarse_rows(int nc, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ w,
                                                    const int32_t* __restrict__ lead,
                                                    const int32_t* __restrict__ match,
                                                    const int32_t* __restrict__ cmap,
                                                    int32_t* __restrict__ cnt,
                                                    const int32_t* __restrict__ crp,
                                                    int32_t* __restrict__ cadj,
                                                    int32_t* __restrict__ cew) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int c = blockIdx.x;
  const int nw = (nc + 31) >> 5;
  uint32_t* bits = reinterpret_cast<uint32_t*>(smem);
  int32_t* pre = reinterpret_cast<int32_t*>(bits + nw);
  int32_t* red = pre + nw + 1;
  int32_t* acc = red + kT;
  const int a = lead[c], b = match[a];
  const int nm = b == a ? 1 : 2;
  for (int q = threadIdx.x; q < nw; q += kT) bits[q] = 0u;
  __syncthreads();
  for (int i = 0; i < nm; ++i) {
    const int m = i ? b : a;
    for (int e = rp[m] + threadIdx.x; e < rp[m + 1]; e += kT) {
      const int cu = cmap[col[e]];
      if (cu != c) atomicOr(&bits[cu >> 5], 1u << (cu & 31));
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nw; q += kT) pre[q] = __popc(bits[q]);
  __syncthreads();
  const int32_t total = lds_exclusive_scan<kT>(pre, nw, red);
  if (PASS == 0) {
    if (threadIdx.x == 0) cnt[c] = total;
    return;
  }
  for (int r = threadIdx.x; r < total; r += kT) acc[r] = 0;
  __syncthreads();
  for (int i = 0; i < nm; ++i) {
    const int m = i ? b : a;
    for (int e = rp[m] + threadIdx.x; e < rp[m + 1]; e += kT) {
      const int cu = cmap[col[e]];
      if (cu == c) continue;
      const int r = pre[cu >> 5] + __popc(bits[cu >> 5] & ((1u << (cu & 31)) - 1u));
      atomicAdd(&acc[r], w[e]);
    }
  }
  __syncthreads();
  const int32_t base = crp[c];
  for (int q = threadIdx.x; q < nw; q += kT) {
    uint32_t word = bits[q];
    int r = pre[q];
    while (word) {
      const int bt = __ffs(word) - 1;
      cadj[base + r] = (q << 5) + bt;
      cew[base + r] = acc[r];
      ++r;
      word &= word - 1u;
    }
  }
}

// The candidate lists of the first coarse level: as k_top_nb, ordered by (weight, -vertex
// weight, -index) -- key (weight << 32) | ~(vw << 24 | u), vw < 256 and u < 2^24 checked on the
// host -- and only for vertices that can pair (vw + min vw <= cap; the others keep -1).
__global__ __launch_bounds__(kT) void k_top_coarse(int nc, const int32_t* __restrict__ crp,
                                                   const int32_t* __restrict__ cadj,
                                                   const int32_t* __restrict__ cew,
                                                   const int32_t* __restrict__ cvw, int cap,
                                                   int min_vw, int32_t* __restrict__ top) {
  const int lane = threadIdx.x & 63;
  const int v = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
  if (v >= nc) return;  // wave-uniform
  uint64_t best[kMlTop];
#pragma unroll
  for (int i = 0; i < kMlTop; ++i) best[i] = 0;
  if (cvw[v] + min_vw <= cap)
    for (int e = crp[v] + lane; e < crp[v + 1]; e += 64) {
      const int u = cadj[e];
      uint64_t x = ((uint64_t)(uint32_t)cew[e] << 32) |
                   (uint32_t)(~(((uint32_t)cvw[u] << 24) | (uint32_t)u));
      if (x <= best[kMlTop - 1]) continue;
#pragma unroll
      for (int i = 0; i < kMlTop; ++i)
        if (x > best[i]) {
          const uint64_t t = best[i];
          best[i] = x;
          x = t;
        }
    }
  for (int r = 0; r < kMlTop; ++r) {
    uint64_t m = best[0];
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t lo = __shfl_xor((uint32_t)m, off, 64);
      const uint32_t hi = __shfl_xor((uint32_t)(m >> 32), off, 64);
      const uint64_t o = ((uint64_t)hi << 32) | lo;
      m = o > m ? o : m;
    }
    if (m != 0 && best[0] == m) {
#pragma unroll
      for (int i = 0; i + 1 < kMlTop; ++i) best[i] = best[i + 1];
      best[kMlTop - 1] = 0;
    }
    if (lane == 0)
      top[(int64_t)v * kMlTop + r] = m ? (int32_t)(~(uint32_t)m & 0xFFFFFFu) : -1;
  }
}

}  // namespace

void partition_block(const Csr& g, int32_t core_size, Part& P, hipStream_t s, int method) {
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
  if (method == GB_PART_BFS) {
    const int nw = (n + 31) >> 5;
    const size_t lds = (size_t)(nw + 1) * 4 + (size_t)kCand * 8 + 64;
    if (lds > 160 * 1024) fail(GB_EUNSUPPORTED, "bfs order: n = %d too large for one LDS bitmap", n);
    DBuf<int32_t> order(n, s), status(1, s);
    int32_t zero = 0;
    GB_HIP(hipMemcpyAsync(status.get(), &zero, 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_cm_order, dim3(1), dim3(kT), lds, s, n, g.row_ptr.get(), g.col.get(),
                       order.get(), status.get());
    GB_LAUNCH_CHECK();
    int32_t st = 0;
    GB_HIP(hipMemcpyAsync(&st, status.get(), 4, hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    if (st) fail(GB_EUNSUPPORTED, "bfs order: a vertex has %d new neighbours (capacity %d)", st, kCand);
    hipLaunchKernelGGL(k_sort_cores, dim3(n_sub), dim3(64), 0, s, order.get(), P.core_ptr.get(),
                       P.core_vtx.get());
    GB_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL(k_iota, dim3((n + kT - 1) / kT), dim3(kT), 0, s, P.core_vtx.get(), n);
    GB_LAUNCH_CHECK();
  }
  finish_partition(g, P, s);
}

void partition_from_cores(const Csr& g, const std::vector<int32_t>& core_ptr,
                          const std::vector<int32_t>& core_vtx, Part& P, hipStream_t s) {
  const int n = g.n;
  if ((int64_t)core_vtx.size() != n || core_ptr.empty() || core_ptr.back() != n)
    fail(GB_ESHAPE, "core lists do not cover the %d vertices", n);
  P.n = n;
  P.n_sub = (int)core_ptr.size() - 1;
  P.h_core_ptr = core_ptr;
  P.core_ptr = DBuf<int32_t>(P.n_sub + 1, s);
  GB_HIP(hipMemcpyAsync(P.core_ptr.get(), core_ptr.data(), core_ptr.size() * 4,
                        hipMemcpyHostToDevice, s));
  P.core_vtx = DBuf<int32_t>(n, s);
  GB_HIP(hipMemcpyAsync(P.core_vtx.get(), core_vtx.data(), (size_t)n * 4, hipMemcpyHostToDevice,
                        s));
  finish_partition(g, P, s);
}

// A second stream per device for the copies that overlap the weights kernel (created on first
// use with the default priority and kept for the life of the process).
static hipStream_t side_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  GB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t st = nullptr;
  GB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  streams[dev] = st;
  return st;
}

struct SideCopy {  // an event that orders the side stream after the caller's stream
  hipEvent_t ev = nullptr;
  hipStream_t cs = nullptr;
  SideCopy(hipStream_t s) : cs(side_stream()) {
    GB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    GB_HIP(hipEventRecord(ev, s));
    GB_HIP(hipStreamWaitEvent(cs, ev, 0));
  }
  ~SideCopy() {
    (void)hipStreamSynchronize(cs);  // nothing of the copies outlives the call
    (void)hipEventDestroy(ev);
  }
};

// Coarse levels on the device (k_coarse_rows, k_top_coarse): the first from the input graph and
// its weights, each later one from the level built before it (kept on the device); rows and
// lists are copied into the lease's pinned arrays.
class DevCoarse : public MlCoarseDevice {
 public:
  DevCoarse(const Csr& g, const int32_t* dw, MlScratch& sc, hipStream_t s)
      : g_(g), dw_(dw), sc_(sc), s_(s) {}
  bool build(int level, int n, const int32_t* frp, int nc, const std::vector<int32_t>& match,
             const std::vector<int32_t>& cmap, const std::vector<int32_t>& lead,
             const std::vector<int32_t>& cvw, int cap, const int32_t** rp, const int32_t** adj,
             const int32_t** ew, const int32_t** top) override {
    // the fine level: the input graph, or the level built last (its rows still on the device)
    const bool input = level == 0;
    if (input ? n != g_.n : (level != built_ || n != n_built_)) return false;
    if (nc < 1 || nc >= (1 << 24)) return false;
    int min_vw = INT_MAX, max_vw = 0;
    for (int x : cvw) {
      min_vw = std::min(min_vw, x);
      max_vw = std::max(max_vw, x);
    }
    if (max_vw > 255) return false;  // the candidate keys hold 8 bits of vertex weight
    int max_deg = 0;
    for (int v = 0; v < n; ++v) max_deg = std::max(max_deg, frp[v + 1] - frp[v]);
    const int nw = (nc + 31) >> 5;
    const size_t lds0 = ((size_t)2 * nw + 1 + kT) * 4 + 64;
    const size_t lds1 = lds0 + (size_t)2 * max_deg * 4;  // a row: at most both members' degrees
    if (lds1 > 160 * 1024) return false;
    const int32_t* frp_d = input ? g_.row_ptr.get() : rp_.get();
    const int32_t* fadj_d = input ? g_.col.get() : adj_.get();
    const int32_t* few_d = input ? dw_ : ew_.get();
    DBuf<int32_t> dm(n, s_), dc(n, s_), dl(nc, s_), dv(nc, s_), cnt(nc, s_), crp(nc + 1, s_);
    GB_HIP(hipMemcpyAsync(dm.get(), match.data(), (size_t)n * 4, hipMemcpyHostToDevice, s_));
    GB_HIP(hipMemcpyAsync(dc.get(), cmap.data(), (size_t)n * 4, hipMemcpyHostToDevice, s_));
    GB_HIP(hipMemcpyAsync(dl.get(), lead.data(), (size_t)nc * 4, hipMemcpyHostToDevice, s_));
    GB_HIP(hipMemcpyAsync(dv.get(), cvw.data(), (size_t)nc * 4, hipMemcpyHostToDevice, s_));
    hipLaunchKernelGGL(k_coarse_rows<0>, dim3(nc), dim3(kT), lds0, s_, nc, frp_d, fadj_d, few_d,
                       dl.get(), dm.get(), dc.get(), cnt.get(), nullptr, nullptr, nullptr);
    GB_LAUNCH_CHECK();
    exclusive_scan_i32(cnt.get(), crp.get(), nc, s_);
    int32_t nnz = 0;
    GB_HIP(hipMemcpyAsync(&nnz, crp.get() + nc, 4, hipMemcpyDeviceToHost, s_));
    GB_HIP(hipStreamSynchronize(s_));
    DBuf<int32_t> cadj(std::max(nnz, 1), s_), cew(std::max(nnz, 1), s_),
        dtop((size_t)nc * kMlTop, s_);
    hipLaunchKernelGGL(k_coarse_rows<1>, dim3(nc), dim3(kT), lds1, s_, nc, frp_d, fadj_d, few_d,
                       dl.get(), dm.get(), dc.get(), nullptr, crp.get(), cadj.get(), cew.get());
    GB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_top_coarse, dim3((nc + kT / 64 - 1) / (kT / 64)), dim3(kT), 0, s_, nc,
                       crp.get(), cadj.get(), cew.get(), dv.get(), cap, min_vw, dtop.get());
    GB_LAUNCH_CHECK();
    int32_t *hrp, *hadj, *hew, *htop;
    ml_stage1(sc_, nc, nnz, &hrp, &hadj, &hew, &htop);
    GB_HIP(hipMemcpyAsync(hrp, crp.get(), (size_t)(nc + 1) * 4, hipMemcpyDeviceToHost, s_));
    GB_HIP(hipMemcpyAsync(hadj, cadj.get(), (size_t)nnz * 4, hipMemcpyDeviceToHost, s_));
    GB_HIP(hipMemcpyAsync(hew, cew.get(), (size_t)nnz * 4, hipMemcpyDeviceToHost, s_));
    GB_HIP(hipMemcpyAsync(htop, dtop.get(), (size_t)nc * kMlTop * 4, hipMemcpyDeviceToHost, s_));
    GB_HIP(hipStreamSynchronize(s_));
    // the new level becomes the fine level of the next build
    rp_ = std::move(crp);
    adj_ = std::move(cadj);
    ew_ = std::move(cew);
    built_ = level + 1;
    n_built_ = nc;
    *rp = hrp;
    *adj = hadj;
    *ew = hew;
    *top = htop;
    return true;
  }

 private:
  const Csr& g_;
  const int32_t* dw_;
  MlScratch& sc_;
  hipStream_t s_;
  DBuf<int32_t> rp_, adj_, ew_;  // the level built last
  int built_ = -1, n_built_ = 0;
};

void partition_multilevel_dev(const Csr& g, int32_t core_size, Part& P, hipStream_t s,
                              MlStats* stats, const Part* prev) {
  const int n = g.n;
  std::vector<int32_t> cp, cv;
  MlLease lease;  // pinned staging and coarse levels kept from earlier calls
  int32_t *rp, *col, *w;
  if (prev) {
    // on-the-fly update: the previous cores carried to this graph (no weights needed)
    if (prev->n != n) fail(GB_ESHAPE, "previous partition has %d vertices, graph %d", prev->n, n);
    ml_stage(*lease.p, n, g.nnz, &rp, &col, nullptr);
    std::vector<int32_t> pv(n);
    GB_HIP(hipMemcpyAsync(rp, g.row_ptr.get(), (n + 1) * 4, hipMemcpyDeviceToHost, s));
    GB_HIP(hipMemcpyAsync(col, g.col.get(), g.nnz * 4, hipMemcpyDeviceToHost, s));
    GB_HIP(hipMemcpyAsync(pv.data(), prev->core_vtx.get(), (size_t)n * 4, hipMemcpyDeviceToHost,
                          s));
    GB_HIP(hipStreamSynchronize(s));
    partition_update(n, rp, col, prev->h_core_ptr, pv, cp, cv, stats);
    partition_from_cores(g, cp, cv, P, s);
    return;
  }
  // edge weights on the device (the graphs built here hold every self loop), the rest on the
  // host
  ml_stage(*lease.p, n, g.nnz, &rp, &col, &w);
  const size_t lds = (size_t)((n + 31) >> 5) * 4;
  if (lds > 160 * 1024) fail(GB_EUNSUPPORTED, "multilevel: n = %d too large for one LDS bitmap", n);
  DBuf<int32_t> dw(std::max<int64_t>(g.nnz, 1), s), dmiss(1, s);
  // the graph itself goes to the host on the side stream while the weights are computed
  SideCopy side(s);
  GB_HIP(hipMemcpyAsync(rp, g.row_ptr.get(), (n + 1) * 4, hipMemcpyDeviceToHost, side.cs));
  GB_HIP(hipMemcpyAsync(col, g.col.get(), g.nnz * 4, hipMemcpyDeviceToHost, side.cs));
  int32_t miss = n;  // no vertex lacks its self loop
  GB_HIP(hipMemcpyAsync(dmiss.get(), &miss, 4, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_common_nb, dim3(n), dim3(kT), lds, s, n, g.row_ptr.get(), g.col.get(),
                     dw.get(), dmiss.get());
  GB_LAUNCH_CHECK();
  DBuf<int32_t> dtop((size_t)n * kMlTop, s);
  hipLaunchKernelGGL(k_top_nb, dim3((n + kT / 64 - 1) / (kT / 64)), dim3(kT), 0, s, n,
                     g.row_ptr.get(), g.col.get(), dw.get(), dtop.get());
  GB_LAUNCH_CHECK();
  int32_t* top = ml_top_buffer(*lease.p, n);  // read by the matching of the input level
  GB_HIP(hipMemcpyAsync(w, dw.get(), g.nnz * 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipMemcpyAsync(top, dtop.get(), (size_t)n * kMlTop * 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipMemcpyAsync(&miss, dmiss.get(), 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(side.cs));
  GB_HIP(hipStreamSynchronize(s));
  if (miss < n) fail(GB_EINVAL, "multilevel: vertex %d has no self loop", miss);
  DevCoarse dev1(g, dw.get(), *lease.p, s);
  partition_multilevel(n, rp, col, core_size, cp, cv, stats, w, lease.p, top, &dev1);
  partition_from_cores(g, cp, cv, P, s);
}

// halos, subgraph lists and index maps for the cores in P.core_ptr / P.core_vtx (each core's
// vertices ascending)
void finish_partition(const Csr& g, Part& P, hipStream_t s) {
  const int n = g.n;
  const int n_sub = P.n_sub;
  const int nw = (n + 31) >> 5;
  const bool hash = use_hash_sets(n);
  const size_t lds = (size_t)nw * 8 + kT * 4 + 64;
  if (!hash && lds > 160 * 1024)
    fail(GB_EUNSUPPORTED, "partition: n = %d too large for one LDS bitmap", n);
  // hash sets: the union of the core's rows, capacity raised to what a core reports (cap + kT
  // + 1 slots keep inserts that pass cap from filling the set)
  int cap = 4096, log2h = 0, log2u = 0;
  size_t lds_h = 0;
  DBuf<int32_t> ovf(1, s);
  auto sizes = [&] {
    log2h = ceil_log2((int64_t)cap + kT + 1);
    log2u = ceil_log2(cap);
    lds_h = (((size_t)1 << log2h) + ((size_t)1 << log2u)) * 4 + 64;
    if (lds_h > 160 * 1024)
      fail(GB_EUNSUPPORTED, "partition: a core has about %d neighbours, more than LDS holds", cap);
  };
  DBuf<int32_t> cnt(n_sub, s);
  if (hash) {
    for (int attempt = 0;; ++attempt) {
      sizes();
      int32_t h = 0;
      hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, s, ovf.get());
      hipLaunchKernelGGL(k_halo_hash<0>, dim3(n_sub), dim3(kT), lds_h, s, n, g.row_ptr.get(),
                         g.col.get(), P.core_ptr.get(), P.core_vtx.get(), cap, log2h, log2u,
                         cnt.get(), nullptr, nullptr, ovf.get());
      GB_LAUNCH_CHECK();
      GB_HIP(hipMemcpyAsync(&h, ovf.get(), 4, hipMemcpyDeviceToHost, s));
      GB_HIP(hipStreamSynchronize(s));
      if (h == 0) break;
      if (attempt == 2) fail(GB_EUNSUPPORTED, "partition: neighbour count did not settle");
      cap = std::max(((h + 255) / 256) * 256, 2 * cap);
    }
  } else {
    hipLaunchKernelGGL(k_halo<0>, dim3(n_sub), dim3(kT), lds, s, n, g.row_ptr.get(), g.col.get(),
                       P.core_ptr.get(), P.core_vtx.get(), cnt.get(), nullptr, nullptr);
  }
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
  if (hash)
    hipLaunchKernelGGL(k_halo_hash<1>, dim3(n_sub), dim3(kT), lds_h, s, n, g.row_ptr.get(),
                       g.col.get(), P.core_ptr.get(), P.core_vtx.get(), cap, log2h, log2u,
                       nullptr, P.sub_ptr.get(), P.sub_idx.get(), ovf.get());
  else
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
