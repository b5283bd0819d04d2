// Spectral bounds, the SP2 start map X0, and the data-dependency graphs (Eq. 2, Eq. 8,
// obs. viii).  Every floating-point result that decides an integer (a graph edge) is
// evaluated in a canonical order with separately rounded operations, so the graph is the
// same bit for bit as a sequential CPU evaluation: Gershgorin row sums in ascending column
// order, x0 = (e_max*delta_ij - h_ij)/(e_max - e_min), and (X0^2)_ij accumulated over k in
// ascending order.  The library is compiled with floating-point contraction disabled.
#include "internal.h"
#include "lds_hash.h"
#include "lds_scan.h"

#include <cstdlib>
#include <map>
#include <string>
#include <mutex>

#pragma clang fp contract(off)

namespace gbi {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ double x0_entry(double h, bool diag, double emax, double denom) {
  const double num = diag ? (emax - h) : (0.0 - h);
  return num / denom;
}

// One thread per row: Gershgorin ends lo_i = h_ii - R_i, hi_i = h_ii + R_i, with
// R_i = sum_{j != i} |h_ij| accumulated in slot (ascending column) order.
__global__ void k_row_discs(const int32_t* __restrict__ col, const double* __restrict__ val, int n,
                            int w, double* __restrict__ lo, double* __restrict__ hi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t* c = col + (int64_t)i * w;
  const double* v = val + (int64_t)i * w;
  double r = 0.0, d = 0.0;
  for (int t = 0; t < w; ++t) {
    const int32_t j = c[t];
    if (j < 0) break;
    if (j == i) d = v[t];
    else r = r + fabs(v[t]);
  }
  lo[i] = d - r;
  hi[i] = d + r;
}

// min of lo, max of hi over n rows (exact, order-free); one block.  out[2] counts the rows
// whose ends are not finite (a NaN or Inf anywhere in the row makes them so; fmin / fmax would
// silently skip a NaN).
__global__ void k_minmax(const double* __restrict__ lo, const double* __restrict__ hi, int n,
                         double* __restrict__ out) {
  __shared__ double smin[kT], smax[kT], sbad[kT];
  double a = INFINITY, b = -INFINITY, bad = 0.0;
  for (int i = threadIdx.x; i < n; i += kT) {
    const double l = lo[i], h = hi[i];
    if (!isfinite(l) || !isfinite(h)) bad += 1.0;
    a = fmin(a, l);
    b = fmax(b, h);
  }
  smin[threadIdx.x] = a;
  smax[threadIdx.x] = b;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      sbad[threadIdx.x] += sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smin[0];
    out[1] = smax[0];
    out[2] = sbad[0];
  }
}

// ---- spectral bounds without allocated memory ----------------------------------------------
// The same row ends as k_row_discs, reduced per workgroup (rows grid-strided over at most
// kNoallocBlocks workgroups) into (min lo, max hi, non-finite rows) partials, then by one
// workgroup into the final triple; min and max are exact, so the bounds equal k_minmax's bit for
// bit.  Partials and result live in `scratch`, a fixed device array: each workgroup writes its
// own three entries before the final pass reads them, so nothing has to start at zero.
constexpr int kNoallocBlocks = 1024;
static __device__ __align__(256) double scratch[3 * kNoallocBlocks + 3];

__device__ __forceinline__ void reduce3(double& a, double& b, double& c, double* sa, double* sb,
                                        double* sc) {
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int h = kT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      sa[threadIdx.x] = fmin(sa[threadIdx.x], sa[threadIdx.x + h]);
      sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + h]);
      sc[threadIdx.x] += sc[threadIdx.x + h];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
  c = sc[0];
}

__global__ __launch_bounds__(kT) void k_disc_partials(const int32_t* __restrict__ col,
                                                      const double* __restrict__ val, int n, int w,
                                                      double* __restrict__ part) {
  __shared__ double sa[kT], sb[kT], sc[kT];
  double a = INFINITY, b = -INFINITY, bad = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const int32_t* c = col + i * w;
    const double* v = val + i * w;
    double r = 0.0, d = 0.0;
    for (int t = 0; t < w; ++t) {
      const int32_t j = c[t];
      if (j < 0) break;
      if (j == i) d = v[t];
      else r = r + fabs(v[t]);
    }
    const double lo = d - r, hi = d + r;
    if (!isfinite(lo) || !isfinite(hi)) bad += 1.0;
    a = fmin(a, lo);
    b = fmax(b, hi);
  }
  reduce3(a, b, bad, sa, sb, sc);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = a;
    part[3 * blockIdx.x + 1] = b;
    part[3 * blockIdx.x + 2] = bad;
  }
}

__global__ __launch_bounds__(kT) void k_disc_final(const double* __restrict__ part, int nb,
                                                   double* __restrict__ out) {
  __shared__ double sa[kT], sb[kT], sc[kT];
  double a = INFINITY, b = -INFINITY, bad = 0.0;
  for (int q = threadIdx.x; q < nb; q += kT) {
    a = fmin(a, part[3 * q]);
    b = fmax(b, part[3 * q + 1]);
    bad += part[3 * q + 2];
  }
  reduce3(a, b, bad, sa, sb, sc);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
    out[2] = bad;
  }
}

__global__ void k_x0(const int32_t* __restrict__ col, const double* __restrict__ val, int n, int w,
                     double emax, double denom, double* __restrict__ x0) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)n * w) return;
  const int i = (int)(p / w);
  const int32_t j = col[p];
  x0[p] = j < 0 ? 0.0 : x0_entry(val[p], j == i, emax, denom);
}

// ---- X2 graph, one workgroup per row i --------------------------------------------------
// The edge (i, j) is decided by |(X0^2)_ij| >= tau, the entry summed over k in row i in
// ascending order (row i's slots in order), every product and sum rounded separately.  The
// kernels accumulate the entries with LDS atomic adds instead, in whatever order the adds
// land, with no barrier between the rows k, and keep that order's result only where it cannot
// change the decision: two summation orders of the same m rounded products p_k differ by at
// most 2 gamma_{m-1} sum |p_k| (gamma_m = m u / (1 - m u), u = 2^-53; the standard bound on
// recursive summation), and sum_k |x0_ik x0_kj| <= b_i = sum_k |x0_ik| max_l |x0_kl|.  A
// candidate with | |acc| - tau | within twice that of tau (at most a few per graph, usually
// none) is summed again in ascending order by one wave, so the graph is the one of the
// ascending sums bit for bit.
//   1. mark every j in row k for every k in row i (two-hop candidates) and i itself;
//   2. rank = number of candidates below j (per-word popcount prefix);
//   3. acc[rank(j)] += x0_ik * x0_kj over every (k, j), LDS atomic adds;
//   4. keep j if j == i or |acc| >= tau (re-summed in ascending order near tau): the count,
//      and the sorted columns into the row's slot of a staging array (cap entries per row;
//      k_x2_compact then packs them into the CSR), so the product is computed once.
// LDS: candidate bitmap over all n vertices, per-word rank base, accumulators of the
// candidates (indexed by rank), and row i's columns / x0 values.
struct X2Lds {
  uint32_t* bits;
  int32_t* pre;
  double* acc;
  int32_t* ci;
  double* xi;
};

constexpr int kX2Q = 4;  // ELL width limit: kX2Q * kT (the float index split below needs < 2048)
constexpr int kX2B = 8;  // (k, j) pairs whose loads a thread has in flight at once

// the (slot t of row i, slot u of row k) pair number p = t w + u, split without an integer
// division: (p + 0.5) / w is at least 0.5 / w away from an integer and p < w^2 < 2^22, so the
// float quotient truncates to t (the correction below is a guard)
__device__ __forceinline__ void x2_pair(int p, int w, float inv_w, int& t, int& u) {
  t = (int)(((float)p + 0.5f) * inv_w);
  u = p - t * w;
  if (u < 0) {
    --t;
    u += w;
  } else if (u >= w) {
    ++t;
    u -= w;
  }
}

// the rows k of row i are its slots before the first padding entry
__device__ __forceinline__ int x2_row_width(const int32_t* ci, int w, int n, int32_t* red) {
  if (threadIdx.x == 0) red[0] = w;
  __syncthreads();
  for (int t = threadIdx.x; t < w; t += kT)
    if ((unsigned)ci[t] >= (unsigned)n) atomicMin(&red[0], t);
  __syncthreads();
  const int kw = red[0];
  __syncthreads();  // red is reused
  return kw;
}

// step 1 and step 3 over the kw * w pairs: mark(j), or add(j, x0_ik * x0_kj)
template <bool ADD, class F>
__device__ __forceinline__ void x2_pairs(const int32_t* __restrict__ hcol,
                                         const double* __restrict__ x0, const int32_t* ci,
                                         const double* xi, int kw, int w, float inv_w, int n,
                                         F&& f) {
  const int npair = kw * w;
  for (int p0 = threadIdx.x; p0 < npair; p0 += kX2B * kT) {
    int32_t jj[kX2B];
    double xk[kX2B], xx[kX2B];  // x0_ik, x0_kj
#pragma unroll
    for (int q = 0; q < kX2B; ++q) {  // every load of the batch first
      const int p = p0 + q * kT;
      jj[q] = -1;
      xk[q] = xx[q] = 0.0;
      if (p < npair) {
        int t, u;
        x2_pair(p, w, inv_w, t, u);
        const int64_t e = (int64_t)ci[t] * w + u;
        jj[q] = hcol[e];
        if (ADD) {
          xx[q] = x0[e];
          xk[q] = xi[t];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kX2B; ++q)
      if ((unsigned)jj[q] < (unsigned)n) f(jj[q], ADD ? xk[q] * xx[q] : 0.0);
  }
}

// the half-width of the band around tau in which the order of the sum may decide (see above):
// twice the bound, b_i rounded, a term for underflow
__device__ __forceinline__ double x2_margin(int kw, double b, double tau) {
  return (4.0 * kw + 8.0) * 0x1p-53 * b + 4.0 * 0x1p-53 * tau + 1e-300;
}

// (X0^2)_ij summed in ascending order of row i's slots, every product and sum rounded
// separately, by a whole wave: lane l looks j up in the rows k of slots l, l + 64, ... (a scan
// of the row, which assumes nothing of its order) and the products are added one slot after
// the other.
__device__ double x2_sum_ascending(const int32_t* __restrict__ hcol,
                                   const double* __restrict__ x0, const int32_t* ci,
                                   const double* xi, int kw, int w, int32_t j) {
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  for (int t0 = 0; t0 < kw; t0 += 64) {
    const int t = t0 + lane;
    double prod = 0.0;
    int found = 0;
    if (t < kw) {
      const int64_t base = (int64_t)ci[t] * w;
      for (int u = 0; u < w; ++u)
        if (hcol[base + u] == j) {
          found = 1;
          prod = xi[t] * x0[base + u];
          break;
        }
    }
    const int m = min(64, kw - t0);
    for (int l = 0; l < m; ++l)
      if (__shfl(found, l)) acc = acc + __shfl(prod, l);
  }
  return acc;
}

__global__ __launch_bounds__(kT) void k_x2_rows(const int32_t* __restrict__ hcol,
                                                const double* __restrict__ x0,
                                                const double* __restrict__ rbound, int n, int w,
                                                float inv_w, double tau, int all_ascending,
                                                int cap, int32_t* __restrict__ cnt,
                                                int32_t* __restrict__ rows,
                                                int32_t* __restrict__ overflow) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t nband;
  const int i = blockIdx.x;
  const int nw = (n + 31) >> 5;
  X2Lds L;
  L.acc = reinterpret_cast<double*>(smem);
  L.xi = L.acc + cap;
  L.bits = reinterpret_cast<uint32_t*>(L.xi + w);
  L.pre = reinterpret_cast<int32_t*>(L.bits + nw);
  L.ci = L.pre + nw + 1;
  int32_t* red = L.ci + w;  // kT ints

  for (int t = threadIdx.x; t < w; t += kT) {
    L.ci[t] = hcol[(int64_t)i * w + t];
    L.xi[t] = x0[(int64_t)i * w + t];
  }
  for (int q = threadIdx.x; q < nw; q += kT) L.bits[q] = 0u;
  if (threadIdx.x == 0) nband = 0;
  const int kw = x2_row_width(L.ci, w, n, red);
  // 1. two-hop candidates
  x2_pairs<false>(hcol, x0, L.ci, L.xi, kw, w, inv_w, n, [&](int32_t j, double) {
    atomicOr(&L.bits[j >> 5], 1u << (j & 31));
  });
  if (threadIdx.x == 0) atomicOr(&L.bits[i >> 5], 1u << (i & 31));
  __syncthreads();
  // 2. ranks
  for (int q = threadIdx.x; q < nw; q += kT) L.pre[q] = __popc(L.bits[q]);
  __syncthreads();
  const int32_t ncand = lds_exclusive_scan<kT>(L.pre, nw, red);
  if (ncand > cap) {
    if (threadIdx.x == 0) {
      atomicMax(overflow, ncand);
      cnt[i] = 0;
    }
    return;
  }
  for (int r = threadIdx.x; r < ncand; r += kT) L.acc[r] = 0.0;
  __syncthreads();
  // 3. accumulation, adds in any order
  x2_pairs<true>(hcol, x0, L.ci, L.xi, kw, w, inv_w, n, [&](int32_t j, double prod) {
    const uint32_t word = L.bits[j >> 5];
    const int r = L.pre[j >> 5] + __popc(word & ((1u << (j & 31)) - 1u));
    atomicAdd(&L.acc[r], prod);
  });
  __syncthreads();
  // 4. decisions: bits[q] becomes the word's kept set, pre[q] (no longer needed for ranks)
  //    its candidates near tau, then its kept count
  const double margin = x2_margin(kw, rbound[i], tau);
  for (int q = threadIdx.x; q < nw; q += kT) {
    uint32_t word = L.bits[q], keep = 0u, band = 0u;
    int r = L.pre[q];
    while (word) {
      const int b = __ffs(word) - 1;
      const int j = (q << 5) + b;
      const double a = fabs(L.acc[r]);
      if (j == i) keep |= 1u << b;
      else if (all_ascending || fabs(a - tau) <= margin) band |= 1u << b;
      else if (a >= tau) keep |= 1u << b;
      ++r;
      word &= word - 1u;
    }
    L.bits[q] = keep;
    L.pre[q] = (int32_t)band;
    if (band) atomicAdd(&nband, __popc(band));
  }
  __syncthreads();
  if (nband > 0) {
    // ascending sums of the candidates near tau, one wave per word
    for (int q = threadIdx.x >> 6; q < nw; q += kT / 64) {
      uint32_t band = (uint32_t)L.pre[q];
      while (band) {
        const int b = __ffs(band) - 1;
        const double a = fabs(x2_sum_ascending(hcol, x0, L.ci, L.xi, kw, w, (q << 5) + b));
        if ((threadIdx.x & 63) == 0 && a >= tau) atomicOr(&L.bits[q], 1u << b);
        band &= band - 1u;
      }
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < nw; q += kT) L.pre[q] = __popc(L.bits[q]);
  __syncthreads();
  const int32_t kept = lds_exclusive_scan<kT>(L.pre, nw, red);
  if (threadIdx.x == 0) cnt[i] = kept;
  int32_t* dst = rows + (int64_t)i * cap;  // kept <= ncand <= cap
  for (int q = threadIdx.x; q < nw; q += kT) {
    uint32_t word = L.bits[q];
    int32_t pos = L.pre[q];
    while (word) {
      const int b = __ffs(word) - 1;
      dst[pos++] = (q << 5) + b;
      word &= word - 1u;
    }
  }
}

// max_l |x0_kl| of every row k (one wave per row)
__global__ __launch_bounds__(kT) void k_row_absmax(const double* __restrict__ x0, int n, int w,
                                                   double* __restrict__ out) {
  const int row = blockIdx.x * (kT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  double m = 0.0;
  for (int u = lane; u < w; u += 64) m = fmax(m, fabs(x0[(int64_t)row * w + u]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane == 0) out[row] = m;
}

// b_i = sum over the slots of row i of |x0_ik| max_l |x0_kl|, which bounds sum_k |x0_ik x0_kj|
// for every j (one wave per row)
__global__ __launch_bounds__(kT) void k_x2_bound(const int32_t* __restrict__ col,
                                                 const double* __restrict__ x0,
                                                 const double* __restrict__ amax, int n, int w,
                                                 double* __restrict__ out) {
  const int row = blockIdx.x * (kT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  double b = 0.0;
  for (int u = lane; u < w; u += 64) {
    const int64_t e = (int64_t)row * w + u;
    const int32_t k = col[e];
    if ((unsigned)k < (unsigned)n) b += fabs(x0[e]) * amax[k];
  }
  for (int o = 32; o > 0; o >>= 1) b += __shfl_xor(b, o);
  if (lane == 0) out[row] = b;
}

// The same rows for any n: the two-hop candidates of row i go into an LDS hash set instead of
// an n-bit bitmap and are sorted to fix their ranks; accumulation and decisions are those of
// k_x2_rows, so the graph is the same bit for bit.  LDS: acc [cap], x0 of row i [w], keys and
// their ranks [2^log2h each], the sorted candidates [2^log2u >= cap], columns of row i [w],
// scratch [kT].  Inserts stop once more than cap candidates were counted (at most kT more
// land, and 2^log2h >= cap + kT + 1 keeps the set from filling); such a row reports its count
// through `overflow`.
__global__ __launch_bounds__(kT) void k_x2_rows_hash(const int32_t* __restrict__ hcol,
                                                     const double* __restrict__ x0,
                                                     const double* __restrict__ rbound, int n,
                                                     int w, float inv_w, double tau,
                                                     int all_ascending, int cap, int log2h,
                                                     int log2u, int32_t* __restrict__ cnt,
                                                     int32_t* __restrict__ rows,
                                                     int32_t* __restrict__ overflow) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t count, gathered, nband;
  const int i = blockIdx.x;
  const int H = 1 << log2h, P = 1 << log2u;
  double* acc = reinterpret_cast<double*>(smem);
  double* xi = acc + cap;
  int32_t* keys = reinterpret_cast<int32_t*>(xi + w);
  int32_t* rk = keys + H;
  int32_t* U = rk + H;
  int32_t* ci = U + P;
  int32_t* red = ci + w;
  for (int t = threadIdx.x; t < w; t += kT) {
    ci[t] = hcol[(int64_t)i * w + t];
    xi[t] = x0[(int64_t)i * w + t];
  }
  for (int q = threadIdx.x; q < H; q += kT) keys[q] = kHashEmpty;
  if (threadIdx.x == 0) {
    count = 0;
    gathered = 0;
    nband = 0;
  }
  const int kw = x2_row_width(ci, w, n, red);
  // 1. two-hop candidates (and i itself)
  if (threadIdx.x == 0 && hset_insert(keys, log2h, i)) atomicAdd(&count, 1);
  x2_pairs<false>(hcol, x0, ci, xi, kw, w, inv_w, n, [&](int32_t j, double) {
    if (*(volatile int32_t*)&count <= cap && hset_insert(keys, log2h, j)) atomicAdd(&count, 1);
  });
  __syncthreads();
  const int ncand = count;
  if (ncand > cap) {
    if (threadIdx.x == 0) {
      atomicMax(overflow, ncand);
      cnt[i] = 0;
    }
    return;
  }
  // 2. ranks: the candidates sorted ascending
  for (int q = threadIdx.x; q < H; q += kT) {
    const int32_t k = keys[q];
    if (k != kHashEmpty) U[atomicAdd(&gathered, 1)] = k;
  }
  __syncthreads();
  for (int r = ncand + threadIdx.x; r < P; r += kT) U[r] = INT32_MAX;
  bitonic_sort<kT>(U, P);
  for (int r = threadIdx.x; r < ncand; r += kT) {
    rk[hset_find(keys, log2h, U[r])] = r;
    acc[r] = 0.0;
  }
  __syncthreads();
  // 3. accumulation, adds in any order
  x2_pairs<true>(hcol, x0, ci, xi, kw, w, inv_w, n, [&](int32_t j, double prod) {
    atomicAdd(&acc[rk[hset_find(keys, log2h, j)]], prod);
  });
  __syncthreads();
  // 4. decisions (rk reused: 1 kept, 0 dropped, 2 near tau), ascending sums near tau, ordered
  //    compaction
  const double margin = x2_margin(kw, rbound[i], tau);
  for (int r = threadIdx.x; r < ncand; r += kT) {
    const double a = fabs(acc[r]);
    int f;
    if (U[r] == i) f = 1;
    else if (all_ascending || fabs(a - tau) <= margin) f = 2;
    else f = a >= tau ? 1 : 0;
    rk[r] = f;
    if (f == 2) atomicAdd(&nband, 1);
  }
  __syncthreads();
  if (nband > 0) {
    for (int r = threadIdx.x >> 6; r < ncand; r += kT / 64) {
      if (rk[r] != 2) continue;  // uniform over the wave
      const double a = fabs(x2_sum_ascending(hcol, x0, ci, xi, kw, w, U[r]));
      if ((threadIdx.x & 63) == 0) rk[r] = a >= tau ? 1 : 0;
    }
    __syncthreads();
  }
  for (int r = threadIdx.x; r < ncand; r += kT) acc[r] = rk[r];  // the flags, for the writes
  __syncthreads();
  const int32_t kept = lds_exclusive_scan<kT>(rk, ncand, red);
  if (threadIdx.x == 0) cnt[i] = kept;
  int32_t* dst = rows + (int64_t)i * cap;
  for (int r = threadIdx.x; r < ncand; r += kT)
    if (acc[r] != 0.0) dst[rk[r]] = U[r];
}

size_t x2_hash_lds_bytes(int w, int cap, int log2h, int log2u) {
  return (size_t)cap * 8 + (size_t)w * 8 + ((size_t)2 << log2h) * 4 + ((size_t)1 << log2u) * 4 +
         (size_t)w * 4 + (size_t)kT * 4 + 64;
}

// row i of the staging array (cnt[i] columns at i * cap) -> the CSR at row_ptr[i]
__global__ __launch_bounds__(kT) void k_x2_compact(const int32_t* __restrict__ rows, int cap,
                                                   const int32_t* __restrict__ cnt,
                                                   const int32_t* __restrict__ row_ptr,
                                                   int32_t* __restrict__ out_col) {
  const int i = blockIdx.x;
  const int32_t* src = rows + (int64_t)i * cap;
  int32_t* dst = out_col + row_ptr[i];
  for (int t = threadIdx.x; t < cnt[i]; t += kT) dst[t] = src[t];
}

size_t x2_lds_bytes(int n, int w, int cap) {
  const int nw = (n + 31) >> 5;
  return (size_t)cap * 8 + (size_t)w * 8 + (size_t)nw * 4 + (size_t)(nw + 1) * 4 + (size_t)w * 4 +
         (size_t)kT * 4 + 64;
}

// ---- row unions through an LDS bitmap (pattern graphs, symmetrisation) --------------------
// Row i of the result = (row i of up to two CSR inputs) U {i}, sorted and unique.
template <int PASS>
__global__ __launch_bounds__(kT) void k_union_rows(int n, const int32_t* __restrict__ rp0,
                                                   const int32_t* __restrict__ c0,
                                                   const int32_t* __restrict__ rp1,
                                                   const int32_t* __restrict__ c1,
                                                   int32_t* __restrict__ cnt,
                                                   const int32_t* __restrict__ row_ptr,
                                                   int32_t* __restrict__ out_col) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int i = blockIdx.x;
  const int nw = (n + 31) >> 5;
  uint32_t* bits = reinterpret_cast<uint32_t*>(smem);
  int32_t* wc = reinterpret_cast<int32_t*>(bits + nw);
  int32_t* red = wc + nw;
  for (int q = threadIdx.x; q < nw; q += kT) bits[q] = 0u;
  __syncthreads();
  for (int p = rp0[i] + threadIdx.x; p < rp0[i + 1]; p += kT) {
    const int j = c0[p];
    atomicOr(&bits[j >> 5], 1u << (j & 31));
  }
  if (rp1)
    for (int p = rp1[i] + threadIdx.x; p < rp1[i + 1]; p += kT) {
      const int j = c1[p];
      atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
  if (threadIdx.x == 0) atomicOr(&bits[i >> 5], 1u << (i & 31));
  __syncthreads();
  for (int q = threadIdx.x; q < nw; q += kT) wc[q] = __popc(bits[q]);
  __syncthreads();
  const int32_t tot = lds_exclusive_scan<kT>(wc, nw, red);
  if (PASS == 0) {
    if (threadIdx.x == 0) cnt[i] = tot;
    return;
  }
  const int32_t base = row_ptr[i];
  for (int q = threadIdx.x; q < nw; q += kT) {
    uint32_t word = bits[q];
    int32_t pos = base + wc[q];
    while (word) {
      const int b = __ffs(word) - 1;
      out_col[pos++] = (q << 5) + b;
      word &= word - 1u;
    }
  }
}


// two-hop closure: row i of the result = union over k in row i of P of row k of P (paths of
// length two; P contains every self-loop, so one-hop edges are included), sorted, unique
template <int PASS>
__global__ __launch_bounds__(kT) void k_twohop_rows(int n, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ c,
                                                    int32_t* __restrict__ cnt,
                                                    const int32_t* __restrict__ row_ptr,
                                                    int32_t* __restrict__ out_col) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int i = blockIdx.x;
  const int nw = (n + 31) >> 5;
  uint32_t* bits = reinterpret_cast<uint32_t*>(smem);
  int32_t* wc = reinterpret_cast<int32_t*>(bits + nw);
  int32_t* red = wc + nw;
  for (int q = threadIdx.x; q < nw; q += kT) bits[q] = 0u;
  __syncthreads();
  for (int a = rp[i]; a < rp[i + 1]; ++a) {
    const int k = c[a];
    for (int p = rp[k] + threadIdx.x; p < rp[k + 1]; p += kT) {
      const int j = c[p];
      atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
  }
  if (threadIdx.x == 0) atomicOr(&bits[i >> 5], 1u << (i & 31));
  __syncthreads();
  for (int q = threadIdx.x; q < nw; q += kT) wc[q] = __popc(bits[q]);
  __syncthreads();
  const int32_t tot = lds_exclusive_scan<kT>(wc, nw, red);
  if (PASS == 0) {
    if (threadIdx.x == 0) cnt[i] = tot;
    return;
  }
  const int32_t base = row_ptr[i];
  for (int q = threadIdx.x; q < nw; q += kT) {
    uint32_t word = bits[q];
    int32_t pos = base + wc[q];
    while (word) {
      const int b = __ffs(word) - 1;
      out_col[pos++] = (q << 5) + b;
      word &= word - 1u;
    }
  }
}

// entries of an ELL matrix with |a| >= tau, as (row-list) CSR counts / fill (rows unsorted
// only if the ELL rows are; ELL rows are ascending so the output rows are ascending)
template <int PASS>
__global__ void k_ell_threshold(const int32_t* __restrict__ col, const double* __restrict__ val,
                                int n, int w, double tau, int32_t* __restrict__ cnt,
                                const int32_t* __restrict__ row_ptr, int32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c = 0;
  int32_t pos = PASS ? row_ptr[i] : 0;
  for (int t = 0; t < w; ++t) {
    const int32_t j = col[(int64_t)i * w + t];
    if (j < 0) break;
    if ((unsigned)j >= (unsigned)n) continue;
    if (fabs(val[(int64_t)i * w + t]) >= tau) {
      if (PASS) out[pos++] = j;
      ++c;
    }
  }
  if (!PASS) cnt[i] = c;
}

// transpose of a CSR pattern: count per column, then fill (order within a row arbitrary)
__global__ void k_tr_count(const int32_t* __restrict__ rp, const int32_t* __restrict__ c, int n,
                           int32_t* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int p = rp[i]; p < rp[i + 1]; ++p) atomicAdd(&cnt[c[p]], 1);
}
__global__ void k_tr_fill(const int32_t* __restrict__ rp, const int32_t* __restrict__ c, int n,
                          const int32_t* __restrict__ trp, int32_t* __restrict__ fill,
                          int32_t* __restrict__ tc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    const int j = c[p];
    tc[trp[j] + atomicAdd(&fill[j], 1)] = i;
  }
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---- RCUT graph (divide-and-conquer comparison): sites within r_cut, periodic cube ----------
// Site a's neighbours b (ascending, a itself included) with the canonical minimum-image squared
// distance below rc2.  PASS 0 counts per site; PASS 1 writes the orbital rows of site a in
// ascending column order (a block-wide scan over each 256-site window keeps the order).
template <int PASS>
__global__ __launch_bounds__(kT) void k_rcut_rows(const double* __restrict__ pos, int n_sites,
                                                  int m, double box, double rc2,
                                                  int32_t* __restrict__ cnt,
                                                  const int32_t* __restrict__ row_ptr,
                                                  int32_t* __restrict__ col) {
  __shared__ int32_t scan[kT];
  __shared__ int32_t base;
  const int a = blockIdx.x;
  const double xa = pos[3 * a], ya = pos[3 * a + 1], za = pos[3 * a + 2];
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int b0 = 0; b0 < n_sites; b0 += kT) {
    const int b = b0 + threadIdx.x;
    int hit = 0;
    if (b < n_sites) {
      double dx = pos[3 * b] - xa, dy = pos[3 * b + 1] - ya, dz = pos[3 * b + 2] - za;
      dx = dx - box * rint(dx / box);
      dy = dy - box * rint(dy / box);
      dz = dz - box * rint(dz / box);
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      hit = r2 < rc2 ? 1 : 0;
    }
    scan[threadIdx.x] = hit;
    __syncthreads();
    for (int h = 1; h < kT; h <<= 1) {  // inclusive scan (Hillis-Steele)
      const int v = threadIdx.x >= h ? scan[threadIdx.x - h] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (PASS == 1 && hit) {
      const int rank = base + scan[threadIdx.x] - 1;  // neighbour index of b in site a's list
      for (int o = 0; o < m; ++o) {
        int32_t* out = col + row_ptr[a * m + o];
        for (int q = 0; q < m; ++q) out[rank * m + q] = b * m + q;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) base += scan[kT - 1];
    __syncthreads();
  }
  if (PASS == 0 && threadIdx.x == 0)
    for (int o = 0; o < m; ++o) cnt[a * m + o] = base * m;
}

int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

void check_lds(size_t bytes, const char* what) {
  if (bytes > 160 * 1024)
    fail(GB_EUNSUPPORTED, "%s needs %zu bytes of LDS per workgroup (limit 163840)", what, bytes);
}

// union of one or two CSRs plus self-loops -> out (sorted rows)
void union_rows(int n, const int32_t* rp0, const int32_t* c0, const int32_t* rp1,
                const int32_t* c1, Csr& out, hipStream_t s) {
  const int nw = (n + 31) >> 5;
  const size_t lds = (size_t)nw * 8 + kT * 4 + 64;
  check_lds(lds, "graph row union");
  DBuf<int32_t> cnt(n, s);
  out.n = n;
  out.row_ptr = DBuf<int32_t>(n + 1, s);
  hipLaunchKernelGGL(k_union_rows<0>, dim3(n), dim3(kT), lds, s, n, rp0, c0, rp1, c1, cnt.get(),
                     nullptr, nullptr);
  GB_LAUNCH_CHECK();
  exclusive_scan_i32(cnt.get(), out.row_ptr.get(), n, s);
  int32_t nnz = 0;
  GB_HIP(hipMemcpyAsync(&nnz, out.row_ptr.get() + n, 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  out.nnz = nnz;
  out.col = DBuf<int32_t>(nnz, s);
  hipLaunchKernelGGL(k_union_rows<1>, dim3(n), dim3(kT), lds, s, n, rp0, c0, rp1, c1, nullptr,
                     out.row_ptr.get(), out.col.get());
  GB_LAUNCH_CHECK();
}

// CSR of the entries |a| >= tau of an ELL matrix (row-wise, rows ascending)
void ell_threshold(const gb_ell& A, double tau, DBuf<int32_t>& rp, DBuf<int32_t>& c,
                   hipStream_t s) {
  const int n = A.n;
  DBuf<int32_t> cnt(n, s);
  rp = DBuf<int32_t>(n + 1, s);
  hipLaunchKernelGGL(k_ell_threshold<0>, dim3(blocks_for(n, kT)), dim3(kT), 0, s, A.col, A.val, n,
                     A.width, tau, cnt.get(), nullptr, nullptr);
  GB_LAUNCH_CHECK();
  exclusive_scan_i32(cnt.get(), rp.get(), n, s);
  int32_t nnz = 0;
  GB_HIP(hipMemcpyAsync(&nnz, rp.get() + n, 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  c = DBuf<int32_t>(nnz > 0 ? nnz : 1, s);
  hipLaunchKernelGGL(k_ell_threshold<1>, dim3(blocks_for(n, kT)), dim3(kT), 0, s, A.col, A.val, n,
                     A.width, tau, nullptr, rp.get(), c.get());
  GB_LAUNCH_CHECK();
}

void transpose(int n, const int32_t* rp, const int32_t* c, int64_t nnz, DBuf<int32_t>& trp,
               DBuf<int32_t>& tc, hipStream_t s) {
  DBuf<int32_t> cnt(n, s), fill(n, s);
  hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(n, kT)), dim3(kT), 0, s, cnt.get(), (int64_t)n);
  hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(n, kT)), dim3(kT), 0, s, fill.get(), (int64_t)n);
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_tr_count, dim3(blocks_for(n, kT)), dim3(kT), 0, s, rp, c, n, cnt.get());
  GB_LAUNCH_CHECK();
  trp = DBuf<int32_t>(n + 1, s);
  exclusive_scan_i32(cnt.get(), trp.get(), n, s);
  tc = DBuf<int32_t>(nnz > 0 ? nnz : 1, s);
  hipLaunchKernelGGL(k_tr_fill, dim3(blocks_for(n, kT)), dim3(kT), 0, s, rp, c, n, trp.get(),
                     fill.get(), tc.get());
  GB_LAUNCH_CHECK();
}

}  // namespace

bool use_hash_sets(int n) {
  const char* e = std::getenv("GB_VERTEX_SETS");
  if (e && std::string(e) == "hash") return true;
  if (e && std::string(e) == "bitmap") return false;
  return n > (1 << 17);
}

void bounds(const gb_ell& H, hipStream_t s, double* emin, double* emax) {
  const int n = H.n;
  DBuf<double> lo(n, s), hi(n, s), out(3, s);
  hipLaunchKernelGGL(k_row_discs, dim3(blocks_for(n, kT)), dim3(kT), 0, s, H.col, H.val, n,
                     H.width, lo.get(), hi.get());
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_minmax, dim3(1), dim3(kT), 0, s, lo.get(), hi.get(), n, out.get());
  GB_LAUNCH_CHECK();
  double h[3];
  GB_HIP(hipMemcpyAsync(h, out.get(), sizeof(h), hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  if (h[2] != 0.0)
    fail(GB_EINVAL, "H holds NaN or Inf values (%.0f rows): no spectral bounds", h[2]);
  *emin = h[0];
  *emax = h[1];
}

// Device address of `scratch` on the current device, looked up once per device (each GPU holds
// its own copy of the array).  Host code uses only this address, never the array's name.
double* scratch_ptr() {
  static std::mutex mu;
  static std::map<int, double*> ptrs;
  int dev = 0;
  GB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptrs.find(dev);
  if (it != ptrs.end()) return it->second;
  void* p = nullptr;
  GB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) fail(GB_EHIP, "no device address for the bounds scratch array");
  ptrs[dev] = static_cast<double*>(p);
  return static_cast<double*>(p);
}

void bounds_noalloc(const gb_ell& H, hipStream_t s, double* emin, double* emax) {
  double* sc = scratch_ptr();
  const int nb = std::min(blocks_for(H.n, kT), kNoallocBlocks);
  hipLaunchKernelGGL(k_disc_partials, dim3(nb), dim3(kT), 0, s, H.col, H.val, H.n, H.width, sc);
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_disc_final, dim3(1), dim3(kT), 0, s, sc, nb, sc + 3 * kNoallocBlocks);
  GB_LAUNCH_CHECK();
  double h[3];
  GB_HIP(hipMemcpyAsync(h, sc + 3 * kNoallocBlocks, sizeof(h), hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  if (h[2] != 0.0)
    fail(GB_EINVAL, "H holds NaN or Inf values (%.0f rows): no spectral bounds", h[2]);
  *emin = h[0];
  *emax = h[1];
}

void x0_ell(const gb_ell& H, double emin, double emax, double* x0, hipStream_t s) {
  const int64_t tot = (int64_t)H.n * H.width;
  const double denom = emax - emin;
  hipLaunchKernelGGL(k_x0, dim3(blocks_for(tot, kT)), dim3(kT), 0, s, H.col, H.val, H.n, H.width,
                     emax, denom, x0);
  GB_LAUNCH_CHECK();
}

// X2 graph through the hash-set kernel: candidate capacity 2048 to start with (two workgroups
// per CU), raised to the largest count a row reports and run again (at most twice).
// the bounds b_i of the X2 kernels' order-free sums (see k_x2_rows)
void x2_row_bounds(const gb_ell& H, const double* x0, DBuf<double>& rb, hipStream_t s) {
  const int n = H.n, w = H.width;
  DBuf<double> amax(n, s);
  rb = DBuf<double>(n, s);
  const int nb = blocks_for(n, kT / 64);
  hipLaunchKernelGGL(k_row_absmax, dim3(nb), dim3(kT), 0, s, x0, n, w, amax.get());
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_x2_bound, dim3(nb), dim3(kT), 0, s, H.col, x0, amax.get(), n, w,
                     rb.get());
  GB_LAUNCH_CHECK();
}

// GB_X2_SUMS=ascending: every candidate is summed again in ascending order (a check of the
// path that the candidates near tau take)
int x2_all_ascending() {
  const char* e = std::getenv("GB_X2_SUMS");
  return e && std::string(e) == "ascending" ? 1 : 0;
}

void graph_x2_hash(const gb_ell& H, const double* x0, double tau, Csr& out, hipStream_t s) {
  const int n = H.n, w = H.width;
  if (w > kX2Q * kT) fail(GB_EUNSUPPORTED, "X2 graph: ELL width %d above %d", w, kX2Q * kT);
  int cap = (int)std::min<int64_t>(std::min<int64_t>((int64_t)w * w, n) + 1, 2048);
  cap = std::max(cap, kT);
  DBuf<int32_t> cnt(n, s), ovf(1, s), rows;
  DBuf<double> rb;
  x2_row_bounds(H, x0, rb, s);
  const int all_asc = x2_all_ascending();
  out.n = n;
  out.row_ptr = DBuf<int32_t>(n + 1, s);
  int32_t h[2] = {0, 0};
  for (int attempt = 0;; ++attempt) {
    const int log2h = ceil_log2((int64_t)cap + kT + 1), log2u = ceil_log2(cap);
    const size_t lds = x2_hash_lds_bytes(w, cap, log2h, log2u);
    if (lds > 160 * 1024)
      fail(GB_EUNSUPPORTED, "X2 graph: a row has %d two-hop candidates, more than LDS holds", cap);
    rows = DBuf<int32_t>((size_t)n * cap, s);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, ovf.get(), (int64_t)1);
    hipLaunchKernelGGL(k_x2_rows_hash, dim3(n), dim3(kT), lds, s, H.col, x0, rb.get(), n, w,
                       1.0f / (float)w, tau, all_asc, cap, log2h, log2u, cnt.get(), rows.get(),
                       ovf.get());
    GB_LAUNCH_CHECK();
    exclusive_scan_i32(cnt.get(), out.row_ptr.get(), n, s);
    GB_HIP(hipMemcpyAsync(&h[0], out.row_ptr.get() + n, 4, hipMemcpyDeviceToHost, s));
    GB_HIP(hipMemcpyAsync(&h[1], ovf.get(), 4, hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    if (h[1] == 0) break;
    if (attempt == 2) fail(GB_EUNSUPPORTED, "X2 graph: candidate count did not settle");
    // a stopped row counted at least cap + 1 candidates; grow past what was reported
    cap = std::max(((h[1] + 255) / 256) * 256, 2 * cap);
  }
  out.nnz = h[0];
  out.col = DBuf<int32_t>(h[0] > 0 ? h[0] : 1, s);
  hipLaunchKernelGGL(k_x2_compact, dim3(n), dim3(kT), 0, s, rows.get(), cap, cnt.get(),
                     out.row_ptr.get(), out.col.get());
  GB_LAUNCH_CHECK();
}

void graph_x2(const gb_ell& H, const double* x0, double tau, Csr& out, hipStream_t s) {
  const int n = H.n, w = H.width;
  if (use_hash_sets(n)) {
    graph_x2_hash(H, x0, tau, out, s);
    return;
  }
  // candidate capacity: small enough for six or more workgroups per CU at n up to ~2e4 (the
  // accumulators are most of the LDS); a row with more two-hop candidates makes the launch
  // report its count, and the launch reruns with it
  if (w > kX2Q * kT) fail(GB_EUNSUPPORTED, "X2 graph: ELL width %d above %d", w, kX2Q * kT);
  const size_t fixed = x2_lds_bytes(n, w, 0);
  if (fixed > 150 * 1024) fail(GB_EUNSUPPORTED, "X2 graph: n = %d too large for one LDS bitmap", n);
  const int64_t cap_lds = (int64_t)((160 * 1024 - fixed) / 8);
  int64_t cap = std::min<int64_t>(std::min<int64_t>((int64_t)w * w, n), 2048);
  cap = std::min(cap, cap_lds);
  DBuf<int32_t> cnt(n, s), ovf(1, s), rows;
  DBuf<double> rb;
  x2_row_bounds(H, x0, rb, s);
  const int all_asc = x2_all_ascending();
  out.n = n;
  out.row_ptr = DBuf<int32_t>(n + 1, s);
  int32_t h[2];
  for (int attempt = 0; attempt < 2; ++attempt) {
    const size_t lds = x2_lds_bytes(n, w, (int)cap);
    check_lds(lds, "X2 graph");
    rows = DBuf<int32_t>((size_t)n * cap, s);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, ovf.get(), (int64_t)1);
    hipLaunchKernelGGL(k_x2_rows, dim3(n), dim3(kT), lds, s, H.col, x0, rb.get(), n, w,
                       1.0f / (float)w, tau, all_asc, (int)cap, cnt.get(), rows.get(), ovf.get());
    GB_LAUNCH_CHECK();
    exclusive_scan_i32(cnt.get(), out.row_ptr.get(), n, s);
    GB_HIP(hipMemcpyAsync(&h[0], out.row_ptr.get() + n, 4, hipMemcpyDeviceToHost, s));
    GB_HIP(hipMemcpyAsync(&h[1], ovf.get(), 4, hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    if (h[1] == 0) break;
    if (attempt == 1 || h[1] > cap_lds)
      fail(GB_EUNSUPPORTED, "X2 graph: a row has %d two-hop candidates, LDS capacity is %lld",
           h[1], (long long)cap_lds);
    cap = ((h[1] + 255) / 256) * 256;
    cap = std::min(cap, cap_lds);
  }
  out.nnz = h[0];
  out.col = DBuf<int32_t>(h[0] > 0 ? h[0] : 1, s);
  hipLaunchKernelGGL(k_x2_compact, dim3(n), dim3(kT), 0, s, rows.get(), (int)cap, cnt.get(),
                     out.row_ptr.get(), out.col.get());
  GB_LAUNCH_CHECK();
}

void graph_pattern(const gb_ell& A, double tau, Csr& out, hipStream_t s) {
  DBuf<int32_t> rp, c, trp, tc;
  ell_threshold(A, tau, rp, c, s);
  int32_t nnz = 0;
  GB_HIP(hipMemcpyAsync(&nnz, rp.get() + A.n, 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  transpose(A.n, rp.get(), c.get(), nnz, trp, tc, s);
  union_rows(A.n, rp.get(), c.get(), trp.get(), tc.get(), out, s);
}

void graph_rcut(const double* pos, int n_sites, int m, double box, double r_cut, Csr& out,
                hipStream_t s) {
  const int n = n_sites * m;
  DBuf<int32_t> cnt(n, s);
  out.n = n;
  out.row_ptr = DBuf<int32_t>(n + 1, s);
  const double rc2 = r_cut * r_cut;
  hipLaunchKernelGGL(k_rcut_rows<0>, dim3(n_sites), dim3(kT), 0, s, pos, n_sites, m, box, rc2,
                     cnt.get(), nullptr, nullptr);
  GB_LAUNCH_CHECK();
  exclusive_scan_i32(cnt.get(), out.row_ptr.get(), n, s);
  int32_t nnz = 0;
  GB_HIP(hipMemcpyAsync(&nnz, out.row_ptr.get() + n, 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  out.nnz = nnz;
  out.col = DBuf<int32_t>(nnz > 0 ? nnz : 1, s);
  hipLaunchKernelGGL(k_rcut_rows<1>, dim3(n_sites), dim3(kT), 0, s, pos, n_sites, m, box, rc2,
                     nullptr, out.row_ptr.get(), out.col.get());
  GB_LAUNCH_CHECK();
}

void graph_dprev_symbolic(const gb_ell& H, const gb_ell& Dp, double tau_d, Csr& out,
                          hipStream_t s) {
  // P = pattern(H) U {|D_prev| >= tau_d} U its transpose (symmetric, with self-loops), then
  // the symbolic square: Eq. 8 with eps = 0
  Csr hp, P;
  graph_pattern(H, 0.0, hp, s);
  graph_union_dprev(hp, Dp, tau_d, P, s);
  const int n = H.n;
  const int nw = (n + 31) >> 5;
  const size_t lds = (size_t)nw * 8 + kT * 4 + 64;
  check_lds(lds, "two-hop graph");
  DBuf<int32_t> cnt(n, s);
  out.n = n;
  out.row_ptr = DBuf<int32_t>(n + 1, s);
  hipLaunchKernelGGL(k_twohop_rows<0>, dim3(n), dim3(kT), lds, s, n, P.row_ptr.get(), P.col.get(),
                     cnt.get(), nullptr, nullptr);
  GB_LAUNCH_CHECK();
  exclusive_scan_i32(cnt.get(), out.row_ptr.get(), n, s);
  int32_t nnz = 0;
  GB_HIP(hipMemcpyAsync(&nnz, out.row_ptr.get() + n, 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  out.nnz = nnz;
  out.col = DBuf<int32_t>(nnz > 0 ? nnz : 1, s);
  hipLaunchKernelGGL(k_twohop_rows<1>, dim3(n), dim3(kT), lds, s, n, P.row_ptr.get(), P.col.get(),
                     nullptr, out.row_ptr.get(), out.col.get());
  GB_LAUNCH_CHECK();
}

void graph_union_dprev(const Csr& base, const gb_ell& Dp, double tau_d, Csr& out,
                       hipStream_t s) {
  // column-ELL row i lists the rows r of column i with |D_ri| >= tau_d: edges (r, i).
  // The union of base (symmetric), that list (row i gets r) and its transpose (row r gets i)
  // is symmetric.
  DBuf<int32_t> rp, c, trp, tc;
  ell_threshold(Dp, tau_d, rp, c, s);
  int32_t nnz = 0;
  GB_HIP(hipMemcpyAsync(&nnz, rp.get() + Dp.n, 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  transpose(Dp.n, rp.get(), c.get(), nnz, trp, tc, s);
  Csr tmp;
  union_rows(Dp.n, rp.get(), c.get(), trp.get(), tc.get(), tmp, s);
  union_rows(Dp.n, base.row_ptr.get(), base.col.get(), tmp.row_ptr.get(), tmp.col.get(), out, s);
}

}  // namespace gbi
