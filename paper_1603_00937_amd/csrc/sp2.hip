// Batched SP2 on the subgraph blocks: gather, the MFMA squaring kernel, the FP64 trace /
// branch decision, the update, refinement, the column scatter into D and the final checks.
//
// Data layout in HBM: every subgraph s owns a dense row-major block of npad_s x npad_s
// elements (npad_s = n_s rounded up to 64) at element offset off_s of one batch buffer; the
// padding rows and columns are zero and stay zero under X^2 and 2X - X^2.  Two (three with
// refinement) such buffers ping-pong.  Core vertices are the first k_s rows of each block.
#include "internal.h"

#include <cmath>
#include <numeric>

#pragma clang fp contract(off)

namespace gbi {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  using acc_t = d4v;
  static constexpr int KC = 16;  // k elements per 128-byte row chunk
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output register r of lane l holds row (4r + l/16), column l%16 of the 16x16 block
  __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct Mfma<float> {
  using acc_t = f4v;
  static constexpr int KC = 32;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output register r of lane l holds row (4(l/16) + r), column l%16
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

namespace {

constexpr int kT = 256;
constexpr int kBT = 128;  // workgroup tile edge

// ---- gather: x0[s] = principal submatrix of X0 on the subgraph, zero padded -------------
// Block (s, chunk) writes rows [chunk*kRows, +kRows) of block s.  The subgraph list sits in
// LDS; the local column of an ELL entry is found by binary search in the core run and in
// the halo run (both ascending).
constexpr int kRows = 16;

template <typename T>
__global__ __launch_bounds__(kT) void k_gather(const int32_t* __restrict__ hcol,
                                               const double* __restrict__ x0, int w,
                                               const int32_t* __restrict__ core_ptr,
                                               const int32_t* __restrict__ sub_ptr,
                                               const int32_t* __restrict__ sub_idx,
                                               const int64_t* __restrict__ offs,
                                               const int32_t* __restrict__ npad, T* __restrict__ X) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int s = blockIdx.x;
  const int np = npad[s];
  const int a0 = blockIdx.y * kRows;
  if (a0 >= np) return;
  const int b = sub_ptr[s], n = sub_ptr[s + 1] - b;
  const int k = core_ptr[s + 1] - core_ptr[s];
  double* row = reinterpret_cast<double*>(smem);
  int32_t* sub = reinterpret_cast<int32_t*>(row + np);
  for (int a = threadIdx.x; a < n; a += kT) sub[a] = sub_idx[b + a];
  T* base = X + offs[s];
  for (int a = a0; a < a0 + kRows && a < np; ++a) {
    for (int c = threadIdx.x; c < np; c += kT) row[c] = 0.0;
    __syncthreads();
    if (a < n) {
      const int i = sub[a];
      for (int t = threadIdx.x; t < w; t += kT) {
        const int32_t j = hcol[(int64_t)i * w + t];
        if (j < 0) continue;
        // core run [0, k)
        int lo = 0, hi = k;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (sub[mid] < j) lo = mid + 1;
          else hi = mid;
        }
        int loc = -1;
        if (lo < k && sub[lo] == j) loc = lo;
        else {
          lo = k;
          hi = n;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sub[mid] < j) lo = mid + 1;
            else hi = mid;
          }
          if (lo < n && sub[lo] == j) loc = lo;
        }
        if (loc >= 0) row[loc] = x0[(int64_t)i * w + t];
      }
    }
    __syncthreads();
    T* dst = base + (int64_t)a * np;
    for (int c = threadIdx.x; c < np; c += kT) dst[c] = (T)row[c];
    __syncthreads();
  }
}

// ---- the squaring kernel ----------------------------------------------------------------
// One workgroup (4 waves, 2 x 2) computes a 128 x 128 tile (bi, bj), bi <= bj, of a product of
// two symmetric blocks that commute (X*X, or X^2*X), so the result is symmetric: the tile is
// written at (bi, bj) and mirrored to (bj, bi).  Both operands are read as row panels (for a
// symmetric B, column j of B is row j).  k is consumed in 128-byte chunks staged in LDS
// (double buffered, one barrier per chunk).  Inside a chunk lane group g = lane/16 takes the
// k slice [g*KC/4, (g+1)*KC/4): the contraction is a sum over k, so any k order shared by
// both operands is valid, and each lane reads its slice with 16-byte LDS loads.
//   MODE 0: out = A*B          MODE 1: out = alpha*(A*B) + beta*E   (E symmetric)
template <typename T, int MODE>
__global__ __launch_bounds__(kT, 2) void k_symm_mm(const T* __restrict__ A, const T* __restrict__ B,
                                                   const T* __restrict__ E, T* __restrict__ out,
                                                   T alpha, T beta, const int4* __restrict__ tiles,
                                                   const int64_t* __restrict__ offs) {
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  constexpr int KC = M::KC;
  constexpr int V = 16 / sizeof(T);      // elements per 16-byte vector
  constexpr int STR = KC + V;            // padded LDS row stride (elements)
  constexpr int KG = KC / 4;             // k elements per lane group per chunk
  __shared__ __align__(16) T As[2][kBT * STR];
  __shared__ __align__(16) T Bs[2][kBT * STR];

  const int4 tl = tiles[blockIdx.x];
  const int s = tl.x, bi = tl.y, bj = tl.z, np = tl.w;
  const int64_t off = offs[s];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // global -> LDS staging: thread -> one row, one 64-byte half of the chunk
  const int lr = tid >> 1, lh = tid & 1;
  const int arow = bi * kBT + lr, brow = bj * kBT + lr;
  const bool aok = arow < np, bok = brow < np;
  const T* ap = A + off + (int64_t)(aok ? arow : 0) * np + lh * (KC / 2);
  const T* bp = B + off + (int64_t)(bok ? brow : 0) * np + lh * (KC / 2);
  uint4 ra[4], rb[4];
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);

  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ra[q] = aok ? *reinterpret_cast<const uint4*>(ap + k0 + q * V) : z4;
      rb[q] = bok ? *reinterpret_cast<const uint4*>(bp + k0 + q * V) : z4;
    }
  };
  auto sstore = [&](int buf) {
    T* da = &As[buf][lr * STR + lh * (KC / 2)];
    T* db = &Bs[buf][lr * STR + lh * (KC / 2)];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<uint4*>(da + q * V) = ra[q];
      *reinterpret_cast<uint4*>(db + q * V) = rb[q];
    }
  };

  acc_t acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[m][n] = acc_t{0, 0, 0, 0};

  const int g = lane >> 4, r16 = lane & 15;
  const int nk = np / KC;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * KC);
    const T* as = &As[buf][(wr * 64 + r16) * STR + g * KG];
    const T* bs = &Bs[buf][(wc * 64 + r16) * STR + g * KG];
#pragma unroll
    for (int h = 0; h < KG; h += V) {
      T fa[4][V], fb[4][V];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const uint4 va = *reinterpret_cast<const uint4*>(as + m * 16 * STR + h);
        const uint4 vb = *reinterpret_cast<const uint4*>(bs + m * 16 * STR + h);
        __builtin_memcpy(fa[m], &va, 16);
        __builtin_memcpy(fb[m], &vb, 16);
      }
#pragma unroll
      for (int e = 0; e < V; ++e)
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[m][n] = M::mma(fa[m][e], fb[n][e], acc[m][n]);
    }
    if (kc + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  T* o = out + off;
  const T* e = E + off;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int grow = bi * kBT + wr * 64 + m * 16 + M::row(lane, r);
        const int gcol = bj * kBT + wc * 64 + n * 16 + r16;
        if (grow < np && gcol < np) {
          T v = acc[m][n][r];
          if (MODE == 1) v = alpha * v + beta * e[(int64_t)grow * np + gcol];
          o[(int64_t)grow * np + gcol] = v;
          if (bi != bj) o[(int64_t)gcol * np + grow] = v;
        }
      }
}

// ---- traces and the branch decision (one workgroup, deterministic order) -----------------
struct StepRec {
  double t1, t2, e, margin;
  int32_t b, stop, pad0, pad1;
};

// forced: -1 choose by the trace rule, 0/1 replay that branch, 2 stop (replay exhausted)
template <typename T>
__global__ __launch_bounds__(kT) void k_trace_branch(const T* __restrict__ X, const T* __restrict__ S,
                                                     const int64_t* __restrict__ offs,
                                                     const int32_t* __restrict__ npad,
                                                     const int32_t* __restrict__ core_ptr, int n_sub,
                                                     double n_occ, double tol, int forced,
                                                     int at_max, StepRec* __restrict__ rec) {
  __shared__ double r1[kT], r2[kT];
  double p1 = 0.0, p2 = 0.0;
  for (int s = threadIdx.x; s < n_sub; s += kT) {
    const int np = npad[s];
    const int k = core_ptr[s + 1] - core_ptr[s];
    const T* xs = X + offs[s];
    const T* ss = S + offs[s];
    for (int j = 0; j < k; ++j) {
      p1 += (double)xs[(int64_t)j * np + j];
      p2 += (double)ss[(int64_t)j * np + j];
    }
  }
  r1[threadIdx.x] = p1;
  r2[threadIdx.x] = p2;
  __syncthreads();
  for (int h = kT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      r1[threadIdx.x] += r1[threadIdx.x + h];
      r2[threadIdx.x] += r2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double t1 = r1[0], t2 = r2[0];
    const double e = fabs(t1 - t2);
    const double dsq = fabs(t2 - n_occ), dlin = fabs(2.0 * t1 - t2 - n_occ);
    StepRec q;
    q.t1 = t1;
    q.t2 = t2;
    q.e = e;
    q.margin = fabs(dsq - dlin);
    q.pad0 = q.pad1 = 0;
    if (forced == 2) {
      q.stop = 1;
      q.b = -1;
    } else if (forced >= 0) {
      q.stop = 0;
      q.b = forced;
    } else if (e <= tol) {
      q.stop = 1;
      q.b = -1;
    } else if (at_max) {
      q.stop = 2;
      q.b = -1;
    } else {
      q.stop = 0;
      q.b = dsq < dlin ? 0 : 1;
    }
    *rec = q;
  }
}

// S <- 2X - S over the whole batch buffer (padding stays 0)
template <typename T>
__global__ void k_lin_update(const T* __restrict__ X, T* __restrict__ S, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = i; p < n; p += stride) S[p] = (T)2 * X[p] - S[p];
}

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = i; p < n; p += stride) out[p] = (TO)in[p];
}

// ---- scatter: column i of D = column (= row, X symmetric) j of its subgraph block -------
template <typename T>
__global__ __launch_bounds__(kT) void k_scatter(const T* __restrict__ X, const int64_t* __restrict__ offs,
                                                const int32_t* __restrict__ npad,
                                                const int32_t* __restrict__ sub_ptr,
                                                const int32_t* __restrict__ sub_idx,
                                                const int32_t* __restrict__ sub_pos,
                                                const int32_t* __restrict__ col_sub,
                                                const int32_t* __restrict__ col_loc, int w,
                                                int32_t* __restrict__ dcol, double* __restrict__ dval) {
  const int i = blockIdx.x;
  const int s = col_sub[i], j = col_loc[i];
  const int b = sub_ptr[s], n = sub_ptr[s + 1] - b, np = npad[s];
  const T* xr = X + offs[s] + (int64_t)j * np;
  int32_t* oc = dcol + (int64_t)i * w;
  double* ov = dval + (int64_t)i * w;
  for (int a = threadIdx.x; a < n; a += kT) {
    const int p = sub_pos[b + a];
    oc[p] = sub_idx[b + a];
    ov[p] = (double)xr[a];
  }
  for (int r = n + threadIdx.x; r < w; r += kT) {
    oc[r] = -1;
    ov[r] = 0.0;
  }
}

// max over core rows j < k_s and columns a < n_s of |S - X| (one block per subgraph)
template <typename T>
__global__ __launch_bounds__(kT) void k_idem(const T* __restrict__ X, const T* __restrict__ S,
                                             const int64_t* __restrict__ offs,
                                             const int32_t* __restrict__ npad,
                                             const int32_t* __restrict__ core_ptr,
                                             const int32_t* __restrict__ sub_ptr,
                                             double* __restrict__ out) {
  __shared__ double red[kT];
  const int s = blockIdx.x;
  const int np = npad[s], n = sub_ptr[s + 1] - sub_ptr[s], k = core_ptr[s + 1] - core_ptr[s];
  double m = 0.0;
  for (int64_t p = threadIdx.x; p < (int64_t)k * n; p += kT) {
    const int j = (int)(p / n), a = (int)(p - (int64_t)j * n);
    const int64_t q = offs[s] + (int64_t)j * np + a;
    m = fmax(m, fabs((double)S[q] - (double)X[q]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = kT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[s] = red[0];
}

__global__ void k_max(const double* __restrict__ in, int n, double* __restrict__ out) {
  __shared__ double red[kT];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kT) m = fmax(m, in[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = kT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

int grid_for(int64_t n, int t, int cap = 1 << 20) {
  const int64_t b = (n + t - 1) / t;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// ---- plan: padded sizes, offsets, tile list --------------------------------------------
struct Plan {
  int n_sub = 0;
  std::vector<int32_t> npad;
  std::vector<int64_t> off;
  int64_t total = 0;
  std::vector<int4> tiles;
  double flops_alg = 0, flops_exec = 0;
  int max_npad = 0;
};

Plan make_plan(const Part& P) {
  Plan pl;
  pl.n_sub = P.n_sub;
  pl.npad.resize(P.n_sub);
  pl.off.resize(P.n_sub);
  std::vector<int> order(P.n_sub);
  for (int s = 0; s < P.n_sub; ++s) {
    const int n = P.h_sub_ptr[s + 1] - P.h_sub_ptr[s];
    pl.npad[s] = ((n + 63) / 64) * 64;
    pl.off[s] = pl.total;
    pl.total += (int64_t)pl.npad[s] * pl.npad[s];
    pl.flops_alg += 2.0 * (double)n * n * n;
    pl.max_npad = std::max(pl.max_npad, pl.npad[s]);
    order[s] = s;
  }
  // longest first: tiles of the largest blocks (most k work per tile) start earliest
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return pl.npad[a] > pl.npad[b]; });
  for (int s : order) {
    const int np = pl.npad[s];
    const int nb = (np + kBT - 1) / kBT;
    for (int bi = 0; bi < nb; ++bi)
      for (int bj = bi; bj < nb; ++bj) {
        pl.tiles.push_back(make_int4(s, bi, bj, np));
        pl.flops_exec += 2.0 * kBT * kBT * (double)np;
      }
  }
  return pl;
}

template <typename T>
void launch_square(const T* X, T* S, const DBuf<int4>& tiles, int ntiles, const int64_t* offs,
                   hipStream_t s) {
  hipLaunchKernelGGL((k_symm_mm<T, 0>), dim3(ntiles), dim3(kT), 0, s, X, X, X, S, (T)1, (T)0,
                     tiles.get(), offs);
  GB_LAUNCH_CHECK();
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  explicit Timer() {
    GB_HIP(hipEventCreate(&a));
    GB_HIP(hipEventCreate(&b));
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  GB_HIP(hipEventElapsedTime(&ms, a, b));
  return ms;
}

struct PinnedRec {
  StepRec* h = nullptr;
  PinnedRec() { GB_HIP(hipHostMalloc((void**)&h, sizeof(StepRec), hipHostMallocDefault)); }
  ~PinnedRec() {
    if (h) (void)hipHostFree(h);
  }
};

// Runs the SP2 loop in precision T on buffers X (current iterate) and S (scratch).
// Returns when the stop rule fires, the replay ends, max_iter is reached, or (low precision)
// when the idempotency error stagnates.  Records every step into stats.
template <typename T>
int sp2_loop(T*& X, T*& S, const Plan& pl, const DBuf<int4>& tiles, const DBuf<int64_t>& offs,
             const DBuf<int32_t>& npad, const Part& P, double n_occ, double tol, int max_iter,
             const uint8_t* branch_in, int n_branch_in, bool stagnation_stop, int it0,
             gb_sp2_stats& st, DBuf<StepRec>& recs, hipStream_t s, int* stop_kind) {
  Timer tm;
  PinnedRec pin;
  int it = it0;
  std::vector<double> es;
  const int ntiles = (int)pl.tiles.size();
  for (;;) {
    GB_HIP(hipEventRecord(tm.a, s));
    launch_square<T>(X, S, tiles, ntiles, offs.get(), s);
    GB_HIP(hipEventRecord(tm.b, s));
    int forced = -1;
    if (branch_in) forced = it < n_branch_in ? (int)branch_in[it] : 2;
    const int at_max = it >= max_iter ? 1 : 0;
    hipLaunchKernelGGL(k_trace_branch<T>, dim3(1), dim3(kT), 0, s, X, S, offs.get(), npad.get(),
                       P.core_ptr.get(), P.n_sub, n_occ, tol, forced, at_max, recs.get() + (it % 2));
    GB_LAUNCH_CHECK();
    GB_HIP(hipMemcpyAsync(pin.h, recs.get() + (it % 2), sizeof(StepRec), hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    st.ms_square += elapsed(tm.a, tm.b);
    st.n_square += 1;
    const StepRec r = *pin.h;
    if (it < 128) {
      st.t1[it] = r.t1;
      st.t2[it] = r.t2;
    }
    st.idem = r.e;
    es.push_back(r.e);
    if (r.stop) {
      *stop_kind = (r.stop == 1 && (branch_in == nullptr || r.e <= tol)) ? 1 : 2;
      if (branch_in && r.stop == 1) *stop_kind = r.e <= tol ? 1 : 3;
      return it;
    }
    if (stagnation_stop && es.size() >= 10 && es.back() > es[es.size() - 3]) {
      *stop_kind = 4;
      return it;
    }
    if (it < 128) st.branch[it] = (uint8_t)r.b;
    if (branch_in == nullptr) st.min_margin = std::min(st.min_margin, r.margin);
    if (r.b == 1) {
      const int64_t n = pl.total;
      hipLaunchKernelGGL(k_lin_update<T>, dim3(grid_for(n, kT, 65536)), dim3(kT), 0, s, X, S, n);
      GB_LAUNCH_CHECK();
    }
    std::swap(X, S);
    ++it;
  }
}

}  // namespace

// Full gb_density pipeline on an already built partition.
void density(const gb_ell& H, int32_t n_occ, const gb_sp2_opts& o, const Part& P, double emin,
             double emax, const double* x0, gb_ell& D, gb_sp2_stats& st, hipStream_t s) {
  Timer t_all, t_stage;
  GB_HIP(hipEventRecord(t_all.a, s));
  const Plan pl = make_plan(P);
  st.square_flops = pl.flops_alg;
  st.square_flops_exec = pl.flops_exec;
  DBuf<int64_t> offs(pl.n_sub, s);
  DBuf<int32_t> npad(pl.n_sub, s);
  DBuf<int4> tiles(pl.tiles.size(), s);
  GB_HIP(hipMemcpyAsync(offs.get(), pl.off.data(), pl.n_sub * 8, hipMemcpyHostToDevice, s));
  GB_HIP(hipMemcpyAsync(npad.get(), pl.npad.data(), pl.n_sub * 4, hipMemcpyHostToDevice, s));
  GB_HIP(hipMemcpyAsync(tiles.get(), pl.tiles.data(), pl.tiles.size() * sizeof(int4),
                        hipMemcpyHostToDevice, s));
  DBuf<StepRec> recs(2, s);
  const int N = H.n;
  const double tol = o.idem_tol > 0 ? o.idem_tol : 1e-10 * N / 1024.0;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 100;
  const bool low = o.precision == GB_FP32_REFINE;
  const int n_refine = o.n_refine;
  int stop_kind = 0;
  // the gather is timed with the first buffer allocation included
  GB_HIP(hipEventRecord(t_stage.a, s));
  const size_t lds_g = (size_t)pl.max_npad * 8 + (size_t)P.max_sub * 4 + 64;
  if (lds_g > 160 * 1024) fail(GB_EUNSUPPORTED, "subgraph of %d vertices too large", P.max_sub);
  const dim3 ggrid(pl.n_sub, (pl.max_npad + kRows - 1) / kRows);
  DBuf<double> X64, S64, T64;
  double* xd = nullptr;
  double* sd = nullptr;
  int it_end = 0;
  if (low) {
    DBuf<float> X32(pl.total, s), S32(pl.total, s);
    hipLaunchKernelGGL(k_gather<float>, ggrid, dim3(kT), lds_g, s, H.col, x0, H.width,
                       P.core_ptr.get(), P.sub_ptr.get(), P.sub_idx.get(), offs.get(), npad.get(),
                       X32.get());
    GB_LAUNCH_CHECK();
    GB_HIP(hipEventRecord(t_stage.b, s));
    GB_HIP(hipStreamSynchronize(s));
    st.ms_gather = elapsed(t_stage.a, t_stage.b);
    GB_HIP(hipEventRecord(t_stage.a, s));
    float* xf = X32.get();
    float* sf = S32.get();
    const double tol_lo = 1e-5 * N / 1024.0;
    it_end = sp2_loop<float>(xf, sf, pl, tiles, offs, npad, P, n_occ, tol_lo, max_iter, o.branch_in,
                             o.n_branch_in, true, 0, st, recs, s, &stop_kind);
    // the final low-precision square was only the stop test: continue from X in FP64
    X64 = DBuf<double>(pl.total, s);
    S64 = DBuf<double>(pl.total, s);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(pl.total, kT, 65536)), dim3(kT), 0,
                       s, xf, X64.get(), pl.total);
    GB_LAUNCH_CHECK();
    GB_HIP(hipEventRecord(t_stage.b, s));
    GB_HIP(hipStreamSynchronize(s));
    st.ms_sp2 = elapsed(t_stage.a, t_stage.b);
  } else {
    X64 = DBuf<double>(pl.total, s);
    S64 = DBuf<double>(pl.total, s);
    hipLaunchKernelGGL(k_gather<double>, ggrid, dim3(kT), lds_g, s, H.col, x0, H.width,
                       P.core_ptr.get(), P.sub_ptr.get(), P.sub_idx.get(), offs.get(), npad.get(),
                       X64.get());
    GB_LAUNCH_CHECK();
    GB_HIP(hipEventRecord(t_stage.b, s));
    GB_HIP(hipStreamSynchronize(s));
    st.ms_gather = elapsed(t_stage.a, t_stage.b);
  }
  xd = X64.get();
  sd = S64.get();
  GB_HIP(hipEventRecord(t_stage.a, s));
  if (low) {
    // FP64 refinement: SP2 steps with FP64 traces from where the FP32 loop stopped
    const uint8_t* bin = nullptr;
    int nbin = 0;
    if (o.branch_in && o.n_branch_in > it_end) {
      bin = o.branch_in;
      nbin = o.n_branch_in;
    }
    const int cap = n_refine > 0 ? it_end + n_refine : max_iter;
    it_end = sp2_loop<double>(xd, sd, pl, tiles, offs, npad, P, n_occ, tol, cap, bin, nbin, false,
                              it_end, st, recs, s, &stop_kind);
  } else {
    it_end = sp2_loop<double>(xd, sd, pl, tiles, offs, npad, P, n_occ, tol, max_iter, o.branch_in,
                              o.n_branch_in, false, 0, st, recs, s, &stop_kind);
  }
  GB_HIP(hipEventRecord(t_stage.b, s));
  GB_HIP(hipStreamSynchronize(s));
  if (low) st.ms_refine = elapsed(t_stage.a, t_stage.b);
  else st.ms_sp2 = elapsed(t_stage.a, t_stage.b);
  st.iters = it_end;
  st.converged = stop_kind == 1 ? 1 : 0;

  // checks on the final X (S = X^2 from the last square)
  DBuf<double> per(pl.n_sub, s), mx(1, s);
  hipLaunchKernelGGL(k_idem<double>, dim3(pl.n_sub), dim3(kT), 0, s, xd, sd, offs.get(), npad.get(),
                     P.core_ptr.get(), P.sub_ptr.get(), per.get());
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_max, dim3(1), dim3(kT), 0, s, per.get(), pl.n_sub, mx.get());
  GB_LAUNCH_CHECK();
  // scatter
  GB_HIP(hipEventRecord(t_stage.a, s));
  hipLaunchKernelGGL(k_scatter<double>, dim3(N), dim3(kT), 0, s, xd, offs.get(), npad.get(),
                     P.sub_ptr.get(), P.sub_idx.get(), P.sub_pos.get(), P.col_sub.get(),
                     P.col_loc.get(), D.width, D.col, D.val);
  GB_LAUNCH_CHECK();
  GB_HIP(hipEventRecord(t_stage.b, s));
  double idem_max = 0;
  GB_HIP(hipMemcpyAsync(&idem_max, mx.get(), 8, hipMemcpyDeviceToHost, s));
  GB_HIP(hipEventRecord(t_all.b, s));
  GB_HIP(hipStreamSynchronize(s));
  st.ms_scatter = elapsed(t_stage.a, t_stage.b);
  st.idem_max = idem_max;
  const int last = std::min(it_end, 127);
  st.trace = st.t1[last];
  st.ms_total += elapsed(t_all.a, t_all.b);
}

}  // namespace gbi
