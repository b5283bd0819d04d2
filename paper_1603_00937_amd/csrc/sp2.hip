// Batched SP2 on the subgraph blocks: gather, the MFMA squaring kernel, the FP64 trace /
// branch decision, the update, refinement, the column scatter into D and the final checks.
//
// Data layout in HBM: every subgraph s owns a dense row-major block of npad_s x npad_s
// elements (npad_s = n_s rounded up to 64) at element offset off_s of one batch buffer; the
// padding rows and columns are zero and stay zero under X^2 and 2X - X^2.  Two (three with
// refinement) such buffers ping-pong.  Core vertices are the first k_s rows of each block.
#include "internal.h"

#include <cmath>
#include <cstring>
#include <cstdlib>
#include <deque>
#include <string>
#include <map>
#include <mutex>
#include <numeric>
#include <type_traits>

#pragma clang fp contract(off)

namespace gbi {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

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

typedef __attribute__((address_space(3))) void lds_void;

// Target builtins are called only from these non-template device functions: a kernel template
// that names one directly is dropped from the host pass (no launch stub is emitted for it).
// 16-byte global -> LDS copy of one lane: lane L of the wave fills bytes [16L, 16L + 16) of
// the 1-KB LDS window that starts at `lds` (the same for every lane of the wave).
__device__ inline void load_lds16(const void* g, void* lds) {
  __builtin_amdgcn_global_load_lds(g, (lds_void*)lds, 16, 0, 0);
}
__device__ inline f4v mma_bf16(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
// fp16 planes travel in the same 16-byte registers as bf16 ones and are reinterpreted here
__device__ inline f4v mma_f16(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a),
                                                __builtin_bit_cast(h8v, b), c, 0, 0, 0);
}
// plane products of either type
template <bool F16>
__device__ __forceinline__ f4v mma_p(bf8v a, bf8v b, f4v c) {
  if constexpr (F16) return mma_f16(a, b, c);
  else return mma_bf16(a, b, c);
}


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
                                               const int32_t* __restrict__ npad, T* __restrict__ X,
                                               T scale) {
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
    for (int c = threadIdx.x; c < np; c += kT) dst[c] = (T)row[c] * scale;
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
//   MODE 3: out = A*B for a general (non-symmetric) product with B symmetric: every tile
//           (bi, bj) is listed and nothing is mirrored (the adjoint's Gbar*X)
//   MODE 4: as MODE 1, and dacc += cn * out (the Chebyshev recurrence with the running sum)
// In MODE 0 (A = B = X) the SP2 update is fused into the epilogue: with the branch
// 2X - X^2 selected (lin, or *lin_flag on the device-driven loop) the kernel writes 2X - X^2,
// else X^2.  X is symmetric, so the mirrored entry takes the same value.
// STAGES = 2: the next chunk loads while the current one is consumed; STAGES = 3: the two next
// chunks are in flight (one more LDS buffer), for latency the second buffer cannot hide.
// LOADER = 0: chunks go from global memory straight into LDS; LOADER = 1 (two stages): the
// chunk after next is loaded into registers under the current products and written to LDS
// once they are done.
template <typename T, int MODE, int BT = 128, int STAGES = 2, int LOADER = 0>
__global__ __launch_bounds__(kT, 2) void k_symm_mm(const T* __restrict__ A, const T* __restrict__ B,
                                                   const T* __restrict__ E, T* __restrict__ out,
                                                   T alpha, T beta, const int4* __restrict__ tiles,
                                                   const int64_t* __restrict__ offs,
                                                   const int32_t* __restrict__ stopped,
                                                   int lin, const int32_t* __restrict__ lin_flag,
                                                   T* __restrict__ dacc, T cn) {
  if (stopped && *stopped) return;  // device-driven loop: the expansion already stopped
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  constexpr int KC = M::KC;              // k elements per 128-byte row chunk
  constexpr int V = 16 / sizeof(T);      // elements per 16-byte piece
  constexpr int KG = KC / 4;             // k elements per lane group per chunk (two pieces)
  constexpr int WM = BT / 2;             // wave tile edge (2 x 2 waves)
  constexpr int MB = WM / 16;            // 16 x 16 blocks per wave tile edge
  constexpr int OPB = BT * 128;          // LDS bytes per operand per buffer
  constexpr int NLD = BT / 32;           // 1-KB wave loads per operand per chunk
  // [buffer][operand][row-major 128-byte rows, the eight 16-byte pieces of row r stored at
  // slot (piece ^ (r & 7)) so that sixteen lanes reading one piece of sixteen rows hit
  // different banks]
  __shared__ __align__(1024) unsigned char lds[STAGES][2][OPB];

  const int4 tl = tiles[blockIdx.x];
  if (tl.x < 0) return;  // padding entry of an XCD queue
  const int s = tl.x, bi = tl.y, bj = tl.z, np = tl.w;
  const int64_t off = offs[s];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // Global -> LDS without registers (global_load_lds_dwordx4: lane L of a wave writes bytes
  // [16 L, 16 L + 16) of the wave's 1-KB LDS window).  Each lane's source is chosen so the
  // window receives the swizzled layout; rows beyond np (half-empty edge tiles) read row 0
  // instead, which only feeds output rows / columns that are never stored.
  const T* asrc[NLD];
  const T* bsrc[NLD];
#pragma unroll
  for (int j = 0; j < NLD; ++j) {
    const int slot = (wave * NLD + j) * 64 + lane;
    const int r = slot >> 3, c = (slot & 7) ^ (r & 7);
    const int ar = bi * BT + r, br = bj * BT + r;
    asrc[j] = A + off + (int64_t)(ar < np ? ar : 0) * np + c * V;
    bsrc[j] = B + off + (int64_t)(br < np ? br : 0) * np + c * V;
  }
#define GB_ISSUE(buf, k0)                                                                   \
  _Pragma("unroll") for (int j = 0; j < NLD; ++j) {                                         \
    load_lds16(asrc[j] + (k0), &lds[buf][0][(wave * NLD + j) * 1024]);                      \
    load_lds16(bsrc[j] + (k0), &lds[buf][1][(wave * NLD + j) * 1024]);                      \
  }

  acc_t acc[MB][MB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < MB; ++n) acc[m][n] = acc_t{0, 0, 0, 0};

  const int g = lane >> 4, r16 = lane & 15;
  const int nk = np / KC;
  // a wave whose row or column block lies in the padding beyond np has nothing to compute;
  // on a diagonal tile of a symmetric product the lower-left block is the transpose of the
  // upper-right one, which that wave writes twice
  const bool in_range = bi * BT + wr * WM < np && bj * BT + wc * WM < np;
  const bool lower_diag = MODE != 3 && bi == bj && wr > wc;
  const bool active = in_range && !lower_diag;
  // byte offsets of this lane's pieces (2g + h) in rows wr*WM + m*16 + r16 (A) and
  // wc*WM + n*16 + r16 (B); (row & 7) = (r16 & 7) for every m
  const int sw = r16 & 7;
  const int pa0 = (wr * WM + r16) * 128, pb0 = (wc * WM + r16) * 128;
  const int pc0 = (((2 * g) ^ sw) << 4), pc1 = (((2 * g + 1) ^ sw) << 4);

  // each wave issues 2 NLD loads per chunk; loads complete in order, so waiting until at most
  // 2 NLD are outstanding means every chunk but the newest has landed
  static_assert(STAGES == 2 || STAGES == 3, "two or three LDS stages");
  static_assert(STAGES == 2 || 2 * NLD == 4 || 2 * NLD == 8, "wait count");
#define GB_WAIT_ALL_BUT_NEWEST()                                   \
  do {                                                             \
    if constexpr (2 * NLD == 4) asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); \
    else asm volatile("s_waitcnt vmcnt(8)" ::: "memory");          \
  } while (0)
  static_assert(LOADER == 0 || STAGES == 2, "register staging uses two LDS buffers");
  u4v stg[2][NLD];  // LOADER = 1: [operand][j], the 16 bytes this lane moves
#define GB_STAGE(k0)                                                                        \
  _Pragma("unroll") for (int j = 0; j < NLD; ++j) {                                         \
    stg[0][j] = *reinterpret_cast<const u4v*>(asrc[j] + (k0));                             \
    stg[1][j] = *reinterpret_cast<const u4v*>(bsrc[j] + (k0));                             \
  }
#define GB_PUT(buf)                                                                         \
  _Pragma("unroll") for (int j = 0; j < NLD; ++j) {                                         \
    *reinterpret_cast<u4v*>(&lds[buf][0][(wave * NLD + j) * 1024 + lane * 16]) = stg[0][j]; \
    *reinterpret_cast<u4v*>(&lds[buf][1][(wave * NLD + j) * 1024 + lane * 16]) = stg[1][j]; \
  }
  if (LOADER == 1) {
    GB_STAGE(0)
    GB_PUT(0)
    if (nk > 1) {
      GB_STAGE(KC)
    }
  } else {
    GB_ISSUE(0, 0)
    if (STAGES == 3 && nk > 1) {
      GB_ISSUE(1, KC)
      GB_WAIT_ALL_BUT_NEWEST();
    } else {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
  }
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc % STAGES;
    const int ahead = kc + STAGES - 1;  // the chunk issued in this iteration
    if (LOADER == 0 && ahead < nk) {
      GB_ISSUE(ahead % STAGES, ahead * KC)
    }
    if (active) {
      const unsigned char* la = lds[buf][0];
      const unsigned char* lb = lds[buf][1];
      // FP32: the chunk's 32 k-terms go to a fresh partial sum that is added to the running
      // one once per chunk (blocked summation): an output then passes through n/32 + 8
      // roundings instead of n/4 accumulating MFMAs, which keeps FP32 squares of blocks of
      // ~2000 rows well inside the 1e-6 accuracy bar after refinement.  FP64 accumulates
      // directly.
      constexpr bool kBlocked = std::is_same<T, float>::value;
      acc_t part[kBlocked ? MB : 1][kBlocked ? MB : 1];
      if constexpr (kBlocked) {
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
          for (int n = 0; n < MB; ++n) part[m][n] = acc_t{0, 0, 0, 0};
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int pc = h ? pc1 : pc0;
        T fa[MB][V], fb[MB][V];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          __builtin_memcpy(fa[m], la + pa0 + m * 16 * 128 + pc, 16);
          __builtin_memcpy(fb[m], lb + pb0 + m * 16 * 128 + pc, 16);
        }
#pragma unroll
        for (int e = 0; e < V; ++e)
#pragma unroll
          for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < MB; ++n) {
              if constexpr (kBlocked) part[m][n] = M::mma(fa[m][e], fb[n][e], part[m][n]);
              else acc[m][n] = M::mma(fa[m][e], fb[n][e], acc[m][n]);
            }
      }
      if constexpr (kBlocked) {
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
          for (int n = 0; n < MB; ++n) acc[m][n] += part[m][n];
      }
    }
    if (LOADER == 1) {
      // chunk kc + 1 (in registers) into the other buffer, then the chunk after it
      if (kc + 1 < nk) {
        GB_PUT(buf ^ 1)
      }
      if (kc + 2 < nk) {
        GB_STAGE((kc + 2) * KC)
      }
    } else if (STAGES == 3 && kc + 2 < nk) {
      // chunk kc + 1 must have landed; with three stages chunk kc + 2 may stay in flight
      GB_WAIT_ALL_BUT_NEWEST();
    } else {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
  }
#undef GB_PUT
#undef GB_STAGE
#undef GB_WAIT_ALL_BUT_NEWEST
#undef GB_ISSUE

  if (!active) return;
  T* o = out + off;
  const T* e = E + off;
  const T* xa = A + off;
  const bool do_lin = MODE == 0 && (lin_flag ? *lin_flag == 1 : lin != 0);
  const bool mirror = MODE != 3 && (bi != bj || wr < wc);
  if constexpr (std::is_same<T, float>::value && MODE == 0) {
    // FP32 layout: lane l holds rows 4(l/16) .. +3 of column l%16, one contiguous run of the
    // transposed row, so the mirrored copy (and the symmetric X read of 2X - X^2) moves as one
    // 16-byte access; row groups of four lie entirely inside or outside npad
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int n = 0; n < MB; ++n) {
        const int grow0 = bi * BT + wr * WM + m * 16 + 4 * (lane >> 4);
        const int gcol = bj * BT + wc * WM + n * 16 + r16;
        if (grow0 >= np || gcol >= np) continue;
        const int64_t qt = (int64_t)gcol * np + grow0;
        f4v v = acc[m][n];
        if (do_lin) v = 2.0f * *reinterpret_cast<const f4v*>(xa + qt) - v;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[(int64_t)(grow0 + r) * np + gcol] = v[r];
        if (mirror) *reinterpret_cast<f4v*>(o + qt) = v;
      }
    return;
  }
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < MB; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int grow = bi * BT + wr * WM + m * 16 + M::row(lane, r);
        const int gcol = bj * BT + wc * WM + n * 16 + r16;
        if (grow < np && gcol < np) {
          const int64_t q1 = (int64_t)grow * np + gcol, q2 = (int64_t)gcol * np + grow;
          T v = acc[m][n][r];
          if (MODE == 1 || MODE == 4) v = alpha * v + beta * e[q1];
          if (do_lin) v = (T)2 * xa[q1] - v;
          o[q1] = v;
          if (MODE == 4) dacc[off + q1] += cn * v;
          if (mirror) {
            o[q2] = v;
            if (MODE == 4) dacc[off + q2] += cn * v;
          }
        }
      }
}


// ---- split squaring ---------------------------------------------------------------------
// An FP32 iterate x is split into planes: bf16 ones hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid) (each remainder is exact in FP32, and hi + mid + lo = x whenever x
// is an FP32 number), or two fp16 planes of 2^14 x.  X*X is summed over the plane products
// that keep about NP*8 bits (NP = 1: hi*hi; NP = 2 (hi, lo = bf16(x - hi)): + hi*lo, lo*hi;
// NP = 3: + hi*mid, mid*hi, hi*lo, lo*hi, mid*mid) or, for the fp16 planes, hi*hi + hi*lo +
// lo*hi (about 22 bits), on the 16 x 16 x 32 matrix cores with FP32 accumulation.

// The split of two values at once, each plane's pair packed in one 32-bit word (x0 in the low
// half): one packed conversion per plane, the plane values recovered from that word (a shift or
// a mask for bf16, a conversion for fp16) for the next remainder.
// F16: two fp16 planes of 2^14 x instead (hi = fp16(2^14 x), lo = fp16(2^14 x - hi), about 22
// bits; |x| <= 1 for an iterate with its spectrum in [0, 1], so 2^14 x stays far below the fp16
// maximum and values down to ~4e-9 stay normal).  The fp16 loop keeps its FP32 iterate stored
// as x' = 2^14 x (the gather and the conversion into the loop scale it, the traces and the
// conversion out of the loop scale back, all exact powers of two), so the split needs no
// multiply: hi = fp16(x'), lo = fp16(x' - hi).  The products then carry 2^28 = 2^14 * 2^14;
// the epilogue multiplies by 2^-14 to store the next iterate, again as 2^14 times its value.
constexpr float kF16Scale = 16384.0f;                    // 2^14
constexpr float kF16Down = 6.103515625e-05f;             // 2^-14
constexpr double kF16TraceDown1 = 6.103515625e-05;       // 2^-14 (diagonal sums)
constexpr double kF16TraceDown2 = 3.7252902984619140625e-09;  // 2^-28 (sums of squares)
// neg1 is -1: passed as a value the compiler cannot see (a register), the remainder
// r - fp16(r) = fma(-1, fp16(r), r) (exact product, one rounding, as the subtraction) becomes one
// mixed-precision FMA that reads the fp16 half directly, instead of a conversion and a
// subtraction.
template <int NP, bool F16 = false>
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t* w, float neg1 = -1.0f) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  if constexpr (F16) {
    typedef _Float16 h2v __attribute__((ext_vector_type(2)));
    float r0 = x0, r1 = x1;  // the stored iterate is already 2^14 x
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const h2v h = __builtin_convertvector(f2v{r0, r1}, h2v);
      uint32_t u;
      __builtin_memcpy(&u, &h, 4);
      w[p] = u;
      if (p + 1 < NP) {
        r0 = __builtin_fmaf(neg1, (float)h[0], r0);
        r1 = __builtin_fmaf(neg1, (float)h[1], r1);
      }
    }
  } else {
    float r0 = x0, r1 = x1;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
      const bf2v h = __builtin_convertvector(f2v{r0, r1}, bf2v);
      uint32_t u;
      __builtin_memcpy(&u, &h, 4);
      w[p] = u;
      if (p + 1 < NP) {
        r0 -= __uint_as_float(u << 16);
        r1 -= __uint_as_float(u & 0xffff0000u);
      }
    }
  }
}

// Epilogue of the split kernels: the new iterate v = big + small (times 2^-28 for fp16 planes),
// or 2x - v, written at (row, col) and, off the diagonal blocks, at (col, row).  Lane l holds
// rows 4(l/16) .. 4(l/16) + 3 of column l%16 of each 16 x 16 block, so its four values are one
// contiguous run of the transposed row: the mirrored copy (and the x read by the 2x - v branch,
// X being symmetric) moves as one 16-byte access.  Rows come in groups of four and npad is a
// multiple of 64, so a group is entirely inside or outside.
template <int BT, bool F16>
__device__ __forceinline__ void split_epilogue(const f4v (&big)[BT / 32][BT / 32],
                                               const f4v (&small)[BT / 32][BT / 32],
                                               float* __restrict__ S, const float* __restrict__ X,
                                               int64_t off, int np, int bi, int bj, int wr, int wc,
                                               int lane, bool do_lin) {
  constexpr int MB = BT / 32, WT = BT / 2;
  float* o = S + off;
  const float* xa = X + off;
  const int r16 = lane & 15;
  const bool mirror = bi != bj || wr < wc;
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < MB; ++n) {
      const int grow0 = bi * BT + wr * WT + m * 16 + 4 * (lane >> 4);
      const int gcol = bj * BT + wc * WT + n * 16 + r16;
      if (grow0 >= np || gcol >= np) continue;
      const int64_t qt = (int64_t)gcol * np + grow0;  // (gcol, grow0 .. grow0 + 3)
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] = big[m][n][r] + small[m][n][r];
        if (F16) v[r] *= kF16Down;
      }
      if (do_lin) {
        const f4v xt = *reinterpret_cast<const f4v*>(xa + qt);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = 2.0f * xt[r] - v[r];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) o[(int64_t)(grow0 + r) * np + gcol] = v[r];
      if (mirror) *reinterpret_cast<f4v*>(o + qt) = f4v{v[0], v[1], v[2], v[3]};
    }
}

// Split squaring: the FP32 iterate itself is read and each lane splits the 16 bytes it loads
// into the NP planes (bf16, or fp16 of 2^14 x) while staging them into the swizzled LDS layout
// (eight 16-byte pieces per 64-byte plane row, piece index XORed with bits of the row so that
// sixteen lanes reading one piece of sixteen rows hit different banks).  X^2 is the sum of the
// plane products that keep about 8 NP bits (bf16) or 22 bits (two fp16 planes) on the 16 x 16 x
// 32 matrix cores, the leading product and the corrections in separate FP32 accumulators, added
// once at the end; the epilogue applies the SP2 update and writes only the FP32 result.  The
// next chunk is loaded into registers under the current chunk's products.  A workgroup of four
// waves (2 x 2) computes a BT x BT tile (bi <= bj) of the symmetric product, BT = 128 or 64;
// tiles and XCD order as in k_symm_mm.
template <int NP, bool F16, int BT>
__global__ __launch_bounds__(kT, 2) void k_symm_mm_split(const float* __restrict__ X,
                                                        float* __restrict__ S,
                                                        const int4* __restrict__ tiles,
                                                        const int64_t* __restrict__ offs,
                                                        const int32_t* __restrict__ stopped,
                                                        int lin,
                                                        const int32_t* __restrict__ lin_flag) {
  if (stopped && *stopped) return;
  constexpr int KC = 32;           // k per chunk (64 bytes per plane row)
  constexpr int OPB = BT * 64;     // bytes per plane and operand
  constexpr int MB = BT / 32;      // 16 x 16 blocks per wave-tile edge
  constexpr int WT = BT / 2;       // wave-tile edge
  constexpr int NQ = BT / 32;      // rows per staging thread and operand
  __shared__ __align__(1024) unsigned char lds[NP][2][OPB];
  const int4 tl = tiles[blockIdx.x];
  if (tl.x < 0) return;
  const int s = tl.x, bi = tl.y, bj = tl.z, np = tl.w;
  const int64_t off = offs[s];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  // staging: thread t moves FP32 piece c8 = t % 8 (k = 4 c8 .. 4 c8 + 3) of rows
  // t / 8 + 32 q (q < NQ) of each operand; eight threads cover one row's 128 bytes.  Rows beyond
  // np read row 0 (they only feed outputs that are never stored).
  const int c8 = tid & 7, r0 = tid >> 3;
  const float* asrc[NQ];
  const float* bsrc[NQ];
  int ldo[NQ];  // byte offset of the 8-byte run in a plane's operand array
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = r0 + 32 * q;
    const int ar = bi * BT + r, br = bj * BT + r;
    asrc[q] = X + off + (int64_t)(ar < np ? ar : 0) * np + 4 * c8;
    bsrc[q] = X + off + (int64_t)(br < np ? br : 0) * np + 4 * c8;
    ldo[q] = r * 64 + (((c8 >> 1) ^ ((r >> 2) & 3)) << 4) + (c8 & 1) * 8;
  }
  f4v big[MB][MB], small[MB][MB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < MB; ++n) {
      big[m][n] = f4v{0, 0, 0, 0};
      small[m][n] = f4v{0, 0, 0, 0};
    }
  const int g = lane >> 4, r16 = lane & 15;
  const int nk = np / KC;
  // a wave whose block lies in the padding beyond np has nothing to compute; on a diagonal tile
  // the lower-left block is the transpose of the upper-right one, which that wave writes twice
  const bool in_range = bi * BT + wr * WT < np && bj * BT + wc * WT < np;
  const bool active = in_range && !(bi == bj && wr > wc);
  const int pa0 = (wr * WT + r16) * 64, pb0 = (wc * WT + r16) * 64;
  const int pc = (g ^ ((r16 >> 2) & 3)) << 4;
  f4v stg[2][NQ];  // [operand][q]
  float neg1 = -1.0f;  // see split_pair
  asm volatile("" : "+v"(neg1));
#define GB_STAGE(k0)                                                                          \
  _Pragma("unroll") for (int q = 0; q < NQ; ++q) {                                            \
    stg[0][q] = *reinterpret_cast<const f4v*>(asrc[q] + (k0));                                \
    stg[1][q] = *reinterpret_cast<const f4v*>(bsrc[q] + (k0));                                \
  }
#define GB_FRAG(dst, plane, opnd, base, m) \
  __builtin_memcpy(&(dst), &lds[plane][opnd][(base) + (m) * 16 * 64 + pc], 16)
  GB_STAGE(0)
  for (int kc = 0; kc < nk; ++kc) {
    __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        uint32_t lo[NP], hi[NP];
        split_pair<NP, F16>(stg[o][q][0], stg[o][q][1], lo, neg1);
        split_pair<NP, F16>(stg[o][q][2], stg[o][q][3], hi, neg1);
#pragma unroll
        for (int p = 0; p < NP; ++p)
          *reinterpret_cast<uint2*>(&lds[p][o][ldo[q]]) = uint2{lo[p], hi[p]};
      }
    __syncthreads();
    if (kc + 1 < nk) {
      GB_STAGE((kc + 1) * KC)
    }
    if (active) {
      bf8v A0[MB], B0[MB];
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        GB_FRAG(A0[m], 0, 0, pa0, m);
        GB_FRAG(B0[m], 0, 1, pb0, m);
      }
#pragma unroll
      for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < MB; ++n) big[m][n] = mma_p<F16>(A0[m], B0[n], big[m][n]);
      if (NP >= 2) {
        // hi x last plane, last plane x hi (lo for NP = 2, lo for NP = 3)
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          bf8v BL;
          GB_FRAG(BL, NP - 1, 1, pb0, m);
#pragma unroll
          for (int r = 0; r < MB; ++r) small[r][m] = mma_p<F16>(A0[r], BL, small[r][m]);
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          bf8v AL;
          GB_FRAG(AL, NP - 1, 0, pa0, m);
#pragma unroll
          for (int n = 0; n < MB; ++n) small[m][n] = mma_p<F16>(AL, B0[n], small[m][n]);
        }
      }
      if (NP >= 3) {
        // hi x mid, mid x hi, mid x mid
        bf8v BM[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) GB_FRAG(BM[m], 1, 1, pb0, m);
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
          for (int n = 0; n < MB; ++n) small[m][n] = mma_p<F16>(A0[m], BM[n], small[m][n]);
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          bf8v AM;
          GB_FRAG(AM, 1, 0, pa0, m);
#pragma unroll
          for (int n = 0; n < MB; ++n) {
            small[m][n] = mma_p<F16>(AM, B0[n], small[m][n]);
            small[m][n] = mma_p<F16>(AM, BM[n], small[m][n]);
          }
        }
      }
    }
  }
#undef GB_FRAG
#undef GB_STAGE
  if (!active) return;
  split_epilogue<BT, F16>(big, small, S, X, off, np, bi, bj, wr, wc, lane,
                          lin_flag ? *lin_flag == 1 : lin != 0);
}

// ---- split squaring with the split under the products -------------------------------------
// Scheduling hints (the compiler places the named instruction classes in the given order
// within a block of straight-line code): one matrix-core instruction, n vector-ALU ones, one
// LDS read or write.
__device__ inline void sched_mfma1() { __builtin_amdgcn_sched_group_barrier(0x008, 1, 0); }
__device__ inline void sched_valu2() { __builtin_amdgcn_sched_group_barrier(0x002, 2, 0); }
__device__ inline void sched_valu4() { __builtin_amdgcn_sched_group_barrier(0x002, 4, 0); }
__device__ inline void sched_dsr1() { __builtin_amdgcn_sched_group_barrier(0x100, 1, 0); }
__device__ inline void sched_dsr8() { __builtin_amdgcn_sched_group_barrier(0x100, 8, 0); }
__device__ inline void sched_dsw1() { __builtin_amdgcn_sched_group_barrier(0x200, 1, 0); }
__device__ inline void sched_vmr4() { __builtin_amdgcn_sched_group_barrier(0x020, 4, 0); }

// fp16 x 2 planes (three products), as k_symm_mm_split<2, true, BT>, with two LDS buffers: the
// planes of chunk kc + 1 are split from registers and written to one buffer while the products
// of chunk kc read the other, the split's vector instructions and LDS writes interleaved with
// the matrix-core instructions (the first operand's split under the leading products, the
// second's under the correction products), one barrier per chunk.  Each operand's next chunk
// is loaded into registers once its split has consumed them.  The two buffers are separate
// arrays and the loop is unrolled by two, so reads of one and writes of the other are known
// not to alias.  Products, their order and the accumulators are those of k_symm_mm_split, so
// both give the same bits.
template <int BT>
__global__ __launch_bounds__(kT, 2) void k_symm_mm_split_il(const float* __restrict__ X,
                                                           float* __restrict__ S,
                                                           const int4* __restrict__ tiles,
                                                           const int64_t* __restrict__ offs,
                                                           const int32_t* __restrict__ stopped,
                                                           int lin,
                                                           const int32_t* __restrict__ lin_flag) {
  if (stopped && *stopped) return;
  constexpr int NP = 2;
  constexpr int KC = 32;           // k per chunk (64 bytes per plane row)
  constexpr int OPB = BT * 64;     // bytes per plane and operand
  constexpr int MB = BT / 32;      // 16 x 16 blocks per wave-tile edge
  constexpr int WT = BT / 2;       // wave-tile edge
  constexpr int NQ = BT / 32;      // rows per staging thread and operand
  __shared__ __align__(1024) unsigned char lds0[NP][2][OPB];
  __shared__ __align__(1024) unsigned char lds1[NP][2][OPB];
  const int4 tl = tiles[blockIdx.x];
  if (tl.x < 0) return;
  const int s = tl.x, bi = tl.y, bj = tl.z, np = tl.w;
  const int64_t off = offs[s];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int c8 = tid & 7, r0 = tid >> 3;
  // 32-bit element offsets into the block (np^2 < 2^31) from one workgroup-uniform base
  const float* xblk = X + off;
  int asrc[NQ], bsrc[NQ], ldo[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = r0 + 32 * q;
    const int ar = bi * BT + r, br = bj * BT + r;
    asrc[q] = (ar < np ? ar : 0) * np + 4 * c8;
    bsrc[q] = (br < np ? br : 0) * np + 4 * c8;
    ldo[q] = r * 64 + (((c8 >> 1) ^ ((r >> 2) & 3)) << 4) + (c8 & 1) * 8;
  }
  f4v big[MB][MB], small[MB][MB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < MB; ++n) {
      big[m][n] = f4v{0, 0, 0, 0};
      small[m][n] = f4v{0, 0, 0, 0};
    }
  const int g = lane >> 4, r16 = lane & 15;
  const int nk = np / KC;
  const bool in_range = bi * BT + wr * WT < np && bj * BT + wc * WT < np;
  const bool active = in_range && !(bi == bj && wr > wc);
  const int pa0 = (wr * WT + r16) * 64, pb0 = (wc * WT + r16) * 64;
  const int pc = (g ^ ((r16 >> 2) & 3)) << 4;
  f4v stg[2][NQ];  // [operand][q]
  float neg1 = -1.0f;  // see split_pair
  asm volatile("" : "+v"(neg1));
  auto load_op = [&](int o, int k0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      stg[o][q] = *reinterpret_cast<const f4v*>(xblk + (o ? bsrc[q] : asrc[q]) + k0);
  };
  // the split of operand o, row groups q0 .. q0 + nq - 1, into dst
  auto split_op = [&](int o, unsigned char (&dst)[NP][2][OPB], int q0, int nq) {
#pragma unroll
    for (int q = q0; q < q0 + nq; ++q) {
      // an empty statement the value passes through, so that the split stays where it is
      // written (the same code on both sides of the `active` branch would otherwise be hoisted
      // above it, waiting for every load at the top of the chunk)
      asm volatile("" : "+v"(stg[o][q]));
      uint32_t lo[NP], hi[NP];
      split_pair<NP, true>(stg[o][q][0], stg[o][q][1], lo, neg1);
      split_pair<NP, true>(stg[o][q][2], stg[o][q][3], hi, neg1);
#pragma unroll
      for (int p = 0; p < NP; ++p)
        *reinterpret_cast<uint2*>(&dst[p][o][ldo[q]]) = uint2{lo[p], hi[p]};
    }
  };
  // one chunk: products from `cur`, the next chunk's planes into `nxt`, then the chunk after
  // that (k element k2) into registers; past the end k2 repeats the last chunk, just read by
  // the same lanes (a cache hit), whose planes are never written (no branch inside the
  // interleaved code)
  auto step = [&](unsigned char (&cur)[NP][2][OPB], unsigned char (&nxt)[NP][2][OPB], int k2) {
    if (active) {
      bf8v A0[MB], B0[MB];
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        __builtin_memcpy(&A0[m], &cur[0][0][pa0 + m * 16 * 64 + pc], 16);
        __builtin_memcpy(&B0[m], &cur[0][1][pb0 + m * 16 * 64 + pc], 16);
      }
#pragma unroll
      for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < MB; ++n) big[m][n] = mma_f16(A0[m], B0[n], big[m][n]);
      split_op(0, nxt, 0, NQ);
      // 2 MB fragment reads, then MB^2 products each with four split instructions, and one
      // plane write (both planes of a row group) per MB^2 / NQ products
      sched_dsr8();
#pragma unroll
      for (int i = 0; i < MB * MB; ++i) {
        sched_mfma1();
        sched_valu4();
        if (i % (MB * MB / NQ) == MB * MB / NQ - 1) sched_dsw1();
      }
      load_op(0, k2);
      sched_vmr4();  // the next loads after the split that frees their registers
      // the second operand's split in two halves, under the hi x lo and the lo x hi products
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        bf8v BL;
        __builtin_memcpy(&BL, &cur[1][1][pb0 + m * 16 * 64 + pc], 16);
#pragma unroll
        for (int r = 0; r < MB; ++r) small[r][m] = mma_f16(A0[r], BL, small[r][m]);
      }
      split_op(1, nxt, 0, NQ / 2);
#pragma unroll
      for (int i = 0; i < MB * MB; ++i) {
        if (i % MB == 0) sched_dsr1();
        sched_mfma1();
        sched_valu2();
        if (i % (2 * MB * MB / NQ) == 2 * MB * MB / NQ - 1) sched_dsw1();
      }
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        bf8v AL;
        __builtin_memcpy(&AL, &cur[1][0][pa0 + m * 16 * 64 + pc], 16);
#pragma unroll
        for (int n = 0; n < MB; ++n) small[m][n] = mma_f16(AL, B0[n], small[m][n]);
      }
      split_op(1, nxt, NQ / 2, NQ / 2);
#pragma unroll
      for (int i = 0; i < MB * MB; ++i) {
        if (i % MB == 0) sched_dsr1();
        sched_mfma1();
        sched_valu2();
        if (i % (2 * MB * MB / NQ) == 2 * MB * MB / NQ - 1) sched_dsw1();
      }
      load_op(1, k2);
      sched_vmr4();
    } else {
      split_op(0, nxt, 0, NQ);
      split_op(1, nxt, 0, NQ);
      load_op(0, k2);
      load_op(1, k2);
    }
    __syncthreads();
  };
  load_op(0, 0);
  load_op(1, 0);
  split_op(0, lds0, 0, NQ);
  split_op(1, lds0, 0, NQ);
  if (nk > 1) {
    load_op(0, KC);
    load_op(1, KC);
  }
  __syncthreads();
  // the planes written past the last chunk are never read
  for (int kc = 0; kc < nk; kc += 2) {
    step(lds0, lds1, min(kc + 2, nk - 1) * KC);
    if (kc + 1 < nk) step(lds1, lds0, min(kc + 3, nk - 1) * KC);
  }
  if (!active) return;
  split_epilogue<BT, true>(big, small, S, X, off, np, bi, bj, wr, wc, lane,
                           lin_flag ? *lin_flag == 1 : lin != 0);
}

// ---- traces and the branch decision --------------------------------------------------------
// t1 = sum over subgraphs of the core diagonal of X; t2 = the same for X^2, which for the
// symmetric X is the sum of the squared entries of the core rows.  Taking t2 from X lets the
// stop test and the branch come before the square: the last square of the loop is not
// needed, and the square kernel applies the update in its epilogue.  One workgroup per
// subgraph writes its two partial sums (fixed order); one workgroup adds them (fixed order)
// and decides.
struct StepRec {
  double t1, t2, e, margin;
  int32_t b, stop, pad0, pad1;
};

template <typename T>
__global__ __launch_bounds__(kT) void k_trace_rows(const T* __restrict__ X,
                                                   const int64_t* __restrict__ offs,
                                                   const int32_t* __restrict__ npad,
                                                   const int32_t* __restrict__ core_ptr,
                                                   double* __restrict__ part,
                                                   const int32_t* __restrict__ stopped,
                                                   double s1, double s2) {
  if (stopped && *stopped) return;
  constexpr int V = 16 / sizeof(T);  // values per 16-byte load
  typedef T vec __attribute__((ext_vector_type(V)));
  __shared__ double r1[kT], r2[kT];
  const int s = blockIdx.x;
  const int np = npad[s], k = core_ptr[s + 1] - core_ptr[s];
  const int nv = np / V;  // np is a multiple of 64
  const T* xs = X + offs[s];
  double p1 = 0.0, p2 = 0.0;
  // 16-byte loads, four rows at a time, so that each thread has several loads in flight; the
  // thread whose load holds element (j, j) adds it to the diagonal sum
  auto row_sums = [&](int j, const vec& v, int a) {
#pragma unroll
    for (int e = 0; e < V; ++e) p2 += (double)v[e] * (double)v[e];
    if (a == j / V) p1 += (double)v[j % V];
  };
  int j = 0;
  for (; j + 4 <= k; j += 4) {
    const vec* r0 = reinterpret_cast<const vec*>(xs + (int64_t)j * np);
    const vec* r1p = reinterpret_cast<const vec*>(xs + (int64_t)(j + 1) * np);
    const vec* r2p = reinterpret_cast<const vec*>(xs + (int64_t)(j + 2) * np);
    const vec* r3p = reinterpret_cast<const vec*>(xs + (int64_t)(j + 3) * np);
    for (int a = threadIdx.x; a < nv; a += kT) {
      const vec v0 = r0[a], v1 = r1p[a], v2 = r2p[a], v3 = r3p[a];
      row_sums(j, v0, a);
      row_sums(j + 1, v1, a);
      row_sums(j + 2, v2, a);
      row_sums(j + 3, v3, a);
    }
  }
  for (; j < k; ++j) {
    const vec* r0 = reinterpret_cast<const vec*>(xs + (int64_t)j * np);
    for (int a = threadIdx.x; a < nv; a += kT) row_sums(j, r0[a], a);
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
    part[2 * s] = r1[0] * s1;
    part[2 * s + 1] = r2[0] * s2;
  }
}

__device__ void sum_partials(const double* __restrict__ part, int n_sub, double* t1, double* t2) {
  __shared__ double r1[kT], r2[kT];
  double p1 = 0.0, p2 = 0.0;
  for (int s = threadIdx.x; s < n_sub; s += kT) {
    p1 += part[2 * s];
    p2 += part[2 * s + 1];
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
  *t1 = r1[0];
  *t2 = r2[0];
}

// forced: -1 choose by the trace rule, 0/1 replay that branch, 2 stop (record only),
// 10/11 take branch 0/1 unless the stop test holds (alternating refinement)
__global__ __launch_bounds__(kT) void k_decide(const double* __restrict__ part, int n_sub,
                                               double n_occ, double tol, int forced, int at_max,
                                               StepRec* __restrict__ rec) {
  double t1, t2;
  sum_partials(part, n_sub, &t1, &t2);
  if (threadIdx.x == 0) {
    const double e = fabs(t1 - t2);
    const double dsq = fabs(t2 - n_occ), dlin = fabs(2.0 * t1 - t2 - n_occ);
    StepRec q;
    q.t1 = t1;
    q.t2 = t2;
    q.e = e;
    q.margin = fabs(dsq - dlin);
    q.pad0 = q.pad1 = 0;
    q.b = -1;
    q.stop = 0;
    if (forced == 2) q.stop = 1;
    else if (forced >= 10 && e <= tol) q.stop = 1;
    else if (forced >= 10 && at_max) q.stop = 2;
    else if (forced >= 10) q.b = forced - 10;
    else if (forced >= 0) q.b = forced;
    else if (e <= tol) q.stop = 1;
    else if (at_max) q.stop = 2;
    else q.b = dsq < dlin ? 0 : 1;
    *rec = q;
  }
}

// ---- device-driven loop (hipGraph): the stop flag, iteration counter, current branch and
// records live on the device, so a captured pair of iterations can be replayed without host
// round trips.  Every update writes the new iterate into the other buffer, so buffer roles
// simply alternate.
struct LoopState {
  int32_t it, stopped, max_iter, n_forced;  // n_forced < 0: choose by the trace rule
  int32_t stag, cur_b, it0;  // it0: first step of this loop (stagnation looks back 2 steps)
  double n_occ, tol;
  uint8_t forced[128];
  StepRec recs[128];
};
// The loop's parameters, passed by value to the kernel that sets up LoopState.
struct LoopInit {
  int32_t it0, max_iter, n_forced, stag;
  double n_occ, tol;
  uint8_t forced[128];
};

__global__ __launch_bounds__(kT) void k_decide_dev(const double* __restrict__ part, int n_sub,
                                                   LoopState* __restrict__ st) {
  if (st->stopped) return;
  double t1, t2;
  sum_partials(part, n_sub, &t1, &t2);
  if (threadIdx.x == 0) {
    const int it = st->it;
    const double n_occ = st->n_occ;
    const double e = fabs(t1 - t2);
    const double dsq = fabs(t2 - n_occ), dlin = fabs(2.0 * t1 - t2 - n_occ);
    StepRec q;
    q.t1 = t1;
    q.t2 = t2;
    q.e = e;
    q.margin = fabs(dsq - dlin);
    q.pad0 = q.pad1 = 0;
    q.b = -1;
    q.stop = 0;
    if (it >= 127) {
      q.stop = st->n_forced >= 0 ? 1 : 2;  // the records hold 128 steps
    } else if (st->n_forced >= 0) {
      if (it >= st->n_forced) q.stop = 1;
      else q.b = st->forced[it];
    } else if (e <= st->tol) {
      q.stop = 1;
    } else if (it >= st->max_iter) {
      q.stop = 2;
    } else if (st->stag && it - st->it0 >= 9 && e > st->recs[it - 2].e) {
      q.stop = 4;
    } else {
      q.b = dsq < dlin ? 0 : 1;
    }
    st->recs[it] = q;
    st->cur_b = q.b;
    if (q.stop) st->stopped = 1;
    else st->it = it + 1;
  }
}

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, int64_t n, TO scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = i; p < n; p += stride) out[p] = (TO)in[p] * scale;
}

// The FP32 iterate made exactly symmetric in place: the split and FP32 squares compute both
// triangles only inside the 64 x 64 tiles on the diagonal of a block (everything else is
// computed once and mirrored), pairing the planes of an entry and of its transpose
// differently there, so X is symmetric only to rounding inside those tiles; the FP64
// refinement relies on symmetry.  Each such tile becomes (T + T^T)/2, formed in FP64 and
// rounded once (an entry and its transpose round the same sum).  One workgroup per diagonal
// tile, read once through LDS.
__global__ __launch_bounds__(256) void k_sym_diag(float* __restrict__ X,
                                                  const int64_t* __restrict__ offs,
                                                  const int32_t* __restrict__ npad) {
  __shared__ float t[64][65];
  const int s = blockIdx.y, b = blockIdx.x;
  const int np = npad[s];
  if (b * 64 >= np) return;  // the whole workgroup leaves together
  float* x = X + offs[s] + (int64_t)(b * 64) * np + b * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) t[e >> 6][e & 63] = x[(int64_t)(e >> 6) * np + (e & 63)];
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    x[(int64_t)r * np + c] = (float)(0.5 * ((double)t[r][c] + (double)t[c][r]));
  }
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

// ---- core rows of a polynomial in X (FP64 refinement on the rows D keeps) -----------------
// A "row slab" holds k_s rows of width np_s per subgraph at soffs[s] (row stride np_s), the
// same layout as the first k_s rows of a block, so the trace, check and scatter kernels read a
// slab as they read a block.  Since X is symmetric, the core rows of q(X) are the transposed
// core columns, and V q(X) for a slab V needs only products V X.

// W = (scale V) X on the FP64 matrix cores (scale a power of two, applied exactly to V's entries
// as they are loaded: the stored iterate may be X / scale): a wave computes all KMAX rows of 64
// columns of W
// (KMAX/16 x 4 tiles of 16 x 16, v_mfma_f64_16x16x4) and walks the reduction in chunks of 16
// rows of X.  Within a chunk, lane l (i = l%16, q = l/16) takes the four consecutive rows
// a + 4q + u, u = the MFMA index: its A operands of a row tile are one 32-byte run of V
// (V[16m + i][a + 4q .. a + 4q + 3]), and its B operands are 16-byte pairs of columns
// (X[a + 4q + u][c + 32g + 2i, +1]; tile 2g + h holds the columns of parity h of group g), so a
// chunk costs a wave 4 + 8 wide loads for 32 MFMAs.  X is read once; V (a few hundred KB per
// block) comes from L2: the workgroups are numbered so that all column blocks of a subgraph run
// on one XCD (workgroup i goes to XCD i mod 8), which fetches V into its L2 once.  Rows of V
// beyond k_s are read in bounds (row k_s - 1) and zeroed by a select, keeping the loop free of
// branches.  Output register r of lane l holds row 4r + q of its tile.
template <int KMAX, typename TX>
__global__ __launch_bounds__(256) void k_rows_mm(const TX* __restrict__ X,
                                                 const int64_t* __restrict__ offs,
                                                 const int32_t* __restrict__ npad,
                                                 const double* __restrict__ V,
                                                 double* __restrict__ W,
                                                 const int64_t* __restrict__ soffs,
                                                 const int32_t* __restrict__ core_ptr,
                                                 int n_sub, int colblocks, double scale) {
  using M = Mfma<double>;
  constexpr int MT = KMAX / 16, NT = 4, U = 4;
  const int id = blockIdx.x, q8 = id >> 3;
  const int s = (id & 7) + 8 * (q8 / colblocks), cb = q8 % colblocks;
  if (s >= n_sub) return;  // the grid covers n_sub rounded up to 8
  const int np = npad[s];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cw = cb * 256 + wave * 64;
  if (cw >= np) return;  // np is a multiple of 64: a wave is wholly inside or outside
  const int k = core_ptr[s + 1] - core_ptr[s];
  const int i16 = lane & 15, kq = lane >> 4;
  M::acc_t acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[m][n] = M::acc_t{0, 0, 0, 0};
  bool rows_in[MT];
  int64_t roff[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    rows_in[m] = m * 16 + i16 < k;
    roff[m] = (int64_t)min(m * 16 + i16, k - 1) * np;
  }
  const double* vb = V + soffs[s] + 4 * kq;
  const TX* xb = X + offs[s] + (int64_t)(4 * kq) * np + cw + 2 * i16;
  for (int a0 = 0; a0 < np; a0 += 16) {  // np is a multiple of 64
    double fa[U][MT], fb[U][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const double2* pv = reinterpret_cast<const double2*>(vb + roff[m] + a0);
      const double2 v0 = pv[0], v1 = pv[1];
      fa[0][m] = rows_in[m] ? v0.x * scale : 0.0;
      fa[1][m] = rows_in[m] ? v0.y * scale : 0.0;
      fa[2][m] = rows_in[m] ? v1.x * scale : 0.0;
      fa[3][m] = rows_in[m] ? v1.y * scale : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        if constexpr (std::is_same<TX, double>::value) {
          const double2 xv = *reinterpret_cast<const double2*>(xb + (int64_t)(a0 + u) * np + 32 * g);
          fb[u][2 * g] = xv.x;
          fb[u][2 * g + 1] = xv.y;
        } else {  // an FP32 X (exact in FP64): half the bytes per product
          const float2 xv = *reinterpret_cast<const float2*>(xb + (int64_t)(a0 + u) * np + 32 * g);
          fb[u][2 * g] = (double)xv.x;
          fb[u][2 * g + 1] = (double)xv.y;
        }
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = M::mma(fa[u][m], fb[u][n], acc[m][n]);
  }
  double* wb = W + soffs[s] + cw + 2 * i16;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = m * 16 + M::row(lane, r);
      if (j < k) {
#pragma unroll
        for (int g = 0; g < 2; ++g)
          *reinterpret_cast<double2*>(wb + (int64_t)j * np + 32 * g) =
              double2{acc[m][2 * g][r], acc[m][2 * g + 1][r]};
      }
    }
}

// W = the first k_s rows of X (= E X for the core unit rows E), times scale (a power of two)
template <typename TX>
__global__ __launch_bounds__(256) void k_rows_copy(const TX* __restrict__ X,
                                                   const int64_t* __restrict__ offs,
                                                   const int32_t* __restrict__ npad,
                                                   double* __restrict__ W,
                                                   const int64_t* __restrict__ soffs,
                                                   const int32_t* __restrict__ core_ptr,
                                                   double scale) {
  const int s = blockIdx.y;
  const int np = npad[s], k = core_ptr[s + 1] - core_ptr[s];
  const int64_t n = (int64_t)k * np;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
    W[soffs[s] + p] = (double)X[offs[s] + p] * scale;
}

// out = a x + b y over a whole slab (flat)
__global__ void k_lin2(double* __restrict__ out, double a, const double* __restrict__ x, double b,
                       const double* __restrict__ y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    out[p] = a * x[p] + b * y[p];
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


// ---- adjoint kernels ------------------------------------------------------------------------
__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = i; q < n; q += stride) p[q] = v;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Gbar_K of every block from dL/dD on D's column-ELL pattern, symmetrised:
// Gbar[a][j] = (G(a, j) + G(j, a)) / 2 with G(a, j) = dL/dD[sub_a, sub_j] on core columns j.
__global__ __launch_bounds__(kT) void k_seed(const double* __restrict__ gval, int gw,
                                             const int32_t* __restrict__ core_ptr,
                                             const int32_t* __restrict__ sub_ptr,
                                             const int32_t* __restrict__ sub_idx,
                                             const int32_t* __restrict__ sub_pos,
                                             const int64_t* __restrict__ offs,
                                             const int32_t* __restrict__ npad,
                                             double* __restrict__ G) {
  const int s = blockIdx.x;
  const int b = sub_ptr[s], n = sub_ptr[s + 1] - b, k = core_ptr[s + 1] - core_ptr[s];
  const int np = npad[s];
  double* g = G + offs[s];
  for (int64_t p = threadIdx.x; p < (int64_t)n * k; p += kT) {
    const int a = (int)(p / k), j = (int)(p - (int64_t)a * k);
    double v = gval[(int64_t)sub_idx[b + j] * gw + sub_pos[b + a]];
    if (a < k) v += gval[(int64_t)sub_idx[b + a] * gw + sub_pos[b + j]];
    v *= 0.5;
    g[(int64_t)a * np + j] = v;
    if (a >= k) g[(int64_t)j * np + a] = v;
  }
}

// out = c1 (P + P^T) + c2 G per block, through a 32 x 32 LDS transpose
__global__ __launch_bounds__(256) void k_sym_combine(const double* __restrict__ P,
                                                     const double* __restrict__ G,
                                                     double* __restrict__ out, double c1, double c2,
                                                     const int64_t* __restrict__ offs,
                                                     const int32_t* __restrict__ npad, int max_nt) {
  __shared__ double t[32][33];
  const int s = blockIdx.y;
  const int np = npad[s], nt = np / 32;
  const int bx = blockIdx.x % max_nt, by = blockIdx.x / max_nt;
  if (bx >= nt || by >= nt) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double* p = P + offs[s];
  for (int r = ty; r < 32; r += 8) t[r][tx] = p[(int64_t)(bx * 32 + r) * np + by * 32 + tx];
  __syncthreads();
  const double* g = G + offs[s];
  double* o = out + offs[s];
  for (int r = ty; r < 32; r += 8) {
    const int64_t q = (int64_t)(by * 32 + r) * np + bx * 32 + tx;
    o[q] = c1 * (p[q] + t[tx][r]) + c2 * g[q];
  }
}

// vertex -> subgraphs holding it: counts, fill, per-vertex sort by subgraph
__global__ void k_vs_count(const int32_t* __restrict__ sub_ptr, const int32_t* __restrict__ sub_idx,
                           int32_t* __restrict__ cnt) {
  const int s = blockIdx.x;
  for (int p = sub_ptr[s] + threadIdx.x; p < sub_ptr[s + 1]; p += blockDim.x)
    atomicAdd(&cnt[sub_idx[p]], 1);
}
__global__ void k_vs_fill(const int32_t* __restrict__ sub_ptr, const int32_t* __restrict__ sub_idx,
                          const int32_t* __restrict__ vs_ptr, int32_t* __restrict__ fill,
                          int32_t* __restrict__ vs_sub, int32_t* __restrict__ vs_loc) {
  const int s = blockIdx.x;
  for (int p = sub_ptr[s] + threadIdx.x; p < sub_ptr[s + 1]; p += blockDim.x) {
    const int v = sub_idx[p];
    const int q = vs_ptr[v] + atomicAdd(&fill[v], 1);
    vs_sub[q] = s;
    vs_loc[q] = p - sub_ptr[s];
  }
}
__global__ void k_vs_sort(int n, const int32_t* __restrict__ vs_ptr, int32_t* __restrict__ vs_sub,
                          int32_t* __restrict__ vs_loc) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  for (int p = vs_ptr[v] + 1; p < vs_ptr[v + 1]; ++p) {
    const int ks = vs_sub[p], kl = vs_loc[p];
    int q = p - 1;
    while (q >= vs_ptr[v] && vs_sub[q] > ks) {
      vs_sub[q + 1] = vs_sub[q];
      vs_loc[q + 1] = vs_loc[q];
      --q;
    }
    vs_sub[q + 1] = ks;
    vs_loc[q + 1] = kl;
  }
}

// dL/dH per ELL slot (i, j): sum over the subgraphs holding both i and j, ascending, of
// scale * Gbar_0[loc(i)][loc(j)]
__global__ void k_assemble(const int32_t* __restrict__ hcol, int n, int w,
                           const int32_t* __restrict__ vs_ptr, const int32_t* __restrict__ vs_sub,
                           const int32_t* __restrict__ vs_loc, const int64_t* __restrict__ offs,
                           const int32_t* __restrict__ npad, const double* __restrict__ G0,
                           double scale, double* __restrict__ gh) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * w) return;
  const int i = (int)(q / w);
  const int j = hcol[q];
  if ((unsigned)j >= (unsigned)n) {
    gh[q] = 0.0;
    return;
  }
  int pi = vs_ptr[i], ei = vs_ptr[i + 1], pj = vs_ptr[j], ej = vs_ptr[j + 1];
  double acc = 0.0;
  while (pi < ei && pj < ej) {
    const int si = vs_sub[pi], sj = vs_sub[pj];
    if (si < sj) ++pi;
    else if (sj < si) ++pj;
    else {
      const double g = G0[offs[si] + (int64_t)vs_loc[pi] * npad[si] + vs_loc[pj]];
      acc = acc + scale * g;
      ++pi;
      ++pj;
    }
  }
  gh[q] = acc;
}

int grid_for(int64_t n, int t, int cap = 1 << 20) {
  const int64_t b = (n + t - 1) / t;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// ---- plan: padded sizes, offsets, tile lists ---------------------------------------------
// Square tiles are listed 128-edge tiles first, then 64-edge tiles; within each group the
// largest blocks come first (most k work per tile).
// Kernel variants of the batched products, one code per subgraph: 128 (128-edge tiles, two LDS
// stages), 64 (64-edge, two stages), 63 (64-edge, three stages), 62 (64-edge, two stages,
// register-staged loads); split squares: 128 and 64, and for fp16 planes 129 and 65 (128- and
// 64-edge tiles with the split under the products, k_symm_mm_split_il).
constexpr int kNVar = 6;
constexpr int kVariants[kNVar] = {128, 64, 63, 62, 129, 65};
inline int variant_edge(int code) { return code >= 128 ? 128 : 64; }
inline bool split_il_code(int code) { return code == 129 || code == 65; }
inline int variant_index(int code) {
  for (int v = 0; v < kNVar; ++v)
    if (kVariants[v] == code) return v;
  return -1;
}

// tiles per variant group (launch order as kVariants)
struct Groups {
  int n[kNVar] = {};
};

struct Plan {
  int n_sub = 0;
  std::vector<int32_t> npad;
  std::vector<int64_t> off;
  std::vector<int> bt;           // kernel variant code chosen for each subgraph
  int64_t total = 0;
  std::vector<int4> tiles;       // bi <= bj (symmetric products), grouped by variant
  Groups tg;                     //   (subgraph-major; per-subgraph launches use `ranges`)
  std::vector<int4> launch;      // the same tiles as launched in one batch, each variant group
  Groups lg;                     //   in XCD order
  std::vector<int4> tiles_full;  // every (bi, bj) with edge 128 (general products)
  std::vector<int4> full_launch; // the same in XCD order (the launch list of general products)
  std::vector<int4> ranges;      // per subgraph: first tile, tile count, variant code, s
  std::vector<int4> idem;        // 128-edge upper tiles covering the core rows (final check)
  double flops_alg = 0, flops_exec = 0;
  int max_npad = 0;
};

// XCD-aware order: the hardware hands workgroup b to XCD b % 8.  Whole subgraphs are dealt to
// the eight XCD queues (greedy, costliest first, onto the least loaded queue) and the queues
// are interleaved, so every tile of a subgraph runs on one XCD and its row panels stay in that
// XCD's L2.  Queues are padded to equal length with empty entries (subgraph -1).
constexpr int kXcd = 8;

void xcd_order(std::vector<int4>& out, const std::vector<int4>& tiles,
               const std::vector<int4>& ranges, size_t r0, size_t r1) {
  if (r1 <= r0) return;
  std::vector<std::vector<int4>> q(kXcd);
  std::vector<double> load(kXcd, 0.0);
  for (size_t r = r0; r < r1; ++r) {
    const int4 rg = ranges[r];
    int best = 0;
    for (int x = 1; x < kXcd; ++x)
      if (load[x] < load[best]) best = x;
    for (int t = 0; t < rg.y; ++t) q[best].push_back(tiles[rg.x + t]);
    load[best] += (double)rg.y * tiles[rg.x].w;
  }
  size_t len = 0;
  for (auto& v : q) len = std::max(len, v.size());
  const size_t base = out.size();
  out.resize(base + len * kXcd, make_int4(-1, 0, 0, 0));
  for (int x = 0; x < kXcd; ++x)
    for (size_t j = 0; j < q[x].size(); ++j) out[base + j * kXcd + x] = q[x][j];
}

Plan make_plan(const Part& P, const std::vector<int>* bt = nullptr, bool xcd = true) {
  Plan pl;
  pl.n_sub = P.n_sub;
  pl.npad.resize(P.n_sub);
  pl.off.resize(P.n_sub);
  pl.bt.assign(P.n_sub, kBT);
  if (bt) pl.bt = *bt;
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
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return pl.npad[a] > pl.npad[b]; });
  size_t r_first[kNVar + 1] = {};
  for (int v = 0; v < kNVar; ++v) {
    const int code = kVariants[v], edge = variant_edge(code);
    const int t0 = (int)pl.tiles.size();
    r_first[v] = pl.ranges.size();
    for (int s : order) {
      if (pl.bt[s] != code) continue;
      const int np = pl.npad[s];
      const int nb = (np + edge - 1) / edge;
      const int first = (int)pl.tiles.size();
      const int wt = edge / 2;  // wave tile edge (2 x 2 waves per tile)
      for (int bi = 0; bi < nb; ++bi)
        for (int bj = bi; bj < nb; ++bj) {
          pl.tiles.push_back(make_int4(s, bi, bj, np));
          // matrix-core work the tile executes: every wave whose block lies inside npad, except
          // the lower-left one of a diagonal tile
          for (int wr = 0; wr < 2; ++wr)
            for (int wc = 0; wc < 2; ++wc)
              if (bi * edge + wr * wt < np && bj * edge + wc * wt < np && !(bi == bj && wr > wc))
                pl.flops_exec += 2.0 * wt * wt * (double)np;
        }
      pl.ranges.push_back(make_int4(first, (int)pl.tiles.size() - first, code, s));
    }
    pl.tg.n[v] = (int)pl.tiles.size() - t0;
  }
  r_first[kNVar] = pl.ranges.size();
  // launch list of the batched squaring: each group in XCD order (or as listed)
  if (xcd) {
    for (int v = 0; v < kNVar; ++v) {
      const size_t before = pl.launch.size();
      xcd_order(pl.launch, pl.tiles, pl.ranges, r_first[v], r_first[v + 1]);
      pl.lg.n[v] = (int)(pl.launch.size() - before);
    }
  } else {
    pl.launch = pl.tiles;
    pl.lg = pl.tg;
  }
  std::vector<int4> full_ranges;
  for (int s : order) {
    const int np = pl.npad[s];
    const int nb = (np + kBT - 1) / kBT;
    const int k = P.h_core_ptr[s + 1] - P.h_core_ptr[s];
    const int first = (int)pl.tiles_full.size();
    for (int bi = 0; bi < nb; ++bi)
      for (int bj = 0; bj < nb; ++bj) {
        pl.tiles_full.push_back(make_int4(s, bi, bj, np));
        if (bj >= bi && bi * kBT < k) pl.idem.push_back(make_int4(s, bi, bj, np));
      }
    full_ranges.push_back(make_int4(first, (int)pl.tiles_full.size() - first, 128, s));
  }
  // the general-product tiles in XCD order (queues padded with empty entries) or as listed
  if (xcd) xcd_order(pl.full_launch, pl.tiles_full, full_ranges, 0, full_ranges.size());
  else pl.full_launch = pl.tiles_full;
  return pl;
}

}  // namespace

struct TapeData {
  int N = 0, K = 0, stride = 4, max_sub = 0;
  double emin = 0, emax = 0;
  std::vector<uint8_t> branch;
  Plan pl;
  DBuf<int64_t> offs;
  DBuf<int32_t> npad;
  DBuf<int4> tiles, tiles_full;
  DBuf<int32_t> core_ptr, sub_ptr, sub_idx, sub_pos;
  std::vector<DBuf<double>> ckpt;  // X_0, X_stride, X_2stride, ...
};

namespace {

// One batched symmetric product over the variant groups of a tile list (see k_symm_mm).
template <typename T, int MODE>
void launch_symm(const T* A, const T* B, const T* E, T* out, T alpha, T beta, const int4* tiles,
                 const Groups& g, const int64_t* offs, hipStream_t s,
                 const int32_t* stopped = nullptr, int lin = 0,
                 const int32_t* lin_flag = nullptr, T* dacc = nullptr, T cn = (T)0) {
  if (g.n[4] > 0 || g.n[5] > 0) fail(GB_EHIP, "split-square tiles given to an FP64/FP32 product");
  const int4* t = tiles;
  if (g.n[0] > 0)
    hipLaunchKernelGGL((k_symm_mm<T, MODE, 128, 2>), dim3(g.n[0]), dim3(kT), 0, s, A, B, E, out,
                       alpha, beta, t, offs, stopped, lin, lin_flag, dacc, cn);
  t += g.n[0];
  if (g.n[1] > 0)
    hipLaunchKernelGGL((k_symm_mm<T, MODE, 64, 2>), dim3(g.n[1]), dim3(kT), 0, s, A, B, E, out,
                       alpha, beta, t, offs, stopped, lin, lin_flag, dacc, cn);
  t += g.n[1];
  if (g.n[2] > 0)
    hipLaunchKernelGGL((k_symm_mm<T, MODE, 64, 3>), dim3(g.n[2]), dim3(kT), 0, s, A, B, E, out,
                       alpha, beta, t, offs, stopped, lin, lin_flag, dacc, cn);
  t += g.n[2];
  if (g.n[3] > 0)
    hipLaunchKernelGGL((k_symm_mm<T, MODE, 64, 2, 1>), dim3(g.n[3]), dim3(kT), 0, s, A, B, E,
                       out, alpha, beta, t, offs, stopped, lin, lin_flag, dacc, cn);
  GB_LAUNCH_CHECK();
}

// One SP2 step on a tile list: the new iterate X^2 (lin = 0) or 2X - X^2 (lin = 1), or the
// branch read from *lin_flag on the device-driven loop.
template <typename T>
void launch_square(const T* X, T* S, const int4* tiles, const Groups& g, const int64_t* offs,
                   hipStream_t s, int lin = 0, const int32_t* stopped = nullptr,
                   const int32_t* lin_flag = nullptr) {
  launch_symm<T, 0>(X, X, X, S, (T)1, (T)0, tiles, g, offs, s, stopped, lin, lin_flag);
}

// a single group (the idempotency check's 128-edge tiles, one subgraph's range)
inline Groups one_group(int code, int count) {
  Groups g;
  g.n[variant_index(code)] = count;
  return g;
}

// the same with split squares (FP32 iterate X -> new FP32 iterate S; `planes` 1-3 bf16 planes
// or 4 = two fp16 planes), 128-edge tiles first, then 64-edge tiles
template <int NP, bool F16>
void launch_split_np(const float* X, float* S, const int4* tiles, const Groups& g,
                     const int64_t* offs, hipStream_t s, int lin, const int32_t* stopped,
                     const int32_t* lin_flag) {
  if (g.n[2] > 0 || g.n[3] > 0) fail(GB_EHIP, "split squares take 128- or 64-edge tiles only");
  const int4* t = tiles;
  if (g.n[0] > 0)
    hipLaunchKernelGGL((k_symm_mm_split<NP, F16, 128>), dim3(g.n[0]), dim3(kT), 0, s, X, S, t,
                       offs, stopped, lin, lin_flag);
  t += g.n[0];
  if (g.n[1] > 0)
    hipLaunchKernelGGL((k_symm_mm_split<NP, F16, 64>), dim3(g.n[1]), dim3(kT), 0, s, X, S, t,
                       offs, stopped, lin, lin_flag);
  t += g.n[1];
  if (g.n[4] > 0 || g.n[5] > 0) {
    if constexpr (NP == 2 && F16) {
      if (g.n[4] > 0)
        hipLaunchKernelGGL(k_symm_mm_split_il<128>, dim3(g.n[4]), dim3(kT), 0, s, X, S, t, offs,
                           stopped, lin, lin_flag);
      t += g.n[4];
      if (g.n[5] > 0)
        hipLaunchKernelGGL(k_symm_mm_split_il<64>, dim3(g.n[5]), dim3(kT), 0, s, X, S, t, offs,
                           stopped, lin, lin_flag);
    } else {
      fail(GB_EHIP, "the interleaved split squares take fp16 planes only");
    }
  }
  GB_LAUNCH_CHECK();
}

void launch_split(const float* X, float* S, const int4* tiles, const Groups& g,
                  const int64_t* offs, hipStream_t s, int planes, int lin,
                  const int32_t* stopped = nullptr, const int32_t* lin_flag = nullptr) {
  if (planes == 1) launch_split_np<1, false>(X, S, tiles, g, offs, s, lin, stopped, lin_flag);
  else if (planes == 2) launch_split_np<2, false>(X, S, tiles, g, offs, s, lin, stopped, lin_flag);
  else if (planes == 4) launch_split_np<2, true>(X, S, tiles, g, offs, s, lin, stopped, lin_flag);
  else launch_split_np<3, false>(X, S, tiles, g, offs, s, lin, stopped, lin_flag);
}

// device tile table: the launch list, then the subgraph-major list
DBuf<int4> upload_tiles(const Plan& pl, hipStream_t s) {
  DBuf<int4> t(pl.launch.size() + pl.tiles.size(), s);
  GB_HIP(hipMemcpyAsync(t.get(), pl.launch.data(), pl.launch.size() * sizeof(int4),
                        hipMemcpyHostToDevice, s));
  GB_HIP(hipMemcpyAsync(t.get() + pl.launch.size(), pl.tiles.data(), pl.tiles.size() * sizeof(int4),
                        hipMemcpyHostToDevice, s));
  return t;
}

void launch_plan_square_f64(const double* X, double* S, const Plan& pl, const int4* tiles,
                            const int64_t* offs, hipStream_t s, int lin = 0) {
  launch_square<double>(X, S, tiles, pl.lg, offs, s, lin);
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  explicit Timer() {
    GB_HIP(hipEventCreate(&a));
    GB_HIP(hipEventCreate(&b));
  }
  Timer(const Timer&) = delete;
  Timer& operator=(const Timer&) = delete;
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

// ---- autotuner: tile edge per size bucket ----------------------------------------------------
// Subgraphs are bucketed by padded size (256-wide buckets).  The first time a bucket is seen
// for a kind of square (0 FP64, 1 FP32, 10 + planes for the split squares), one squaring
// launch of that bucket's blocks is timed with each kernel variant (one warm-up, two timed
// launches each) and the fastest is kept.  The table lives for the process and can be kept in
// a JSON file (gb_tune_save / gb_tune_load, or the GB_TUNE_FILE environment variable: read at
// the first tuning, rewritten after every new entry), tagged with the library's source hash and
// the device; a file with another tag is not used.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tune;  // (square kind, bucket) -> variant code
bool g_tune_env_read = false;

#ifndef GB_SOURCE_SHA
#define GB_SOURCE_SHA "unknown"
#endif

std::string tune_identity() {
  int dev = 0;
  GB_HIP(hipGetDevice(&dev));
  hipDeviceProp_t pr;
  GB_HIP(hipGetDeviceProperties(&pr, dev));
  char buf[512];
  snprintf(buf, sizeof(buf), "%s cu=%d %s", pr.gcnArchName, pr.multiProcessorCount, pr.name);
  for (char* c = buf; *c; ++c)
    if (*c == '"' || *c == '\\') *c = ' ';
  return buf;
}

// writes the table (caller holds g_tune_mu); false if the file cannot be written
bool tune_write(const char* path) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\"format\": \"libgb-tune-1\", \"library\": \"%s\", \"device\": \"%s\",\n \"entries\": [",
          GB_SOURCE_SHA, tune_identity().c_str());
  bool first = true;
  for (const auto& kv : g_tune) {
    fprintf(f, "%s\n  {\"kind\": %d, \"bucket\": %d, \"variant\": %d}", first ? "" : ",",
            kv.first.first, kv.first.second, kv.second);
    first = false;
  }
  fprintf(f, "]}\n");
  const bool ok = fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

// reads a table written by tune_write into g_tune (caller holds g_tune_mu); returns the number
// of entries, or -1 (message in *why) if the file is missing, malformed or for another library
// or device
int tune_read(const char* path, std::string* why) {
  FILE* f = fopen(path, "r");
  if (!f) {
    *why = "cannot open the file";
    return -1;
  }
  std::string txt;
  char chunk[4096];
  size_t got;
  while ((got = fread(chunk, 1, sizeof(chunk), f)) > 0) txt.append(chunk, got);
  fclose(f);
  auto field = [&](const char* key) -> std::string {
    const std::string k = std::string("\"") + key + "\": \"";
    const size_t a = txt.find(k);
    if (a == std::string::npos) return std::string("\x01");
    const size_t b = txt.find('"', a + k.size());
    return b == std::string::npos ? std::string("\x01") : txt.substr(a + k.size(), b - a - k.size());
  };
  if (field("format") != "libgb-tune-1") {
    *why = "not a libgb tuning table";
    return -1;
  }
  if (field("library") != GB_SOURCE_SHA) {
    *why = "written by another build of the library";
    return -1;
  }
  if (field("device") != tune_identity()) {
    *why = "written on another device";
    return -1;
  }
  std::map<std::pair<int, int>, int> t;
  size_t pos = 0;
  while ((pos = txt.find("{\"kind\":", pos)) != std::string::npos) {
    int kind, bucket, variant;
    if (sscanf(txt.c_str() + pos, "{\"kind\": %d, \"bucket\": %d, \"variant\": %d}", &kind,
               &bucket, &variant) != 3) {
      *why = "malformed entry";
      return -1;
    }
    // kinds: 0 FP64, 1 FP32, 10 + planes split squares; the interleaved split (129, 65)
    // exists for the fp16 planes (kind 14) only
    const bool known = variant_index(variant) >= 0;
    const bool split = kind >= 11 && kind <= 14;
    const bool split_ok = variant == 128 || variant == 64 || (kind == 14 && split_il_code(variant));
    if (!known || bucket < 1 || !(kind == 0 || kind == 1 || split) || (split && !split_ok) ||
        (!split && split_il_code(variant))) {
      *why = "entry with an unknown kind, bucket or variant";
      return -1;
    }
    t[{kind, bucket}] = variant;
    pos += 8;
  }
  for (const auto& kv : t) g_tune[kv.first] = kv.second;
  return (int)t.size();
}

// the GB_TUNE_FILE table, read once (caller holds g_tune_mu; an unusable file is ignored)
void tune_env_read() {
  if (g_tune_env_read) return;
  g_tune_env_read = true;
  const char* path = std::getenv("GB_TUNE_FILE");
  std::string why;
  if (path && *path) (void)tune_read(path, &why);
}

void tune_env_write() {
  const char* path = std::getenv("GB_TUNE_FILE");
  if (path && *path) (void)tune_write(path);
}

// planes = 0: launch_square<T>; planes > 0 (T = float): the split squares, 128- or 64-edge tiles
template <typename T>
std::vector<int> tune_tiles(const Part& P, const Plan& pl, T* X, T* S, const int64_t* offs,
                            hipStream_t s, int kind, bool xcd, int planes = 0) {
  std::vector<int> bt(pl.n_sub, kBT);
  std::map<int, std::vector<int>> buckets;
  for (int i = 0; i < pl.n_sub; ++i) buckets[(pl.npad[i] + 255) / 256].push_back(i);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_read();
  }
  Timer tm;
  bool added = false;
  for (auto& kv : buckets) {
    int choice = 0;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find({kind, kv.first});
      if (it != g_tune.end()) choice = it->second;
    }
    if (!choice) {
      float best = INFINITY;
      for (int code : kVariants) {
        if (planes > 0 && code != 128 && code != 64 && !(planes == 4 && split_il_code(code)))
          continue;
        if (planes == 0 && split_il_code(code)) continue;
        std::vector<int> e(pl.n_sub, 0);
        for (int i : kv.second) e[i] = code;
        const Plan sub = make_plan(P, &e, xcd);
        DBuf<int4> tl = upload_tiles(sub, s);
        auto run = [&] {
          if constexpr (std::is_same<T, float>::value) {
            if (planes > 0) {
              launch_split(X, S, tl.get(), sub.lg, offs, s, planes, 0);
              return;
            }
          }
          launch_square<T>(X, S, tl.get(), sub.lg, offs, s);
        };
        run();
        GB_HIP(hipEventRecord(tm.a, s));
        run();
        run();
        GB_HIP(hipEventRecord(tm.b, s));
        GB_HIP(hipStreamSynchronize(s));
        const float ms = elapsed(tm.a, tm.b);
        if (ms < best) {
          best = ms;
          choice = code;
        }
      }
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[{kind, kv.first}] = choice;
      added = true;
    }
    for (int i : kv.second) bt[i] = choice;
  }
  if (added) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_write();
  }
  return bt;
}

template <typename T>
void choose_tiles(const Part& P, Plan& pl, T* X, T* S, DBuf<int4>& tiles, const int64_t* offs,
                  hipStream_t s, int policy, int kind, gb_sp2_stats& st, bool xcd,
                  int planes = 0, bool record = true) {
  std::vector<int> bt(pl.n_sub, kBT);
  if (policy == 2) bt.assign(pl.n_sub, 64);
  else if (policy == 4 && planes == 0) bt.assign(pl.n_sub, 63);
  else if (policy == 5 && planes == 0) bt.assign(pl.n_sub, 62);
  else if (policy == 6 && planes == 4) bt.assign(pl.n_sub, 129);
  else if (policy == 7 && planes == 4) bt.assign(pl.n_sub, 65);
  // FP64 / FP32 squares: the register-staged 64-edge variant, the fastest measured in every
  // size bucket of the N = 1024, 18000 and 100000 systems (the others stay selectable); split
  // squares: timed per bucket
  else if (policy != 1 && planes == 0) bt.assign(pl.n_sub, 62);
  else if (policy != 1) bt = tune_tiles<T>(P, pl, X, S, offs, s, kind, xcd, planes);
  if (policy == 1) return;
  pl = make_plan(P, &bt, xcd);
  tiles = upload_tiles(pl, s);
  if (!record) return;  // the refinement's squares: the stats describe the loop's
  st.n_tile64 = 0;
  st.n_stage3 = 0;
  st.n_regstage = 0;
  st.n_split_il = 0;
  for (int e : bt) {
    st.n_split_il += split_il_code(e);
    st.n_tile64 += variant_edge(e) == 64;
    st.n_stage3 += e == 63;
    st.n_regstage += e == 62;
  }
  st.square_flops_exec = pl.flops_exec;
}

// Decisions whose margin | |t2 - n| - |2 t1 - t2 - n| | is within the rounding of the summed
// traces (64 units in the last place of |t1| + |t2| + n_occ) could go the other way under
// another summation order; they are counted in the stats.
inline bool near_tie(const StepRec& r, double n_occ) {
  return r.margin <= 64.0 * 1.1102230246251565e-16 * (fabs(r.t1) + fabs(r.t2) + fabs(n_occ));
}

// Records of one step into the stats (it < 128).
inline void record_step(gb_sp2_stats& st, int it, const StepRec& r, bool applied, bool by_rule,
                        double n_occ) {
  if (it >= 128) return;
  st.t1[it] = r.t1;
  st.t2[it] = r.t2;
  st.idem = r.e;
  if (!applied) return;
  st.branch[it] = (uint8_t)r.b;
  if (by_rule) {
    st.min_margin = std::min(st.min_margin, r.margin);
    if (near_tie(r, n_occ)) ++st.n_near_tie;
  }
}

// One squaring launch of a step: the new iterate S = X^2 or 2X - X^2 (lin, or *lin_flag on the
// device-driven loops), batched over every subgraph or (per_subgraph) one launch per subgraph.
template <typename T>
void launch_step(const T* X, T* S, const Plan& pl, const int4* tiles, const int64_t* offs,
                 hipStream_t s, int planes, int lin, bool per_subgraph,
                 const int32_t* stopped = nullptr, const int32_t* lin_flag = nullptr) {
  const int nl = (int)pl.launch.size();
  if constexpr (std::is_same<T, float>::value) {
    if (planes > 0) {
      if (per_subgraph)
        for (const int4& rg : pl.ranges)
          launch_split(X, S, tiles + nl + rg.x, one_group(rg.z, rg.y), offs, s, planes, lin,
                       stopped, lin_flag);
      else
        launch_split(X, S, tiles, pl.lg, offs, s, planes, lin, stopped, lin_flag);
      return;
    }
  }
  if (per_subgraph)
    for (const int4& rg : pl.ranges)
      launch_square<T>(X, S, tiles + nl + rg.x, one_group(rg.z, rg.y), offs, s, lin, stopped,
                       lin_flag);
  else
    launch_square<T>(X, S, tiles, pl.lg, offs, s, lin, stopped, lin_flag);
}

// Host-driven SP2 loop in precision T on buffers X (current iterate) and S (scratch): each step
// takes the core traces of X and X^2 (from X), the FP64 decision, reads it back (one host round
// trip per step), then one squaring launch writes the next iterate.  Used for one launch per
// subgraph, for the tape of the adjoint and for the alternating FP64 refinement.  Returns the
// step index at which the stop rule fired, the replay ended, max_iter was reached, or (low
// precision) the idempotency error stagnated; X then holds the result.
template <typename T>
int sp2_loop(T*& X, T*& S, const Plan& pl, const DBuf<int4>& tiles, const DBuf<int64_t>& offs,
             const DBuf<int32_t>& npad, const Part& P, double n_occ, double tol, int max_iter,
             const uint8_t* branch_in, int n_branch_in, bool stagnation_stop, int it0,
             gb_sp2_stats& st, DBuf<StepRec>& recs, hipStream_t s, int* stop_kind,
             TapeData* tape = nullptr, int planes = 0, bool per_subgraph = false,
             bool alternate = false) {
  Timer tm;
  PinnedRec pin;
  int it = it0;
  // the fp16 loop's iterate is stored as 2^14 X: its traces are scaled back
  const bool scaled = std::is_same<T, float>::value && planes == 4;
  const double ts1 = scaled ? kF16TraceDown1 : 1.0, ts2 = scaled ? kF16TraceDown2 : 1.0;
  int prev_b = -1;
  std::vector<double> es;
  DBuf<double> part(2 * (size_t)pl.n_sub, s);
  for (;;) {
    hipLaunchKernelGGL(k_trace_rows<T>, dim3(pl.n_sub), dim3(kT), 0, s, X, offs.get(), npad.get(),
                       P.core_ptr.get(), part.get(), nullptr, ts1, ts2);
    int forced = -1;
    if (branch_in) forced = it < n_branch_in ? (int)branch_in[it] : 2;
    else if (alternate && prev_b >= 0) forced = 10 + (1 - prev_b);
    const int at_max = it >= max_iter || it >= 127 ? 1 : 0;
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(kT), 0, s, part.get(), pl.n_sub, n_occ, tol, forced,
                       at_max, recs.get());
    GB_LAUNCH_CHECK();
    GB_HIP(hipMemcpyAsync(pin.h, recs.get(), sizeof(StepRec), hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    const StepRec r = *pin.h;
    es.push_back(r.e);
    const bool stag = !r.stop && stagnation_stop && es.size() >= 10 &&
                      es.back() > es[es.size() - 3];
    record_step(st, it, r, !r.stop && !stag, branch_in == nullptr && !alternate, n_occ);
    if (r.stop) {
      *stop_kind = (r.stop == 1 && (branch_in == nullptr || r.e <= tol)) ? 1 : 2;
      if (branch_in && r.stop == 1) *stop_kind = r.e <= tol ? 1 : 3;
      return it;
    }
    if (stag) {
      *stop_kind = 4;
      return it;
    }
    prev_b = r.b;
    GB_HIP(hipEventRecord(tm.a, s));
    launch_step<T>(X, S, pl, tiles.get(), offs.get(), s, planes, r.b == 1 ? 1 : 0, per_subgraph);
    GB_HIP(hipEventRecord(tm.b, s));
    std::swap(X, S);
    ++it;
    if (tape) {
      tape->branch.push_back((uint8_t)r.b);
      if (it % tape->stride == 0) {
        DBuf<double> c(pl.total, nullptr);
        GB_HIP(hipMemcpyAsync(c.get(), X, pl.total * sizeof(T), hipMemcpyDeviceToDevice, s));
        tape->ckpt.push_back(std::move(c));
      }
    }
    GB_HIP(hipEventSynchronize(tm.b));
    if (std::is_same<T, float>::value) {
      st.ms_square_lo += elapsed(tm.a, tm.b);
      st.n_square_lo += 1;
    } else {
      st.ms_square += elapsed(tm.a, tm.b);
      st.n_square += 1;
    }
  }
}

// Events of the device-driven loop (one pair per enqueued step), kept per thread and device for
// the life of the process.
std::vector<hipEvent_t>& step_events(size_t need) {
  thread_local std::map<int, std::vector<hipEvent_t>> pool;
  int dev = 0;
  GB_HIP(hipGetDevice(&dev));
  auto& v = pool[dev];
  while (v.size() < need) {
    hipEvent_t e;
    GB_HIP(hipEventCreate(&e));
    v.push_back(e);
  }
  return v;
}

__global__ void k_loop_init(LoopState* __restrict__ st, LoopInit in) {
  st->it = in.it0;
  st->it0 = in.it0;
  st->stopped = 0;
  st->max_iter = in.max_iter;
  st->n_forced = in.n_forced;
  st->stag = in.stag;
  st->cur_b = -1;
  st->n_occ = in.n_occ;
  st->tol = in.tol;
  for (int i = 0; i < 128; ++i) st->forced[i] = in.forced[i];
}

// Device-driven SP2 loop (launch modes 0 and 2): the stop flag, the step counter, the branch
// and the step records live on the device, each squaring launch reads the branch there, and
// every kernel of a step returns at once after the stop, so steps are enqueued without waiting
// for any decision.  The host enqueues the first kFirst steps (or every step the loop can still
// take, if fewer), then reads the loop state once; only an expansion longer than that costs one
// more read per kMore further steps.  Mode 0 enqueues the kernels on the stream (a pair of
// events around every square gives its duration); mode 2 captures two steps, one per buffer
// parity, in a hipGraph and replays it.
template <typename T>
int sp2_loop_dev(T*& X, T*& S, const Plan& pl, const DBuf<int4>& tiles, const DBuf<int64_t>& offs,
                 const DBuf<int32_t>& npad, const Part& P, double n_occ, double tol, int max_iter,
                 const uint8_t* branch_in, int n_branch_in, bool stagnation_stop, int it0,
                 gb_sp2_stats& st, hipStream_t s, int* stop_kind, int planes, bool graph) {
  constexpr int kFirst = 32, kMore = 8;
  // index of the last decision the loop can reach: it stops there at the latest
  const int last = branch_in ? std::min(n_branch_in, 127) : std::min(max_iter, 127);
  if (last < it0) fail(GB_EINVAL, "no SP2 step left (first step %d, last %d)", it0, last);
  const int max_dec = last - it0 + 1;
  LoopInit in{};
  in.it0 = it0;
  in.max_iter = max_iter;
  in.n_forced = branch_in ? std::min(n_branch_in, 127) : -1;
  in.stag = stagnation_stop ? 1 : 0;
  in.n_occ = n_occ;
  in.tol = tol;
  if (branch_in) std::memcpy(in.forced, branch_in, std::min(n_branch_in, 128));
  DBuf<LoopState> d(1, s);
  DBuf<double> part(2 * (size_t)pl.n_sub, s);
  // the fp16 loop's iterate is stored as 2^14 X: its traces are scaled back
  const bool scaled = std::is_same<T, float>::value && planes == 4;
  const double ts1 = scaled ? kF16TraceDown1 : 1.0, ts2 = scaled ? kF16TraceDown2 : 1.0;
  hipLaunchKernelGGL(k_loop_init, dim3(1), dim3(1), 0, s, d.get(), in);
  GB_LAUNCH_CHECK();
  const int32_t* stopped = &d.get()->stopped;
  const int32_t* cur_b = &d.get()->cur_b;
  auto& ev = step_events(2 * (size_t)max_dec);
  auto enqueue = [&](hipStream_t q, int k, bool timed) {  // step k of the loop (0-based)
    T* A = (k & 1) ? S : X;
    T* B = (k & 1) ? X : S;
    hipLaunchKernelGGL(k_trace_rows<T>, dim3(pl.n_sub), dim3(kT), 0, q, A, offs.get(),
                       npad.get(), P.core_ptr.get(), part.get(), stopped, ts1, ts2);
    hipLaunchKernelGGL(k_decide_dev, dim3(1), dim3(kT), 0, q, part.get(), pl.n_sub, d.get());
    GB_LAUNCH_CHECK();
    if (timed) GB_HIP(hipEventRecord(ev[2 * k], q));
    launch_step<T>(A, B, pl, tiles.get(), offs.get(), q, planes, 0, false, stopped, cur_b);
    if (timed) GB_HIP(hipEventRecord(ev[2 * k + 1], q));
  };
  hipStream_t cs = nullptr;
  hipGraph_t gr = nullptr;
  hipGraphExec_t exec = nullptr;
  struct Cleanup {
    hipStream_t& cs;
    hipGraph_t& g;
    hipGraphExec_t& e;
    ~Cleanup() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
      if (cs) (void)hipStreamDestroy(cs);
    }
  } cleanup{cs, gr, exec};
  if (graph) {
    GB_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    GB_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    enqueue(cs, 0, false);
    enqueue(cs, 1, false);
    GB_HIP(hipStreamEndCapture(cs, &gr));
    GB_HIP(hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0));
  }
  LoopState h;
  int queued = 0;
  for (;;) {
    const int batch = std::min(queued == 0 ? kFirst : kMore, max_dec - queued);
    if (graph) {
      const int pairs = (batch + 1) / 2;  // the graph holds two steps
      for (int r = 0; r < pairs; ++r) GB_HIP(hipGraphLaunch(exec, s));
      queued += 2 * pairs;
    } else {
      for (int k = queued; k < queued + batch; ++k) enqueue(s, k, true);
      queued += batch;
    }
    GB_HIP(hipMemcpyAsync(&h, d.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    if (h.stopped) break;
    if (queued >= max_dec) fail(GB_EHIP, "device-driven SP2 loop did not stop");
  }
  const int it_stop = h.it;
  for (int it = it0; it <= it_stop && it < 128; ++it)
    record_step(st, it, h.recs[it], it < it_stop, branch_in == nullptr, n_occ);
  const int n_sq = it_stop - it0;
  float ms = 0.f;
  if (!graph)
    for (int k = 0; k < n_sq; ++k) ms += elapsed(ev[2 * k], ev[2 * k + 1]);
  if (std::is_same<T, float>::value) {
    st.n_square_lo += n_sq;
    st.ms_square_lo += ms;
  } else {
    st.n_square += n_sq;
    st.ms_square += ms;
  }
  const StepRec& lr = h.recs[it_stop];
  if (lr.stop == 1) *stop_kind = (branch_in && lr.e > tol) ? 3 : 1;
  else *stop_kind = lr.stop == 4 ? 4 : 2;
  // n_sq squares were applied, each moving the iterate to the other buffer
  if (n_sq % 2 == 1) std::swap(X, S);
  return it_stop;
}

}  // namespace

// Full gb_density pipeline on an already built partition.
// ---- FP64 McWeeny refinement on the core rows --------------------------------------------
// D keeps only the core columns of each block, i.e. (X symmetric) its core rows E q(X) for the
// core unit rows E.  For p(x) = 3x^2 - 2x^3: E p(X) = 3 E X^2 - 2 E X^3, V p(X) = 3 V X^2 -
// 2 V X^3 for any slab V, and p(p(X)) = 3 p(X)^2 - 2 p(X)^3, so one or two McWeeny steps on the
// core rows take 2 or 8 slab products V X (2 n^2 k flops each instead of 2 n^3 for a block
// square), evaluated nested so every intermediate stays a polynomial bounded on [0, 1].
struct CoreRows {
  int kmax = 0;
  int colblocks = 0;
  int64_t total = 0;  // doubles per slab
  std::vector<int64_t> so;  // slab offset of each subgraph (host)
  DBuf<int64_t> soffs;      // the same on the device
};

// host part: the slab layout (false when a core exceeds 32 rows: whole blocks instead)
bool core_rows_sizes(const Part& P, const Plan& pl, CoreRows& cr) {
  int kmax = 0;
  for (int q = 0; q < pl.n_sub; ++q) {
    kmax = std::max(kmax, P.h_core_ptr[q + 1] - P.h_core_ptr[q]);
    if (pl.npad[q] % 64) return false;
  }
  if (kmax > 32) return false;
  cr.so.resize(pl.n_sub);
  int64_t t = 0;
  for (int q = 0; q < pl.n_sub; ++q) {
    cr.so[q] = t;
    t += (int64_t)(P.h_core_ptr[q + 1] - P.h_core_ptr[q]) * pl.npad[q];
  }
  cr.kmax = kmax <= 16 ? 16 : 32;
  cr.colblocks = (pl.max_npad + 255) / 256;
  cr.total = std::max<int64_t>(t, 1);
  return true;
}

bool core_rows_plan(const Part& P, const Plan& pl, CoreRows& cr, hipStream_t s) {
  if (!core_rows_sizes(P, pl, cr)) return false;
  cr.soffs = DBuf<int64_t>(pl.n_sub, s);
  // cr.so lives as long as cr, so the copy needs no wait
  GB_HIP(hipMemcpyAsync(cr.soffs.get(), cr.so.data(), pl.n_sub * 8, hipMemcpyHostToDevice, s));
  return true;
}

struct RowsCtx {
  const CoreRows& cr;
  const Plan& pl;
  const Part& P;
  const int64_t* offs;
  const int32_t* npad;
  hipStream_t s;
  double xscale;  // the stored iterate is X / xscale
  template <typename TX>
  void mm(const TX* X, const double* V, double* W) const {
    const dim3 grid(cr.colblocks * ((pl.n_sub + 7) / 8 * 8));
    if (cr.kmax == 16)
      hipLaunchKernelGGL((k_rows_mm<16, TX>), grid, dim3(256), 0, s, X, offs, npad, V, W,
                         cr.soffs.get(), P.core_ptr.get(), pl.n_sub, cr.colblocks, xscale);
    else
      hipLaunchKernelGGL((k_rows_mm<32, TX>), grid, dim3(256), 0, s, X, offs, npad, V, W,
                         cr.soffs.get(), P.core_ptr.get(), pl.n_sub, cr.colblocks, xscale);
    GB_LAUNCH_CHECK();
  }
  void lin2(double* out, double a, const double* x, double b, const double* y) const {
    hipLaunchKernelGGL(k_lin2, dim3(grid_for(cr.total, 256, 65536)), dim3(256), 0, s, out, a, x, b,
                       y, cr.total);
    GB_LAUNCH_CHECK();
  }
  // out = V p(X) (out may be V); t0, t1 scratch slabs
  template <typename TX>
  void apply_p(const TX* X, const double* V, double* out, double* t0, double* t1) const {
    mm(X, V, t0);
    mm(X, t0, t1);
    mm(X, t1, t0);
    lin2(out, 3.0, t1, -2.0, t0);
  }
};

int tune_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_env_read();
  if (!tune_write(path)) return -1;
  return (int)g_tune.size();
}

int tune_load(const char* path, std::string* why) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_env_read = true;  // an explicit table replaces the environment's
  return tune_read(path, why);
}

void density_slots(const Part& P, int n, int width, const gb_sp2_opts& o,
                   size_t bytes[Workspace::kSlots]) {
  for (int i = 0; i < Workspace::kSlots; ++i) bytes[i] = 0;
  const Plan pl = make_plan(P, nullptr, o.tile_order == 0);
  const size_t t = (size_t)pl.total;
  bytes[0] = bytes[1] = t * 8;  // FP64 X, S
  if (o.precision != GB_FP64) {
    bytes[2] = t * 8;             // FP64 McWeeny product (whole-block refinement)
    bytes[3] = bytes[4] = t * 4;  // FP32 X, S
    CoreRows cr;
    if (core_rows_sizes(P, pl, cr)) bytes[7] = 5 * (size_t)cr.total * 8;  // core-row slabs
  }
  bytes[8] = (size_t)n * width * 8;  // X0 on H's pattern
}

void density(const gb_ell& H, int32_t n_occ, const gb_sp2_opts& o, const Part& P, double emin,
             double emax, const double* x0, gb_ell& D, gb_sp2_stats& st, hipStream_t s,
             TapeData** tape_out, Workspace* ext) {
  Timer t_all;
  GB_HIP(hipEventRecord(t_all.a, s));
  const bool xcd = o.tile_order == 0;
  Plan pl = make_plan(P, nullptr, xcd);
  st.square_flops = pl.flops_alg;
  st.square_flops_exec = pl.flops_exec;
  DBuf<int64_t> offs(pl.n_sub, s);
  DBuf<int32_t> npad(pl.n_sub, s);
  DBuf<int4> tiles = upload_tiles(pl, s);
  GB_HIP(hipMemcpyAsync(offs.get(), pl.off.data(), pl.n_sub * 8, hipMemcpyHostToDevice, s));
  GB_HIP(hipMemcpyAsync(npad.get(), pl.npad.data(), pl.n_sub * 4, hipMemcpyHostToDevice, s));
  DBuf<StepRec> recs(2, s);
  const int N = H.n;
  const double tol = o.idem_tol > 0 ? o.idem_tol : 1e-10 * N / 1024.0;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 100;
  const bool low = o.precision != GB_FP64;
  // bf16 planes of the low-precision square: 0 = native FP32 MFMA
  // split planes of the low-precision square: 0 = native FP32 MFMA; 1 / 2 / 3 bf16 planes;
  // 4 = two fp16 planes
  const int planes = o.precision == GB_BF16_REFINE ? 1 : o.precision == GB_BF16X3_REFINE ? 2
                   : o.precision == GB_BF16X6_REFINE ? 3 : o.precision == GB_FP16X3_REFINE ? 4
                   : 0;
  const int n_refine = o.n_refine;
  // launch modes 0 (default) and 2 run the loop on the device; 1 (one launch per subgraph) and
  // 3 read every decision back on the host
  const bool dev_loop = o.launch_mode == 0 || o.launch_mode == 2;
  int stop_kind = 0;
  // stage timings: events read once the call has finished its work (no wait per stage)
  Timer t_gather, t_sp2, t_ref, t_scat;
  // the gather is timed with the first buffer allocation included
  GB_HIP(hipEventRecord(t_gather.a, s));
  const size_t lds_g = (size_t)pl.max_npad * 8 + (size_t)P.max_sub * 4 + 64;
  if (lds_g > 160 * 1024) fail(GB_EUNSUPPORTED, "subgraph of %d vertices too large", P.max_sub);
  const dim3 ggrid(pl.n_sub, (pl.max_npad + kRows - 1) / kRows);
  // batch buffers from the cached workspace or the caller's: slots 0-2 FP64 (X, S, McWeeny
  // T), 3-4 FP32, 7 the core-row slabs
  WsLease ws(ext);
  double* const X64 = ws->get<double>(0, pl.total, s);
  double* const S64 = ws->get<double>(1, pl.total, s);
  double* xd = X64;
  double* sd = S64;
  int it_end = 0;
  bool done = false;  // the FP64 steps before a low-precision loop already converged
  // After a low-precision loop: its iterate made exactly symmetric in FP32 (what the core-row
  // refinement reads; stored as X / xs_scale, the fp16 loop's 2^14 X), and an FP64 copy of X
  // in xd only where whole blocks are refined, checked or scattered (ensure_xd).
  const float* xs = nullptr;
  double xs_scale = 1.0;
  bool xd_ready = true;
  if (low) {
    float* xf = ws->get<float>(3, pl.total, s);
    float* sf = ws->get<float>(4, pl.total, s);
    const int nhi = std::min(std::max(0, o.n_fp64_first), max_iter);
    if (nhi > 0) {
      hipLaunchKernelGGL(k_gather<double>, ggrid, dim3(kT), lds_g, s, H.col, x0, H.width,
                         P.core_ptr.get(), P.sub_ptr.get(), P.sub_idx.get(), offs.get(),
                         npad.get(), xd, 1.0);
    } else {
      hipLaunchKernelGGL(k_gather<float>, ggrid, dim3(kT), lds_g, s, H.col, x0, H.width,
                         P.core_ptr.get(), P.sub_ptr.get(), P.sub_idx.get(), offs.get(),
                         npad.get(), xf, planes == 4 ? kF16Scale : 1.0f);
    }
    GB_LAUNCH_CHECK();
    GB_HIP(hipEventRecord(t_gather.b, s));
    GB_HIP(hipEventRecord(t_sp2.a, s));
    if (nhi > 0) {
      // the first steps, where the spectral gap of X is smallest and rounding errors are
      // amplified most, in FP64
      if (dev_loop)
        it_end = sp2_loop_dev<double>(xd, sd, pl, tiles, offs, npad, P, n_occ, tol, nhi,
                                      o.branch_in, o.n_branch_in, false, 0, st, s, &stop_kind, 0,
                                      o.launch_mode == 2);
      else
        it_end = sp2_loop<double>(xd, sd, pl, tiles, offs, npad, P, n_occ, tol, nhi, o.branch_in,
                                  o.n_branch_in, false, 0, st, recs, s, &stop_kind, nullptr, 0,
                                  o.launch_mode == 1);
      done = stop_kind == 1 || stop_kind == 3;
      if (!done) {
        hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_for(pl.total, kT, 65536)),
                           dim3(kT), 0, s, xd, xf, pl.total, planes == 4 ? kF16Scale : 1.0f);
        GB_LAUNCH_CHECK();
      }
    }
    if (!done) {
      // FP32 squares: kind 1; split squares: kind 10 + planes (128- or 64-edge tiles)
      choose_tiles<float>(P, pl, xf, sf, tiles, offs.get(), s, o.tile_policy,
                          planes ? 10 + planes : 1, st, xcd, planes);
      st.planes_db = planes;
      // The low-precision loop runs until its own rounding floor (the stagnation stop) unless
      // the traces already agree to 1e-7 per 1024 orbitals, so that one FP64 McWeeny step
      // usually finishes the job.
      const double tol_lo = 1e-7 * N / 1024.0;
      if (dev_loop)
        it_end = sp2_loop_dev<float>(xf, sf, pl, tiles, offs, npad, P, n_occ, tol_lo, max_iter,
                                     o.branch_in, o.n_branch_in, true, it_end, st, s, &stop_kind,
                                     planes, o.launch_mode == 2);
      else
        it_end = sp2_loop<float>(xf, sf, pl, tiles, offs, npad, P, n_occ, tol_lo, max_iter,
                                 o.branch_in, o.n_branch_in, true, it_end, st, recs, s, &stop_kind,
                                 nullptr, planes, o.launch_mode == 1);
      // the final low-precision square was only the stop test: continue from X made exactly
      // symmetric, in FP32, in place (every block is padded to a multiple of 64)
      hipLaunchKernelGGL(k_sym_diag, dim3(pl.max_npad / 64, pl.n_sub), dim3(256), 0, s, xf,
                         offs.get(), npad.get());
      GB_LAUNCH_CHECK();
      xs = xf;
      xs_scale = planes == 4 ? (double)kF16Down : 1.0;
      xd_ready = false;
    }
    GB_HIP(hipEventRecord(t_sp2.b, s));
  } else {
    hipLaunchKernelGGL(k_gather<double>, ggrid, dim3(kT), lds_g, s, H.col, x0, H.width,
                       P.core_ptr.get(), P.sub_ptr.get(), P.sub_idx.get(), offs.get(), npad.get(),
                       X64, 1.0);
    GB_LAUNCH_CHECK();
    if (tape_out) {
      TapeData* t = new TapeData();
      *tape_out = t;
      t->N = N;
      t->emin = emin;
      t->emax = emax;
      t->stride = o.tape_stride > 0 ? o.tape_stride : 4;
      t->max_sub = P.max_sub;
      t->pl = pl;
      auto dup_i32 = [&](DBuf<int32_t>& dst, const DBuf<int32_t>& src, size_t n) {
        dst = DBuf<int32_t>(n, nullptr);
        GB_HIP(hipMemcpyAsync(dst.get(), src.get(), n * 4, hipMemcpyDeviceToDevice, s));
      };
      t->offs = DBuf<int64_t>(pl.n_sub, nullptr);
      GB_HIP(hipMemcpyAsync(t->offs.get(), pl.off.data(), pl.n_sub * 8, hipMemcpyHostToDevice, s));
      dup_i32(t->npad, npad, pl.n_sub);
      t->tiles = DBuf<int4>(pl.launch.size(), nullptr);
      GB_HIP(hipMemcpyAsync(t->tiles.get(), pl.launch.data(), pl.launch.size() * sizeof(int4),
                            hipMemcpyHostToDevice, s));
      t->tiles_full = DBuf<int4>(pl.full_launch.size(), nullptr);
      GB_HIP(hipMemcpyAsync(t->tiles_full.get(), pl.full_launch.data(),
                            pl.full_launch.size() * sizeof(int4), hipMemcpyHostToDevice, s));
      dup_i32(t->core_ptr, P.core_ptr, P.n_sub + 1);
      dup_i32(t->sub_ptr, P.sub_ptr, P.n_sub + 1);
      dup_i32(t->sub_idx, P.sub_idx, P.total);
      dup_i32(t->sub_pos, P.sub_pos, P.total);
      DBuf<double> c(pl.total, nullptr);
      GB_HIP(hipMemcpyAsync(c.get(), X64, pl.total * 8, hipMemcpyDeviceToDevice, s));
      t->ckpt.push_back(std::move(c));
      GB_HIP(hipStreamSynchronize(s));  // host plan vectors above are copied before return
    }
    GB_HIP(hipEventRecord(t_gather.b, s));
  }

  if (!low && !tape_out) choose_tiles<double>(P, pl, xd, sd, tiles, offs.get(), s, o.tile_policy, 0, st, xcd);
  // (with split-bf16 squares tile_policy picks that kernel's variant; the FP64 refinement tunes
  // its own tile edge)
  // (after split squares the plan holds the split's tile edges; FP64 squares on whole blocks --
  // the refinement's fallback, refine_kind 1 and 2 -- tune their own variant when they run)
  auto ensure_xd = [&] {
    if (xd_ready) return;
    hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(pl.total, kT, 65536)), dim3(kT),
                       0, s, xs, xd, pl.total, xs_scale);
    GB_LAUNCH_CHECK();
    xd_ready = true;
  };
  auto fp64_tiles_for_blocks = [&] {
    if (low && planes > 0)
      choose_tiles<double>(P, pl, xd, sd, tiles, offs.get(), s, 0, 0, st, xcd, 0, false);
  };
  CoreRows cr;
  const double* rows_final = nullptr;  // core-row refinement: the core rows of D and of D^2
  const double* rows_check = nullptr;
  Timer& t_loop = low ? t_ref : t_sp2;
  GB_HIP(hipEventRecord(t_loop.a, s));
  if (low && done) {
    // converged during the FP64 steps: nothing to refine
  } else if (low && (o.refine_kind == 0 || o.refine_kind == 2)) {
    // FP64 refinement by McWeeny purification X <- 3X^2 - 2X^3.  It drives every eigenvalue to
    // 0 or 1 without acting on the trace, so the occupation the low-precision loop reached is
    // kept.  The stop test takes the traces from X itself, so no square is spent on it.
    const int at = std::min(it_end, 127);
    // Core rows (refine_kind 0): two steps, or one when e <- 12 e^2 (how the summed distances of
    // the eigenvalues from 0 and 1 contract per step, for one block) lands far below the
    // tolerance, evaluated on the core rows only, then the stop test on them; if it fails,
    // whole-block steps from the same X.
    bool refined = false;
    if (o.refine_kind == 0 && xs && core_rows_plan(P, pl, cr, s)) {
      DBuf<double> part(2 * (size_t)pl.n_sub, s);
      StepRec r;
      hipLaunchKernelGGL(k_trace_rows<float>, dim3(pl.n_sub), dim3(kT), 0, s, xs, offs.get(),
                         npad.get(), P.core_ptr.get(), part.get(), nullptr, xs_scale,
                         xs_scale * xs_scale);
      hipLaunchKernelGGL(k_decide, dim3(1), dim3(kT), 0, s, part.get(), pl.n_sub, (double)n_occ,
                         tol, 2, 0, recs.get());
      GB_LAUNCH_CHECK();
      GB_HIP(hipMemcpyAsync(&r, recs.get(), sizeof(r), hipMemcpyDeviceToHost, s));
      GB_HIP(hipStreamSynchronize(s));
      if (r.e <= tol) {
        refined = true;  // nothing to refine; the whole-block check below
      } else {
        const int m = (12.0 * r.e * r.e <= 1e-3 * tol || n_refine == 1) ? 1 : 2;
        double* sl = ws->get<double>(7, 5 * (size_t)cr.total, s);
        double *y = sl, *s1 = sl + cr.total, *s2 = sl + 2 * cr.total, *t0 = sl + 3 * cr.total,
               *t1 = sl + 4 * cr.total;
        const RowsCtx rc{cr, pl, P, offs.get(), npad.get(), s, xs_scale};
        // E p(X) = 3 E X^2 - 2 E X^3 (E X: the first k rows of X)
        hipLaunchKernelGGL(k_rows_copy<float>, dim3(cr.colblocks * 4, pl.n_sub), dim3(256), 0, s,
                           xs, offs.get(), npad.get(), t0, cr.soffs.get(), P.core_ptr.get(),
                           xs_scale);
        GB_LAUNCH_CHECK();
        rc.mm(xs, t0, t1);
        rc.mm(xs, t1, t0);
        rc.lin2(y, 3.0, t1, -2.0, t0);
        if (m == 2) {  // E p(p(X)) = 3 E p(X)^2 - 2 E p(X)^3
          rc.apply_p(xs, y, s1, t0, t1);
          rc.apply_p(xs, s1, s2, t0, t1);
          rc.lin2(y, 3.0, s1, -2.0, s2);
        }
        hipLaunchKernelGGL(k_trace_rows<double>, dim3(pl.n_sub), dim3(kT), 0, s, y,
                           cr.soffs.get(), npad.get(), P.core_ptr.get(), part.get(), nullptr, 1.0,
                           1.0);
        hipLaunchKernelGGL(k_decide, dim3(1), dim3(kT), 0, s, part.get(), pl.n_sub,
                           (double)n_occ, tol, 2, 0, recs.get());
        GB_LAUNCH_CHECK();
        StepRec r2;
        GB_HIP(hipMemcpyAsync(&r2, recs.get(), sizeof(r2), hipMemcpyDeviceToHost, s));
        GB_HIP(hipStreamSynchronize(s));
        if (r2.e <= tol) {
          // the check's square: Z = Y P(X) (P = p or p o p), the core rows of D^2 (nine more
          // slab products; only when the max-norm check is asked for)
          if (o.check_idem) rc.apply_p(xs, y, s1, t0, t1);
          if (o.check_idem && m == 2) {
            rc.apply_p(xs, s1, s2, t0, t1);
            rc.mm(xs, s2, t0);
            rc.mm(xs, t0, t1);
            rc.mm(xs, t1, t0);
            rc.lin2(s1, 3.0, s2, -6.0, t1);  // 3 A2 - 2 (3 A2 X^2 - 2 A2 X^3)
            rc.lin2(s1, 1.0, s1, 4.0, t0);
          }
          rows_final = y;
          rows_check = s1;
          st.n_refine_done = m;
          r = r2;
          refined = true;
        }
      }
      if (refined) {
        st.idem = r.e;
        st.t1[at] = r.t1;
        st.t2[at] = r.t2;
        stop_kind = 1;
      }
    }
    if (!refined) {
      // Whole blocks: X^2 = S, then 3S - 2 S X (S and X commute, so S X is computed on upper
      // tiles and mirrored); steps repeat until the FP64 stop test holds (at most n_refine,
      // default 8).
      ensure_xd();
      fp64_tiles_for_blocks();
      DBuf<double> part(2 * (size_t)pl.n_sub, s);
      double* td = ws->get<double>(2, pl.total, s);
      const int max_steps = n_refine > 0 ? n_refine : 8;
      StepRec r;
      for (int step = 0;; ++step) {
        hipLaunchKernelGGL(k_trace_rows<double>, dim3(pl.n_sub), dim3(kT), 0, s, xd, offs.get(),
                           npad.get(), P.core_ptr.get(), part.get(), nullptr, 1.0, 1.0);
        hipLaunchKernelGGL(k_decide, dim3(1), dim3(kT), 0, s, part.get(), pl.n_sub,
                           (double)n_occ, tol, 2, 0, recs.get());
        GB_LAUNCH_CHECK();
        GB_HIP(hipMemcpyAsync(&r, recs.get(), sizeof(r), hipMemcpyDeviceToHost, s));
        GB_HIP(hipStreamSynchronize(s));
        if (r.e <= tol || step == max_steps) break;
        launch_square<double>(xd, sd, tiles.get(), pl.lg, offs.get(), s);
        launch_symm<double, 1>(sd, xd, sd, td, -2.0, 3.0, tiles.get(), pl.lg, offs.get(), s);
        std::swap(xd, td);
        ++st.n_refine_done;
      }
      st.idem = r.e;
      st.t1[at] = r.t1;
      st.t2[at] = r.t2;
      stop_kind = r.e <= tol ? 1 : 2;
    }
  } else if (low) {
    // FP64 refinement: SP2 steps with FP64 traces from where the FP32 loop stopped
    ensure_xd();
    fp64_tiles_for_blocks();
    const uint8_t* bin = nullptr;
    int nbin = 0;
    if (o.branch_in && o.n_branch_in > it_end) {
      bin = o.branch_in;
      nbin = o.n_branch_in;
    }
    // Without a replayed sequence the steps alternate X^2 and 2X - X^2 (the first one chosen
    // by the trace rule): each pair squares the distance of every eigenvalue from 0 or 1, as a
    // McWeeny step does, and leaves the trace where the low-precision loop put it.  The trace
    // rule itself would steer towards n_occ, which the rounded partitioned trace cannot reach
    // with idempotent blocks, and cycles.
    const int cap = std::min(it_end + (n_refine > 0 ? n_refine : 16), 127);
    it_end = sp2_loop<double>(xd, sd, pl, tiles, offs, npad, P, n_occ, tol, cap, bin, nbin, false,
                              it_end, st, recs, s, &stop_kind, nullptr, 0, o.launch_mode == 1,
                              bin == nullptr);
  } else {
    if (dev_loop && !tape_out)
      it_end = sp2_loop_dev<double>(xd, sd, pl, tiles, offs, npad, P, n_occ, tol, max_iter,
                                    o.branch_in, o.n_branch_in, false, 0, st, s, &stop_kind, 0,
                                    o.launch_mode == 2);
    else
      it_end = sp2_loop<double>(xd, sd, pl, tiles, offs, npad, P, n_occ, tol, max_iter,
                                o.branch_in, o.n_branch_in, false, 0, st, recs, s, &stop_kind,
                                tape_out ? *tape_out : nullptr, 0, o.launch_mode == 1);
    if (tape_out) (*tape_out)->K = it_end;
  }
  GB_HIP(hipEventRecord(t_loop.b, s));
  st.iters = it_end;
  st.converged = stop_kind == 1 ? 1 : 0;

  // final idempotency check on the core rows: X^2 restricted to the tiles that hold them (all
  // upper tiles in tile rows below the core size), then max |X^2 - X| over the core rows
  // (after the core-row refinement the core rows of X and X^2 are already there)
  // (only with check_idem: the trace-based FP64 stop test above is the default check)
  if (!rows_final) ensure_xd();
  const double* xfin = rows_final ? rows_final : xd;
  const int64_t* foffs = rows_final ? cr.soffs.get() : offs.get();
  DBuf<int4> idem_tiles;
  DBuf<double> per, mx;
  if (o.check_idem) {
    if (!rows_final) {
      idem_tiles = DBuf<int4>(std::max<size_t>(pl.idem.size(), 1), s);
      GB_HIP(hipMemcpyAsync(idem_tiles.get(), pl.idem.data(), pl.idem.size() * sizeof(int4),
                            hipMemcpyHostToDevice, s));
      launch_square<double>(xd, sd, idem_tiles.get(), one_group(128, (int)pl.idem.size()),
                            offs.get(), s);
    }
    const double* sfin = rows_final ? rows_check : sd;
    per = DBuf<double>(pl.n_sub, s);
    mx = DBuf<double>(1, s);
    hipLaunchKernelGGL(k_idem<double>, dim3(pl.n_sub), dim3(kT), 0, s, xfin, sfin, foffs,
                       npad.get(), P.core_ptr.get(), P.sub_ptr.get(), per.get());
    GB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_max, dim3(1), dim3(kT), 0, s, per.get(), pl.n_sub, mx.get());
    GB_LAUNCH_CHECK();
  }
  // scatter
  GB_HIP(hipEventRecord(t_scat.a, s));
  hipLaunchKernelGGL(k_scatter<double>, dim3(N), dim3(kT), 0, s, xfin, foffs, npad.get(),
                     P.sub_ptr.get(), P.sub_idx.get(), P.sub_pos.get(), P.col_sub.get(),
                     P.col_loc.get(), D.width, D.col, D.val);
  GB_LAUNCH_CHECK();
  GB_HIP(hipEventRecord(t_scat.b, s));
  double idem_max = NAN;
  if (o.check_idem) GB_HIP(hipMemcpyAsync(&idem_max, mx.get(), 8, hipMemcpyDeviceToHost, s));
  GB_HIP(hipEventRecord(t_all.b, s));
  GB_HIP(hipStreamSynchronize(s));
  st.ms_gather = elapsed(t_gather.a, t_gather.b);
  st.ms_sp2 = elapsed(t_sp2.a, t_sp2.b);
  if (low) st.ms_refine = elapsed(t_ref.a, t_ref.b);
  st.ms_scatter = elapsed(t_scat.a, t_scat.b);
  st.idem_max = idem_max;
  const int last = std::min(it_end, 127);
  st.trace = st.t1[last];
  st.ms_total += elapsed(t_all.a, t_all.b);
}


void tape_destroy(TapeData* t) { delete t; }
void tape_dims(const TapeData* t, int* n, int* max_sub) {
  *n = t->N;
  *max_sub = t->max_sub;
}

// Reverse sweep: Gbar <- Gbar X + X Gbar (X <- X^2) or 2 Gbar - (Gbar X + X Gbar)
// (X <- 2X - X^2) from the last step to the first, recomputing each checkpoint segment
// forward; then dL/dH per slot of H.
void density_vjp(TapeData& t, const gb_ell& G_D, const gb_ell& H, double* G_H, hipStream_t s) {
  const Plan& pl = t.pl;
  const int K = t.K, c = t.stride;
  DBuf<double> G(pl.total, s), G2(pl.total, s), Pm(pl.total, s);
  const int gfill = grid_for(pl.total, kT, 65536);
  hipLaunchKernelGGL(k_fill, dim3(gfill), dim3(kT), 0, s, G.get(), pl.total, 0.0);
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_seed, dim3(pl.n_sub), dim3(kT), 0, s, G_D.val, G_D.width, t.core_ptr.get(),
                     t.sub_ptr.get(), t.sub_idx.get(), t.sub_pos.get(), t.offs.get(), t.npad.get(),
                     G.get());
  GB_LAUNCH_CHECK();
  std::vector<DBuf<double>> seg;
  for (int q = 1; q < c; ++q) seg.emplace_back(pl.total, s);
  const int max_nt = pl.max_npad / 32;
  const dim3 cgrid(max_nt * max_nt, pl.n_sub);
  const int ntf = (int)pl.full_launch.size();
  for (int m = (K - 1) / c; m >= 0 && K > 0; --m) {
    const int start = m * c, end = std::min(start + c, K);
    std::vector<double*> xs;
    xs.push_back(t.ckpt[m].get());
    for (int n = start; n + 1 < end; ++n) {
      double* xin = xs.back();
      double* xout = seg[n - start].get();
      launch_plan_square_f64(xin, xout, pl, t.tiles.get(), t.offs.get(), s, t.branch[n] == 1);
      xs.push_back(xout);
    }
    for (int n = end - 1; n >= start; --n) {
      const double* X = xs[n - start];
      hipLaunchKernelGGL((k_symm_mm<double, 3>), dim3(ntf), dim3(kT), 0, s, G.get(), X, X,
                         Pm.get(), 1.0, 0.0, t.tiles_full.get(), t.offs.get(), nullptr, 0, nullptr,
                         (double*)nullptr, 0.0);
      GB_LAUNCH_CHECK();
      const double c1 = t.branch[n] == 0 ? 1.0 : -1.0, c2 = t.branch[n] == 0 ? 0.0 : 2.0;
      hipLaunchKernelGGL(k_sym_combine, cgrid, dim3(256), 0, s, Pm.get(), G.get(), G2.get(), c1,
                         c2, t.offs.get(), t.npad.get(), max_nt);
      GB_LAUNCH_CHECK();
      std::swap(G, G2);
    }
  }
  // vertex -> subgraph index and the deterministic assembly on H's pattern
  const int n = t.N;
  DBuf<int32_t> cnt(n, s), fill(n, s), vs_ptr(n + 1, s);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, kT)), dim3(kT), 0, s, cnt.get(), (int64_t)n);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, kT)), dim3(kT), 0, s, fill.get(), (int64_t)n);
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_vs_count, dim3(pl.n_sub), dim3(kT), 0, s, t.sub_ptr.get(), t.sub_idx.get(),
                     cnt.get());
  GB_LAUNCH_CHECK();
  exclusive_scan_i32(cnt.get(), vs_ptr.get(), n, s);
  int32_t tot = 0;
  GB_HIP(hipMemcpyAsync(&tot, vs_ptr.get() + n, 4, hipMemcpyDeviceToHost, s));
  GB_HIP(hipStreamSynchronize(s));
  DBuf<int32_t> vs_sub(tot, s), vs_loc(tot, s);
  hipLaunchKernelGGL(k_vs_fill, dim3(pl.n_sub), dim3(kT), 0, s, t.sub_ptr.get(), t.sub_idx.get(),
                     vs_ptr.get(), fill.get(), vs_sub.get(), vs_loc.get());
  GB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_vs_sort, dim3((n + kT - 1) / kT), dim3(kT), 0, s, n, vs_ptr.get(),
                     vs_sub.get(), vs_loc.get());
  GB_LAUNCH_CHECK();
  const int64_t slots = (int64_t)H.n * H.width;
  hipLaunchKernelGGL(k_assemble, dim3(grid_for(slots, kT)), dim3(kT), 0, s, H.col, H.n, H.width,
                     vs_ptr.get(), vs_sub.get(), vs_loc.get(), t.offs.get(), t.npad.get(), G.get(),
                     -1.0 / (t.emax - t.emin), G_H);
  GB_LAUNCH_CHECK();
  GB_HIP(hipStreamSynchronize(s));
}


// ---- finite-temperature Fermi-operator expansion (Eq. 7; terms by the recurrence of Eq. 5,
// per subgraph as in Eq. 6) ----------------------------------------------------------------

namespace {

// Ht = (2h - (e_max + e_min) delta) / (e_max - e_min) on H's ELL pattern (0 on padding)
__global__ void k_ht_ell(const int32_t* __restrict__ col, const double* __restrict__ val, int n,
                         int w, double emin, double emax, double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)n * w) return;
  const int i = (int)(p / w);
  const int32_t j = col[p];
  double v = 0.0;
  if (j >= 0) v = (2.0 * val[p] - (j == i ? emax + emin : 0.0)) / (emax - emin);
  out[p] = v;
}

// X[s] <- identity on the n_s x n_s part (the rest of the batch must already be zero)
__global__ __launch_bounds__(kT) void k_set_identity(double* __restrict__ X,
                                                     const int64_t* __restrict__ offs,
                                                     const int32_t* __restrict__ npad,
                                                     const int32_t* __restrict__ sub_ptr) {
  const int s = blockIdx.x;
  const int np = npad[s], n = sub_ptr[s + 1] - sub_ptr[s];
  double* x = X + offs[s];
  for (int j = threadIdx.x; j < n; j += kT) x[(int64_t)j * np + j] = 1.0;
}

__global__ void k_axpby(double* __restrict__ out, double a, const double* __restrict__ x, double b,
                        const double* __restrict__ y, int64_t n) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n; i += st) out[i] = a * x[i] + b * y[i];
}

// the summed core diagonal (first partial of each subgraph) into *out
__global__ __launch_bounds__(kT) void k_trace_total(const double* __restrict__ part, int n_sub,
                                                    double* __restrict__ out) {
  double t1, t2;
  sum_partials(part, n_sub, &t1, &t2);
  if (threadIdx.x == 0) *out = t1;
}

// Tn = P + P^T - Tp on 32 x 32 tile pairs (P^T through LDS), and with dacc: dacc += cn Tn
__global__ __launch_bounds__(256) void k_cheb_combine(const double* __restrict__ P,
                                                      const double* __restrict__ Tp,
                                                      double* __restrict__ Tn,
                                                      double* __restrict__ dacc, double cn,
                                                      const int64_t* __restrict__ offs,
                                                      const int32_t* __restrict__ npad,
                                                      int max_nt) {
  __shared__ double t[32][33];
  const int s = blockIdx.y;
  const int np = npad[s], nt = np / 32;
  const int bx = blockIdx.x % max_nt, by = blockIdx.x / max_nt;
  if (bx >= nt || by >= nt) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t off = offs[s];
  const double* p = P + off;
  for (int r = ty; r < 32; r += 8) t[r][tx] = p[(int64_t)(bx * 32 + r) * np + by * 32 + tx];
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t q = off + (int64_t)(by * 32 + r) * np + bx * 32 + tx;
    const double v = (P[q] + t[tx][r]) - Tp[q];
    Tn[q] = v;
    if (dacc) dacc[q] += cn * v;
  }
}

// One Chebyshev term, T_next = Ht T_cur + (Ht T_cur)^T - T_prev (= 2 Ht T_cur - T_prev, since
// T_cur is a polynomial in Ht), with dacc += cn T_next.  The product is formed on every tile
// and symmetrised explicitly: taking one triangle of Ht T_cur and mirroring it would turn the
// rounding part of the commutator [Ht, T_cur] into a symmetric error that the recurrence
// amplifies (the traces run away after about 200 terms).
void launch_cheb(const double* A, const double* Tc, const double* Tp, double* Tn, double* dacc,
                 double cn, double* P, const Plan& pl, const int4* tiles_full,
                 const int64_t* offs, const int32_t* npad, hipStream_t s) {
  const int ntf = (int)pl.full_launch.size();
  hipLaunchKernelGGL((k_symm_mm<double, 3>), dim3(ntf), dim3(kT), 0, s, A, Tc, Tc, P, 1.0, 0.0,
                     tiles_full, offs, nullptr, 0, nullptr, (double*)nullptr, 0.0);
  GB_LAUNCH_CHECK();
  const int max_nt = pl.max_npad / 32;
  hipLaunchKernelGGL(k_cheb_combine, dim3(max_nt * max_nt, pl.n_sub), dim3(256), 0, s, P, Tp, Tn,
                     dacc, cn, offs, npad, max_nt);
  GB_LAUNCH_CHECK();
}

int quad_nodes(int order, int n_nodes) { return n_nodes > 0 ? n_nodes : std::max(4 * (order + 1), 1024); }

double fermi(double e, double beta, double mu) { return 1.0 / (1.0 + std::exp(beta * (e - mu))); }

}  // namespace

void chebyshev_fermi(double emin, double emax, double beta, double mu, int order, int n_nodes,
                     double* c) {
  const int K = quad_nodes(order, n_nodes);
  const double mid = 0.5 * (emax + emin), half = 0.5 * (emax - emin);
  std::vector<double> th(K), f(K);
  for (int k = 0; k < K; ++k) {
    th[k] = M_PI * (k + 0.5) / K;
    f[k] = fermi(mid + half * std::cos(th[k]), beta, mu);
  }
  for (int n = 0; n <= order; ++n) {
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += std::cos(n * th[k]) * f[k];
    c[n] = acc * (2.0 / K) * (n == 0 ? 0.5 : 1.0);
  }
}

// sum_n c_n(mu) t_n = sum_k f(e_k; mu) w_k with w_k = (2/K) sum_n' t_n cos(n theta_k) (the n = 0
// term halved): the weights are formed once and each bisection step costs K exponentials.
double foe_solve_mu(const double* traces, int order, double emin, double emax, double beta,
                    double n_occ, int n_nodes) {
  const int K = quad_nodes(order, n_nodes);
  const double mid = 0.5 * (emax + emin), half = 0.5 * (emax - emin);
  std::vector<double> e(K), w(K);
  for (int k = 0; k < K; ++k) {
    const double th = M_PI * (k + 0.5) / K;
    e[k] = mid + half * std::cos(th);
    double acc = 0.5 * traces[0];
    for (int n = 1; n <= order; ++n) acc += std::cos(n * th) * traces[n];
    w[k] = acc * (2.0 / K);
  }
  auto excess = [&](double mu) {
    double t = 0.0;
    for (int k = 0; k < K; ++k) t += fermi(e[k], beta, mu) * w[k];
    return t - n_occ;
  };
  double lo = emin, hi = emax;
  const double glo = excess(lo), ghi = excess(hi);
  if (glo > 0.0 || ghi < 0.0)
    fail(GB_EINVAL, "n_occ = %g is outside the occupations [%g, %g] reachable in [e_min, e_max]",
         n_occ, glo + n_occ, ghi + n_occ);
  for (int it = 0; it < 400; ++it) {
    const double m = 0.5 * (lo + hi);
    if (!(m > lo && m < hi)) break;
    if (excess(m) < 0.0) lo = m;
    else hi = m;
  }
  return 0.5 * (lo + hi);
}

void foe(const gb_ell& H, int32_t n_occ, const gb_foe_opts& o, const Part& P, double emin,
         double emax, gb_ell& D, gb_foe_stats& st, hipStream_t s) {
  Timer t_all, t_stage;
  GB_HIP(hipEventRecord(t_all.a, s));
  const bool xcd = o.tile_order == 0;
  Plan pl = make_plan(P, nullptr, xcd);
  st.product_flops = pl.flops_alg;
  DBuf<int64_t> offs(pl.n_sub, s);
  DBuf<int32_t> npad(pl.n_sub, s);
  GB_HIP(hipMemcpyAsync(offs.get(), pl.off.data(), pl.n_sub * 8, hipMemcpyHostToDevice, s));
  GB_HIP(hipMemcpyAsync(npad.get(), pl.npad.data(), pl.n_sub * 4, hipMemcpyHostToDevice, s));
  DBuf<int4> tiles = upload_tiles(pl, s);
  const int N = H.n;
  const int M = o.order;

  // gather Ht into the batch
  GB_HIP(hipEventRecord(t_stage.a, s));
  const int64_t slots = (int64_t)H.n * H.width;
  DBuf<double> ht(slots, s);
  hipLaunchKernelGGL(k_ht_ell, dim3(grid_for(slots, kT)), dim3(kT), 0, s, H.col, H.val, H.n,
                     H.width, emin, emax, ht.get());
  GB_LAUNCH_CHECK();
  const size_t lds_g = (size_t)pl.max_npad * 8 + (size_t)P.max_sub * 4 + 64;
  if (lds_g > 160 * 1024) fail(GB_EUNSUPPORTED, "subgraph of %d vertices too large", P.max_sub);
  const dim3 ggrid(pl.n_sub, (pl.max_npad + kRows - 1) / kRows);
  WsLease ws;  // cached batch buffers: Ht, three Chebyshev terms, the running sum
  double* const A = ws->get<double>(0, pl.total, s);
  double* const B0 = ws->get<double>(1, pl.total, s);
  double* const B1 = ws->get<double>(2, pl.total, s);
  double* const B2 = ws->get<double>(3, pl.total, s);
  double* const Dacc = ws->get<double>(4, pl.total, s);
  double* const Pm = ws->get<double>(5, pl.total, s);  // the full product Ht T_n
  hipLaunchKernelGGL(k_gather<double>, ggrid, dim3(kT), lds_g, s, H.col, ht.get(), H.width,
                     P.core_ptr.get(), P.sub_ptr.get(), P.sub_idx.get(), offs.get(), npad.get(),
                     A, 1.0);
  GB_LAUNCH_CHECK();
  GB_HIP(hipEventRecord(t_stage.b, s));
  GB_HIP(hipStreamSynchronize(s));
  st.ms_gather = elapsed(t_stage.a, t_stage.b);
  DBuf<int4> tiles_full(pl.full_launch.size(), s);
  GB_HIP(hipMemcpyAsync(tiles_full.get(), pl.full_launch.data(),
                        pl.full_launch.size() * sizeof(int4), hipMemcpyHostToDevice, s));

  double t0 = 0;  // t_0 = sum of the core sizes
  for (int q = 0; q < P.n_sub; ++q) t0 += P.h_core_ptr[q + 1] - P.h_core_ptr[q];
  std::vector<double> traces(M + 1, 0.0);
  DBuf<double> part(2 * (size_t)pl.n_sub, s), tdev(M + 1, s);
  const int gfill = grid_for(pl.total, kT, 65536);
  std::deque<Timer> marks;
  auto record_trace = [&](const double* X, int n) {
    hipLaunchKernelGGL(k_trace_rows<double>, dim3(pl.n_sub), dim3(kT), 0, s, X, offs.get(),
                       npad.get(), P.core_ptr.get(), part.get(), nullptr, 1.0, 1.0);
    hipLaunchKernelGGL(k_trace_total, dim3(1), dim3(kT), 0, s, part.get(), pl.n_sub,
                       tdev.get() + n);
    GB_LAUNCH_CHECK();
  };
  // one pass of the recurrence; with c: the running sum in Dacc
  auto pass = [&](const double* c) {
    double* tp = B0;
    double* tc = B1;
    double* tn = B2;
    hipLaunchKernelGGL(k_fill, dim3(gfill), dim3(kT), 0, s, tp, pl.total, 0.0);
    GB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_set_identity, dim3(pl.n_sub), dim3(kT), 0, s, tp, offs.get(), npad.get(),
                       P.sub_ptr.get());
    GB_LAUNCH_CHECK();
    GB_HIP(hipMemcpyAsync(tc, A, pl.total * 8, hipMemcpyDeviceToDevice, s));
    if (c) {
      hipLaunchKernelGGL(k_axpby, dim3(gfill), dim3(kT), 0, s, Dacc, c[0], tp, c[1], tc,
                         pl.total);
      GB_LAUNCH_CHECK();
    }
    record_trace(tc, 1);
    for (int n = 1; n < M; ++n) {
      marks.emplace_back();
      GB_HIP(hipEventRecord(marks.back().a, s));
      launch_cheb(A, tc, tp, tn, c ? Dacc : nullptr, c ? c[n + 1] : 0.0, Pm, pl,
                  tiles_full.get(), offs.get(), npad.get(), s);
      GB_HIP(hipEventRecord(marks.back().b, s));
      record_trace(tn, n + 1);
      double* r = tp;
      tp = tc;
      tc = tn;
      tn = r;
    }
    GB_HIP(hipMemcpyAsync(traces.data() + 1, tdev.get() + 1, M * 8, hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    traces[0] = t0;
    ++st.passes;
  };

  GB_HIP(hipEventRecord(t_stage.a, s));
  std::vector<double> c(M + 1);
  double mu = o.mu;
  if (std::isnan(mu)) {
    pass(nullptr);
    mu = foe_solve_mu(traces.data(), M, emin, emax, o.beta, (double)n_occ, o.n_nodes);
  }
  chebyshev_fermi(emin, emax, o.beta, mu, M, o.n_nodes, c.data());
  pass(c.data());
  GB_HIP(hipEventRecord(t_stage.b, s));
  GB_HIP(hipStreamSynchronize(s));
  st.ms_terms = elapsed(t_stage.a, t_stage.b);
  for (auto& t : marks) st.ms_product += elapsed(t.a, t.b);
  st.n_product = (int)marks.size();
  st.mu = mu;
  double tr = 0.0;
  for (int n = 0; n <= M; ++n) tr += c[n] * traces[n];
  st.trace = tr;
  st.coef_tail = std::fabs(c[M]) + std::fabs(c[M - 1]);
  if (o.traces) std::memcpy(o.traces, traces.data(), (M + 1) * sizeof(double));

  GB_HIP(hipEventRecord(t_stage.a, s));
  hipLaunchKernelGGL(k_scatter<double>, dim3(N), dim3(kT), 0, s, Dacc, offs.get(),
                     npad.get(), P.sub_ptr.get(), P.sub_idx.get(), P.sub_pos.get(),
                     P.col_sub.get(), P.col_loc.get(), D.width, D.col, D.val);
  GB_LAUNCH_CHECK();
  GB_HIP(hipEventRecord(t_stage.b, s));
  GB_HIP(hipEventRecord(t_all.b, s));
  GB_HIP(hipStreamSynchronize(s));
  st.ms_scatter = elapsed(t_stage.a, t_stage.b);
  st.ms_total += elapsed(t_all.a, t_all.b);
}

}  // namespace gbi
