// A set of int32 keys in LDS (open addressing, linear probing), and a block-wide bitonic sort:
// the graph and partition kernels use them for vertex sets whose members can lie anywhere in
// [0, n), so that their work and LDS do not grow with n.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gbi {

constexpr int32_t kHashEmpty = -1;

__device__ __forceinline__ uint32_t hset_slot(int32_t key, int log2_size) {
  return ((uint32_t)key * 2654435761u) >> (32 - log2_size);
}

// key (>= 0) into the set (size 2^log2_size, empty slots kHashEmpty); returns true if it was
// not there yet.  Safe under concurrent inserts by the whole block.  The caller keeps the set
// less than full.
__device__ __forceinline__ bool hset_insert(int32_t* keys, int log2_size, int32_t key) {
  const uint32_t mask = (1u << log2_size) - 1u;
  uint32_t s = hset_slot(key, log2_size);
  for (;;) {
    const int32_t old = atomicCAS(&keys[s], kHashEmpty, key);
    if (old == kHashEmpty) return true;
    if (old == key) return false;
    s = (s + 1) & mask;
  }
}

// slot of key, or -1 if absent (the set is not modified concurrently)
__device__ __forceinline__ int hset_find(const int32_t* keys, int log2_size, int32_t key) {
  const uint32_t mask = (1u << log2_size) - 1u;
  uint32_t s = hset_slot(key, log2_size);
  for (;;) {
    const int32_t k = keys[s];
    if (k == key) return (int)s;
    if (k == kHashEmpty) return -1;
    s = (s + 1) & mask;
  }
}

// v[0..p) ascending, p a power of two (pad with INT32_MAX); all NT threads of the block call it
template <int NT>
__device__ __forceinline__ void bitonic_sort(int32_t* v, int p) {
  for (int k = 2; k <= p; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < p; i += NT) {
        const int l = i ^ j;
        if (l > i) {
          const int32_t a = v[i], b = v[l];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            v[i] = b;
            v[l] = a;
          }
        }
      }
    }
  __syncthreads();
}

inline int ceil_log2(int64_t x) {
  int l = 0;
  while (((int64_t)1 << l) < x) ++l;
  return l;
}

}  // namespace gbi
