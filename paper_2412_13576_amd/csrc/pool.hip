// Candidate pool maintenance on gfx950: clearing, the exact kernel check
// A g = 0 (condition C1), lexicographic sorting and gathering of int8 keys.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "graver_internal.h"
#include "pool_device.h"

namespace graver {

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t value) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = value;
}

hipError_t launch_fill_u64(hipStream_t s, uint64_t* p, uint64_t n, uint64_t value) {
  int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

hipError_t launch_pool_clear(hipStream_t s, PoolDev p) {
  uint64_t n = p.tmask + 1;
  int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, s, p.table, n, (uint64_t)0);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<uint64_t*>(p.count),
                     (uint64_t)2, (uint64_t)0);
  return hipGetLastError();
}

// Insert the rows of the candidate log into the pool, one thread per row;
// all-zero rows are unused slots (a candidate is never zero).
__global__ void k_log_insert(LogDev log, PoolDev pool) {
  const uint32_t nrows = min(*log.count, log.cap);
  const int nwords = log.stride / 8;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += gridDim.x * blockDim.x) {
    const uint64_t* key = reinterpret_cast<const uint64_t*>(log.rows + (size_t)r * log.stride);
    bool nz = false;
    for (int w = 0; w < nwords; ++w) nz |= key[w] != 0;
    if (!nz) continue;
    pool_insert(pool, key, hash_key_words(key, nwords));
  }
}

hipError_t launch_log_insert(hipStream_t s, LogDev log, PoolDev pool) {
  unsigned blocks = (unsigned)((log.cap + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_log_insert, dim3(blocks), dim3(256), 0, s, log, pool);
  return hipGetLastError();
}

// Condition C1, A g = 0 exactly, for every pool key.  A is given as CSR
// (row_ptr m+1, col and val per nonzero).  A block handles 4 keys per round
// (one per wave): the key rows are staged in LDS with coalesced loads, then
// lane r of each wave forms the sums of rows r, r+64, ... over the row's
// nonzeros in int64 (|A_ij| < 2^31 and |g_j| <= 127 with n <= 4096 keep every
// partial sum below 2^63).
__global__ void k_verify(const int8_t* keys, int stride, uint32_t count, int m, const int32_t* __restrict__ rp,
                         const int32_t* __restrict__ col, const int64_t* __restrict__ val, unsigned int* bad) {
  extern __shared__ __align__(16) int8_t sk[];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int8_t* key = sk + (size_t)wid * stride;
  const int words = stride / 4;
  for (uint32_t base = blockIdx.x * 4u; base < count; base += gridDim.x * 4u) {
    const uint32_t k = base + (uint32_t)wid;
    if (k < count) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(keys + (size_t)k * stride);
      for (int w = lane; w < words; w += 64) reinterpret_cast<uint32_t*>(key)[w] = src[w];
    }
    __syncthreads();
    if (k < count) {
      int ok = 1;
      for (int i = lane; i < m; i += 64) {
        int64_t acc = 0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) acc += val[p] * (int64_t)key[col[p]];
        ok &= acc == 0 ? 1 : 0;
      }
      if (!ok) atomicAdd(bad, 1u);
    }
    __syncthreads();
  }
}

hipError_t launch_verify(hipStream_t s, PoolDev p, uint32_t count, int m, const int32_t* rp, const int32_t* col,
                         const int64_t* val, unsigned int* bad) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<uint64_t*>(bad),
                     (uint64_t)1, (uint64_t)0);
  if (count == 0) return hipGetLastError();
  const uint32_t rounds = (count + 3) / 4;
  const unsigned blocks = (unsigned)std::min<uint32_t>(rounds, 8192u);
  hipLaunchKernelGGL(k_verify, dim3(blocks), dim3(256), (size_t)4 * p.stride, s, p.keys, p.stride, count, m, rp,
                     col, val, bad);
  return hipGetLastError();
}

// Lexicographic order of signed bytes, component 0 first: flipping the sign
// bit maps int8 order to uint8 order, and reading 8 bytes big-endian turns
// the byte sequence order into integer order.
__device__ __forceinline__ int cmp_rows(const int8_t* keys, int stride, uint32_t a, uint32_t b) {
  const uint64_t* ka = reinterpret_cast<const uint64_t*>(keys + (size_t)a * stride);
  const uint64_t* kb = reinterpret_cast<const uint64_t*>(keys + (size_t)b * stride);
  for (int w = 0; w < stride / 8; ++w) {
    uint64_t x = ka[w], y = kb[w];
    if (x != y) {
      x = __builtin_bswap64(x ^ 0x8080808080808080ull);
      y = __builtin_bswap64(y ^ 0x8080808080808080ull);
      return x < y ? -1 : 1;
    }
  }
  return 0;
}

__device__ __forceinline__ bool row_greater(const int8_t* keys, int stride, uint32_t count,
                                            int by_l1, const int32_t* l1, uint32_t a, uint32_t b) {
  if (a >= count || b >= count) return a >= count && (b < count || a > b);
  if (by_l1 && l1[a] != l1[b]) return l1[a] > l1[b];
  int c = cmp_rows(keys, stride, a, b);
  return c != 0 ? c > 0 : a > b;
}

__global__ void k_bitonic_pass(uint32_t* idx, uint32_t p2, uint32_t k, uint32_t j, const int8_t* keys,
                               int stride, uint32_t count, int by_l1, const int32_t* l1) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p2) return;
  uint32_t partner = i ^ j;
  if (partner <= i) return;
  bool ascending = (i & k) == 0;
  uint32_t a = idx[i], b = idx[partner];
  if (row_greater(keys, stride, count, by_l1, l1, a, b) == ascending) {
    idx[i] = b;
    idx[partner] = a;
  }
}

// Bitonic passes with j < 2*blockDim run inside one block in LDS.
__global__ void k_bitonic_local(uint32_t* idx, uint32_t p2, uint32_t k, uint32_t jstart,
                                const int8_t* keys, int stride, uint32_t count, int by_l1,
                                const int32_t* l1) {
  __shared__ uint32_t sh[1024];
  uint32_t base = blockIdx.x * 1024;
  for (int t = threadIdx.x; t < 1024; t += blockDim.x) sh[t] = idx[base + t];
  __syncthreads();
  for (uint32_t j = jstart; j > 0; j >>= 1) {
    for (int t = threadIdx.x; t < 512; t += blockDim.x) {
      // t-th comparator of this block: lower element index
      uint32_t lo = (t / j) * 2 * j + (t % j);
      uint32_t gi = base + lo;
      bool ascending = (gi & k) == 0;
      uint32_t a = sh[lo], b = sh[lo + j];
      if (row_greater(keys, stride, count, by_l1, l1, a, b) == ascending) {
        sh[lo] = b;
        sh[lo + j] = a;
      }
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < 1024; t += blockDim.x) idx[base + t] = sh[t];
}

__global__ void k_iota(uint32_t* idx, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) idx[i] = i;
}

// Sorts row indices 0..count-1 of `keys` (lexicographic; by (l1, lex) when
// by_l1).  idx must hold the next power of two >= max(count, 1024) entries.
hipError_t launch_sort_keys(hipStream_t s, const int8_t* keys, int stride, int n, uint32_t count,
                            uint32_t* idx, uint32_t* tmp, int by_l1, const int32_t* l1) {
  (void)n;
  (void)tmp;
  uint32_t p2 = 1024;
  while (p2 < count) p2 <<= 1;
  hipLaunchKernelGGL(k_iota, dim3((p2 + 255) / 256), dim3(256), 0, s, idx, p2);
  if (count <= 1) return hipGetLastError();
  for (uint32_t k = 2; k <= p2; k <<= 1) {
    uint32_t j = k >> 1;
    for (; j >= 1024; j >>= 1)
      hipLaunchKernelGGL(k_bitonic_pass, dim3((p2 + 255) / 256), dim3(256), 0, s, idx, p2, k, j, keys,
                         stride, count, by_l1, l1);
    hipLaunchKernelGGL(k_bitonic_local, dim3(p2 / 1024), dim3(256), 0, s, idx, p2, k, j, keys, stride,
                       count, by_l1, l1);
  }
  return hipGetLastError();
}

__global__ void k_gather(const int8_t* keys, int stride, int n, const uint32_t* idx, uint32_t count,
                         int8_t* out, int out_stride) {
  uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t total = (uint64_t)count * n;
  if (t >= total) return;
  uint32_t r = (uint32_t)(t / n);
  int c = (int)(t % n);
  out[(size_t)r * out_stride + c] = keys[(size_t)idx[r] * stride + c];
}

hipError_t launch_gather_keys(hipStream_t s, const int8_t* keys, int stride, int n,
                              const uint32_t* idx, uint32_t count, int8_t* out, int out_stride) {
  uint64_t total = (uint64_t)count * n;
  if (total == 0) return hipGetLastError();
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, keys, stride,
                     n, idx, count, out, out_stride);
  return hipGetLastError();
}

}  // namespace graver
