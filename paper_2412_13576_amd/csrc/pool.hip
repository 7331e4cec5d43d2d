// Candidate pool maintenance on gfx950: clearing, the exact kernel check
// A g = 0 (condition C1), lexicographic sorting and gathering of int8 keys.
#include <hip/hip_runtime.h>

#include "graver_internal.h"
#include "pool_device.h"

namespace graver {

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t value) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = value;
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

// One thread per key: every row of A must annihilate the key exactly
// (condition C1).  A is staged in LDS as int32 when every |A_ij| < 2^23, so
// each row sum is below 2^23 * 127 * n < 2^63 in int64 accumulation; the key
// is read four bytes at a time.
__global__ void k_verify(const int8_t* keys, int stride, int n, uint32_t count, int m,
                         const int64_t* __restrict__ A, unsigned int* bad, int use_lds) {
  extern __shared__ int32_t sA[];
  if (use_lds) {
    for (int t = threadIdx.x; t < m * n; t += blockDim.x) sA[t] = (int32_t)A[t];
    __syncthreads();
  }
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const uint32_t* g4 = reinterpret_cast<const uint32_t*>(keys + (size_t)k * stride);
  const int nw = (n + 3) / 4;
  for (int i = 0; i < m; ++i) {
    int64_t s = 0;
    for (int w = 0; w < nw; ++w) {
      uint32_t word = g4[w];
      for (int b = 0; b < 4; ++b) {
        int j = 4 * w + b;
        if (j >= n) break;
        int gv = (int8_t)(word >> (8 * b));
        int64_t av = use_lds ? (int64_t)sA[i * n + j] : A[(size_t)i * n + j];
        s += av * gv;
      }
    }
    if (s != 0) {
      atomicAdd(bad, 1u);
      return;
    }
  }
}

hipError_t launch_verify(hipStream_t s, PoolDev p, uint32_t count, int m, const int64_t* A,
                         unsigned int* bad, int a_small) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<uint64_t*>(bad),
                     (uint64_t)1, (uint64_t)0);
  if (count == 0) return hipGetLastError();
  size_t lds = (size_t)m * p.n * sizeof(int32_t);
  int use_lds = a_small && lds <= 48 * 1024;
  hipLaunchKernelGGL(k_verify, dim3((count + 255) / 256), dim3(256), use_lds ? lds : 0, s, p.keys, p.stride,
                     p.n, count, m, A, bad, use_lds);
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
