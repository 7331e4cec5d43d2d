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

// Insert the rows of the candidate log into the pool in two launches.  No
// key bytes are written while keys are compared, so the comparisons need no
// cross-workgroup ordering beyond the table word itself (on a multi-die
// device, acquire/release at device scope would flush and invalidate the
// per-die caches on every probe).
//   probe : a lane per log row (all-zero rows are unused slots; rows staged
//           in LDS a wave tile at a time) probes the
//           table with relaxed device-scope atomics; an empty slot is claimed
//           by a compare-and-swap with the entry (tag, kLogRow | row), so the
//           entry points at the log row itself.  A tag match is compared
//           against the log row or the pool key it points at, both written
//           by earlier launches.
//   commit: a lane per table slot finds the claimed log rows, the wave
//           copies them into the pool together (indices taken once per wave)
//           and each lane rewrites its entry to (tag, pool index).
constexpr uint32_t kLogRow = 0x80000000u;

// A wave takes a tile of consecutive log rows (at most kProbeTileBytes),
// copies it to LDS with coalesced loads, and then each lane probes with its
// own row read from LDS.  (With a lane reading its row word by word from
// global memory, a wave touches 64 rows' cache lines per load and the lines
// were fetched again and again: 12x the log's bytes.)
constexpr int kProbeWaves = 4;
constexpr int kProbeTileBytes = 8192;

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * kProbeWaves) void k_log_probe(LogDev log, PoolDev pool) {
  extern __shared__ __align__(16) uint64_t ptile[];  // kProbeWaves tiles of trows x stride bytes
  const uint32_t nrows = min(*log.count, log.cap);
  const int nwords = log.stride / 8;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int trows = min(64, kProbeTileBytes / log.stride);
  uint64_t* tile = ptile + (size_t)wid * trows * nwords;
  const uint64_t nwaves = (uint64_t)gridDim.x * kProbeWaves;
  for (uint64_t r0 = ((uint64_t)blockIdx.x * kProbeWaves + wid) * trows; r0 < nrows; r0 += nwaves * trows) {
    const int rows = (int)min((uint64_t)trows, nrows - r0);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(log.rows + r0 * log.stride);
    for (int w = lane; w < rows * nwords; w += 64) tile[w] = src[w];
    wave_sync_lds();
    if (lane < rows) {
      const uint32_t r = (uint32_t)r0 + (uint32_t)lane;
      const uint64_t* key = tile + (size_t)lane * nwords;
      bool nz = false;
      for (int w = 0; w < nwords; ++w) nz |= key[w] != 0;
      if (nz) {
        const uint64_t h = hash_key_words(key, nwords);
        const uint32_t tag = (uint32_t)(h >> 32) | 0x80000000u;
        uint64_t slot = h & pool.tmask;
        bool settled = false;
        for (int it = 0; it < kMaxProbeIters && !settled; ++it) {
          uint64_t e = __hip_atomic_load(&pool.table[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (e == 0) {
            uint64_t expected = 0;
            const uint64_t mine = ((uint64_t)tag << 32) | kLogRow | r;
            if (__hip_atomic_compare_exchange_strong(&pool.table[slot], &expected, mine, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
              settled = true;
              continue;
            }
            e = expected;  // the entry another thread just wrote
          }
          if ((uint32_t)(e >> 32) == tag) {
            const uint32_t lo = (uint32_t)e;
            const uint64_t* other = reinterpret_cast<const uint64_t*>(
                (lo & kLogRow) ? log.rows + (size_t)(lo & ~kLogRow) * log.stride : pool.keys + (size_t)lo * pool.stride);
            bool same = true;
            for (int w = 0; w < nwords && same; ++w) same = other[w] == key[w];
            if (same) {
              settled = true;
              continue;
            }
          }
          slot = (slot + 1) & pool.tmask;
        }
        if (!settled) atomicOr(&pool.count[2], 1u);
      }
    }
    wave_sync_lds();  // every lane's reads of the tile end before it is refilled
  }
}

// A wave owns kCommitIters * 64 consecutive slots (4096): it counts the claimed
// entries with ballots, takes that many pool indices with one atomic, then
// assigns them in slot order.
constexpr int kCommitIters = 64;

__global__ void k_log_commit(LogDev log, PoolDev pool) {
  const int nwords = pool.stride / 8;
  const uint64_t tsize = pool.tmask + 1;
  const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const uint64_t s0 = wave * 64 * kCommitIters;
  if (s0 >= tsize) return;
  uint32_t cnt = 0;
  for (int i = 0; i < kCommitIters; ++i) {
    const uint64_t slot = s0 + (uint64_t)i * 64 + lane;
    const uint64_t e = slot < tsize ? pool.table[slot] : 0ull;
    cnt += (uint32_t)__popcll(__ballot(e != 0 && ((uint32_t)e & kLogRow) != 0));
  }
  if (cnt == 0) return;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(&pool.count[0], cnt);
  base = __shfl(base, 0, 64);
  for (int i = 0; i < kCommitIters; ++i) {
    const uint64_t slot = s0 + (uint64_t)i * 64 + lane;
    const uint64_t e = slot < tsize ? pool.table[slot] : 0ull;
    const bool pending = e != 0 && ((uint32_t)e & kLogRow) != 0;
    const uint64_t wm = __ballot(pending);
    const uint32_t idx =
        base + __builtin_amdgcn_mbcnt_hi((uint32_t)(wm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)wm, 0u));
    const bool fits = pending && idx < pool.cap;
    if (pending && !fits) atomicOr(&pool.count[1], 1u);
    // the wave copies the claimed rows together, four rows per round trip,
    // each row's words spread over the lanes (coalesced loads and stores)
    uint64_t cm = __ballot(fits);
    while (cm != 0) {
      uint32_t srow[4], drow[4];
      int nr = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (cm == 0) break;
        const int l = __builtin_ctzll(cm);
        cm &= cm - 1;
        srow[u] = (uint32_t)__shfl((int)((uint32_t)e & ~kLogRow), l, 64);
        drow[u] = (uint32_t)__shfl((int)idx, l, 64);
        ++nr;
      }
      for (int w0 = 0; w0 < nwords; w0 += 128) {
        uint64_t v[4][2];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int w = w0 + lane + 64 * h;
            if (u < nr && w < nwords)
              v[u][h] = reinterpret_cast<const uint64_t*>(log.rows + (size_t)srow[u] * log.stride)[w];
          }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int w = w0 + lane + 64 * h;
            if (u < nr && w < nwords)
              reinterpret_cast<uint64_t*>(pool.keys + (size_t)drow[u] * pool.stride)[w] = v[u][h];
          }
      }
    }
    if (fits) pool.table[slot] = (e & 0xFFFFFFFF00000000ull) | idx;
    base += (uint32_t)__popcll(wm);
  }
}

hipError_t launch_log_insert(hipStream_t s, LogDev log, PoolDev pool) {
  unsigned blocks = (unsigned)((log.cap + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) blocks = 1;
  const int trows = std::min(64, kProbeTileBytes / log.stride);
  hipLaunchKernelGGL(k_log_probe, dim3(blocks), dim3(64 * kProbeWaves),
                     (size_t)kProbeWaves * trows * log.stride, s, log, pool);
  const uint64_t tsize = pool.tmask + 1;
  const uint64_t waves = (tsize + 64 * kCommitIters - 1) / (64 * kCommitIters);
  hipLaunchKernelGGL(k_log_commit, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, log, pool);
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
      // one count per key (the rows of A are spread over the lanes)
      if (__ballot(!ok) != 0 && lane == 0) atomicAdd(bad, 1u);
    }
    __syncthreads();
  }
}

// The same check for a small A: a thread per key, the block's keys staged
// in LDS with coalesced loads; every thread walks the same CSR entries, so
// their loads are uniform across the wave.
constexpr int kVerifyRows = 256;  // threads per block and most rows per tile
constexpr int kVerifyTileBytes = 32768;
constexpr int64_t kVerifyRowsMaxNnz = 4096;
__global__ __launch_bounds__(kVerifyRows) void k_verify_rows(const int8_t* keys, int stride, uint32_t count, int m,
                                                             int tile_rows, const int32_t* __restrict__ rp,
                                                             const int32_t* __restrict__ col,
                                                             const int64_t* __restrict__ val, unsigned int* bad) {
  extern __shared__ __align__(16) int8_t vtile[];  // tile_rows x stride
  const uint32_t r0 = blockIdx.x * (uint32_t)tile_rows;
  const int rows = (int)min((uint32_t)tile_rows, count - r0);
  const uint64_t* s64 = reinterpret_cast<const uint64_t*>(keys + (size_t)r0 * stride);
  for (int w = threadIdx.x; w < rows * stride / 8; w += blockDim.x) reinterpret_cast<uint64_t*>(vtile)[w] = s64[w];
  __syncthreads();
  if ((int)threadIdx.x >= rows) return;
  const int8_t* g = vtile + threadIdx.x * stride;
  bool ok = true;
  for (int i = 0; i < m; ++i) {
    int64_t acc = 0;
    for (int q = rp[i]; q < rp[i + 1]; ++q) acc += val[q] * (int64_t)g[col[q]];
    ok = ok && acc == 0;
  }
  if (!ok) atomicAdd(bad, 1u);
}

hipError_t launch_verify(hipStream_t s, PoolDev p, uint32_t count, int m, int64_t nnz, const int32_t* rp,
                         const int32_t* col, const int64_t* val, unsigned int* bad) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<uint64_t*>(bad),
                     (uint64_t)1, (uint64_t)0);
  if (count == 0) return hipGetLastError();
  if (nnz <= kVerifyRowsMaxNnz) {
    const int tr = std::max(1, std::min(kVerifyRows, kVerifyTileBytes / p.stride));
    hipLaunchKernelGGL(k_verify_rows, dim3((count + tr - 1) / tr), dim3(kVerifyRows), (size_t)tr * p.stride, s,
                       p.keys, p.stride, count, m, tr, rp, col, val, bad);
    return hipGetLastError();
  }
  const uint32_t rounds = (count + 3) / 4;
  const unsigned blocks = (unsigned)std::min<uint32_t>(rounds, 8192u);
  hipLaunchKernelGGL(k_verify, dim3(blocks), dim3(256), (size_t)4 * p.stride, s, p.keys, p.stride, count, m, rp,
                     col, val, bad);
  return hipGetLastError();
}

// Lexicographic sort of key rows (signed bytes, component 0 first) as
// (prefix, index) pairs.  Flipping the sign bit of each byte maps int8 order
// to uint8 order, and reading 8 bytes big-endian turns byte-sequence order
// into integer order, so the prefix (the first 8 bytes read that way) orders
// rows by their first 8 components.  Only rows whose prefixes tie are read
// again, from the second word on; remaining ties go to the smaller index, so
// the order is total and does not depend on the schedule.  Slots past count
// hold their own index and sort last.
__device__ __forceinline__ uint64_t order_word(uint64_t x) { return __builtin_bswap64(x ^ 0x8080808080808080ull); }

__device__ __forceinline__ bool pair_greater(const int8_t* keys, int stride, uint32_t count, uint64_t pa,
                                             uint32_t a, uint64_t pb, uint32_t b) {
  const bool va = a < count, vb = b < count;
  if (!va || !vb) return !va && (vb || a > b);
  if (pa != pb) return pa > pb;
  // tied prefixes are common (rows of one descent trajectory share long
  // runs of leading components): compare 64 bytes per round trip, four
  // 16-byte loads per row in flight
  const uint4* ka = reinterpret_cast<const uint4*>(keys + (size_t)a * stride);
  const uint4* kb = reinterpret_cast<const uint4*>(keys + (size_t)b * stride);
  const int nc = stride / 16;
  for (int c0 = 0; c0 < nc; c0 += 4) {
    uint4 x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = c0 + u < nc;
      x[u] = in ? ka[c0 + u] : make_uint4(0, 0, 0, 0);
      y[u] = in ? kb[c0 + u] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t x0 = (uint64_t)x[u].x | ((uint64_t)x[u].y << 32), y0 = (uint64_t)y[u].x | ((uint64_t)y[u].y << 32);
      if (x0 != y0) return order_word(x0) > order_word(y0);
      const uint64_t x1 = (uint64_t)x[u].z | ((uint64_t)x[u].w << 32), y1 = (uint64_t)y[u].z | ((uint64_t)y[u].w << 32);
      if (x1 != y1) return order_word(x1) > order_word(y1);
    }
  }
  return a > b;
}

__global__ void k_sort_init(const int8_t* keys, int stride, uint32_t count, uint32_t p2, uint64_t* pk,
                            uint32_t* pi) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p2) return;
  pi[i] = i;
  pk[i] = i < count ? order_word(*reinterpret_cast<const uint64_t*>(keys + (size_t)i * stride)) : ~0ull;
}

// one bitonic stage (k, j) with j >= 1024: thread = comparator
__global__ void k_bitonic_pass(uint64_t* pk, uint32_t* pi, uint32_t p2, uint32_t k, uint32_t j, const int8_t* keys,
                               int stride, uint32_t count) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= p2 / 2) return;
  const uint32_t lo = (t / j) * 2 * j + (t % j), hi = lo + j;
  const bool ascending = (lo & k) == 0;
  const uint64_t pa = pk[lo], pb = pk[hi];
  const uint32_t a = pi[lo], b = pi[hi];
  if (pair_greater(keys, stride, count, pa, a, pb, b) == ascending) {
    pk[lo] = pb;
    pk[hi] = pa;
    pi[lo] = b;
    pi[hi] = a;
  }
}

// every stage with j < 1024 of the merge steps k = kmin .. kmax (powers of
// two), inside 1024-element blocks held in LDS
__global__ __launch_bounds__(256) void k_bitonic_local(uint64_t* pk, uint32_t* pi, uint32_t kmin, uint32_t kmax,
                                                       const int8_t* keys, int stride, uint32_t count) {
  __shared__ uint64_t sk[1024];
  __shared__ uint32_t si[1024];
  const uint32_t base = blockIdx.x * 1024;
  for (int t = threadIdx.x; t < 1024; t += blockDim.x) {
    sk[t] = pk[base + t];
    si[t] = pi[base + t];
  }
  __syncthreads();
  for (uint32_t k = kmin; k <= kmax; k <<= 1) {
    for (uint32_t j = (k >> 1) < 512 ? (k >> 1) : 512; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < 512; t += blockDim.x) {
        const uint32_t lo = (t / j) * 2 * j + (t % j), hi = lo + j;
        const bool ascending = ((base + lo) & k) == 0;
        const uint64_t pa = sk[lo], pb = sk[hi];
        const uint32_t a = si[lo], b = si[hi];
        if (pair_greater(keys, stride, count, pa, a, pb, b) == ascending) {
          sk[lo] = pb;
          sk[hi] = pa;
          si[lo] = b;
          si[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < 1024; t += blockDim.x) {
    pk[base + t] = sk[t];
    pi[base + t] = si[t];
  }
}

// Sorts row indices 0..count-1 of `keys` lexicographically into idx.  idx
// and pk (scratch) must hold the next power of two >= max(count, 1024)
// entries.
hipError_t launch_sort_keys(hipStream_t s, const int8_t* keys, int stride, uint32_t count, uint32_t* idx,
                            uint64_t* pk) {
  uint32_t p2 = 1024;
  while (p2 < count) p2 <<= 1;
  hipLaunchKernelGGL(k_sort_init, dim3((p2 + 255) / 256), dim3(256), 0, s, keys, stride, count, p2, pk, idx);
  if (count <= 1) return hipGetLastError();
  hipLaunchKernelGGL(k_bitonic_local, dim3(p2 / 1024), dim3(256), 0, s, pk, idx, 2u, 1024u, keys, stride, count);
  for (uint32_t k = 2048; k <= p2; k <<= 1) {
    for (uint32_t j = k >> 1; j >= 1024; j >>= 1)
      hipLaunchKernelGGL(k_bitonic_pass, dim3((p2 / 2 + 255) / 256), dim3(256), 0, s, pk, idx, p2, k, j, keys,
                         stride, count);
    hipLaunchKernelGGL(k_bitonic_local, dim3(p2 / 1024), dim3(256), 0, s, pk, idx, k, k, keys, stride, count);
  }
  return hipGetLastError();
}

// a thread per byte, grid-stride (a dispatch counts at most 2^32 - 1 work-items)
__global__ void k_gather(const int8_t* keys, int stride, int n, const uint32_t* idx, uint32_t count,
                         int8_t* out, int out_stride) {
  const uint64_t total = (uint64_t)count * n;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t r = (uint32_t)(t / n);
    const int c = (int)(t % n);
    out[(size_t)r * out_stride + c] = keys[(size_t)idx[r] * stride + c];
  }
}

hipError_t launch_gather_keys(hipStream_t s, const int8_t* keys, int stride, int n,
                              const uint32_t* idx, uint32_t count, int8_t* out, int out_stride) {
  uint64_t total = (uint64_t)count * n;
  if (total == 0) return hipGetLastError();
  hipLaunchKernelGGL(k_gather, dim3(stride_grid(total)), dim3(256), 0, s, keys, stride, n, idx, count, out,
                     out_stride);
  return hipGetLastError();
}

}  // namespace graver
