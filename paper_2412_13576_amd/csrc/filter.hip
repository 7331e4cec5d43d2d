// Minimality filter with deduplication on gfx950 (condition C3; the
// conformal order of Section 1).  Stages:
//   canon   : each key -> representative of {g, -g} (first nonzero > 0)
//   dedup   : lexicographic sort, keep first of each run, drop 0
//   prep    : l1 norm, positive / negative support bit masks
//   order   : sort by (l1, lex) so every possible witness of g (strictly
//             smaller l1) sits in one prefix [0, lo(g))
//   pairs   : g dies if some h in the prefix, or -h, lies conformally below
//             it: support masks first (h's positive support inside g's
//             positive support, negative inside negative; swapped for -h),
//             then |h_i| <= |g_i| on the bytes
//   output  : survivors, sorted lexicographically
#include <hip/hip_runtime.h>

#include "graver_internal.h"
#include "pool_device.h"

namespace graver {

__global__ void k_canon(const int8_t* in, int64_t count, int n, int stride, int8_t* out) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int8_t* g = in + (size_t)k * n;
  int first = 0;
  for (int i = 0; i < n; ++i)
    if (g[i] != 0) {
      first = g[i];
      break;
    }
  int8_t* o = out + (size_t)k * stride;
  for (int i = 0; i < n; ++i) o[i] = first < 0 ? (int8_t)(-g[i]) : g[i];
  for (int i = n; i < stride; ++i) o[i] = 0;
}

__device__ __forceinline__ bool rows_equal(const int8_t* keys, int stride, uint32_t a, uint32_t b) {
  const uint64_t* ka = reinterpret_cast<const uint64_t*>(keys + (size_t)a * stride);
  const uint64_t* kb = reinterpret_cast<const uint64_t*>(keys + (size_t)b * stride);
  for (int w = 0; w < stride / 8; ++w)
    if (ka[w] != kb[w]) return false;
  return true;
}

__global__ void k_mark_unique(const int8_t* keys, int stride, const uint32_t* idx, uint32_t count,
                              uint32_t* flag) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t* k = reinterpret_cast<const uint64_t*>(keys + (size_t)idx[i] * stride);
  bool nz = false;
  for (int w = 0; w < stride / 8; ++w) nz |= k[w] != 0;
  bool first = i == 0 || !rows_equal(keys, stride, idx[i], idx[i - 1]);
  flag[i] = (nz && first) ? 1u : 0u;
}

// ---- exclusive scan of uint32 (order-preserving compaction) --------------
__global__ void k_scan_block(const uint32_t* in, uint32_t* out, uint32_t* bsum, uint32_t n) {
  __shared__ uint32_t wsum[16];
  uint32_t i = blockIdx.x * 1024 + threadIdx.x;
  uint32_t x = i < n ? in[i] : 0u;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t incl = x;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  if (threadIdx.x < 16) {
    uint32_t v = wsum[threadIdx.x];
    for (int o = 1; o < 16; o <<= 1) {
      uint32_t y = __shfl_up(v, o, 16);
      if ((int)threadIdx.x >= o) v += y;
    }
    wsum[threadIdx.x] = v;
  }
  __syncthreads();
  uint32_t base = wid ? wsum[wid - 1] : 0u;
  if (i < n) out[i] = base + incl - x;
  if (threadIdx.x == 1023 && bsum) bsum[blockIdx.x] = wsum[15];
}

__global__ void k_scan_add(uint32_t* out, const uint32_t* boff, uint32_t n) {
  uint32_t i = blockIdx.x * 1024 + threadIdx.x;
  if (i < n) out[i] += boff[blockIdx.x];
}

// Exclusive scan of n values; scratch must hold >= n/1024 + n/2^20 + 64 entries.
static void scan_exclusive(hipStream_t s, const uint32_t* in, uint32_t* out, uint32_t n,
                           uint32_t* scratch) {
  uint32_t blocks = (n + 1023) / 1024;
  if (blocks <= 1) {
    hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(1024), 0, s, in, out, (uint32_t*)nullptr, n);
    return;
  }
  uint32_t* bs = scratch;
  uint32_t* bo = scratch + blocks;
  hipLaunchKernelGGL(k_scan_block, dim3(blocks), dim3(1024), 0, s, in, out, bs, n);
  scan_exclusive(s, bs, bo, blocks, scratch + 2 * (size_t)blocks);
  hipLaunchKernelGGL(k_scan_add, dim3(blocks), dim3(1024), 0, s, out, bo, n);
}

__global__ void k_compact_rows(const int8_t* src, int stride, const uint32_t* idx, const uint32_t* flag,
                               const uint32_t* pos, uint32_t count, int8_t* dst) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count || !flag[i]) return;
  const uint64_t* a = reinterpret_cast<const uint64_t*>(src + (size_t)(idx ? idx[i] : i) * stride);
  uint64_t* b = reinterpret_cast<uint64_t*>(dst + (size_t)pos[i] * stride);
  for (int w = 0; w < stride / 8; ++w) b[w] = a[w];
}

// l1 norm and support masks (W words of positive support, then W of negative).
__global__ void k_prep(const int8_t* keys, int stride, int n, uint32_t count, int W, int32_t* l1,
                       uint64_t* mask) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int8_t* g = keys + (size_t)k * stride;
  int32_t s = 0;
  uint64_t* mk = mask + (size_t)k * 2 * W;
  for (int w = 0; w < W; ++w) {
    uint64_t p = 0, q = 0;
    for (int b = 0; b < 64; ++b) {
      int i = w * 64 + b;
      if (i >= n) break;
      int v = g[i];
      s += v < 0 ? -v : v;
      if (v > 0) p |= 1ull << b;
      if (v < 0) q |= 1ull << b;
    }
    mk[w] = p;
    mk[W + w] = q;
  }
  l1[k] = s;
}

__global__ void k_gather_rows(const int8_t* src, int stride, const uint32_t* idx, uint32_t count,
                              int8_t* dst, const int32_t* l1src, int32_t* l1dst, const uint64_t* msrc,
                              uint64_t* mdst, int W) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t j = idx[i];
  const uint64_t* a = reinterpret_cast<const uint64_t*>(src + (size_t)j * stride);
  uint64_t* b = reinterpret_cast<uint64_t*>(dst + (size_t)i * stride);
  for (int w = 0; w < stride / 8; ++w) b[w] = a[w];
  l1dst[i] = l1src[j];
  for (int w = 0; w < 2 * W; ++w) mdst[(size_t)i * 2 * W + w] = msrc[(size_t)j * 2 * W + w];
}

// lo[p] = first position whose l1 equals l1[p] (l1 sorted ascending).
__global__ void k_level_start(const int32_t* l1, uint32_t count, uint32_t* lo) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  int32_t key = l1[p];
  uint32_t a = 0, b = p;
  while (a < b) {
    uint32_t mid = (a + b) / 2;
    if (l1[mid] < key) a = mid + 1; else b = mid;
  }
  lo[p] = a;
}

constexpr int kTile = 64;

__device__ __forceinline__ bool magnitude_below(const int8_t* h, const int8_t* g, int n) {
  for (int i = 0; i < n; ++i) {
    int a = h[i], b = g[i];
    if ((a < 0 ? -a : a) > (b < 0 ? -b : b)) return false;
  }
  return true;
}

__global__ void k_pairs(const int8_t* keys, int stride, int n, uint32_t count, int W,
                        const uint64_t* __restrict__ mask, const uint32_t* __restrict__ lo,
                        uint32_t* alive) {
  extern __shared__ uint64_t tile[];  // kTile x 2W
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = p < count;
  uint32_t my_lo = valid ? lo[p] : 0;
  uint32_t last = min(count, (blockIdx.x + 1) * blockDim.x) - 1;
  uint32_t block_hi = lo[last];
  bool dead = false;
  uint64_t gp[8], gn[8];
  const int Wr = W < 8 ? W : 8;
  if (valid) {
    for (int w = 0; w < Wr; ++w) {
      gp[w] = mask[(size_t)p * 2 * W + w];
      gn[w] = mask[(size_t)p * 2 * W + W + w];
    }
  }
  const int8_t* g = keys + (size_t)p * stride;
  for (uint32_t base = 0; base < block_hi; base += kTile) {
    __syncthreads();
    for (int t = threadIdx.x; t < kTile * 2 * W; t += blockDim.x) {
      uint32_t h = base + t / (2 * W);
      tile[t] = h < count ? mask[(size_t)base * 2 * W + t] : 0ull;
    }
    __syncthreads();
    if (!valid || dead || base >= my_lo) continue;
    uint32_t hend = min((uint32_t)kTile, my_lo - base);
    for (uint32_t q = 0; q < hend && !dead; ++q) {
      const uint64_t* hm = tile + (size_t)q * 2 * W;
      bool plus = true, minus = true;
      for (int w = 0; w < W && (plus || minus); ++w) {
        uint64_t hp = hm[w], hn = hm[W + w];
        uint64_t mp = w < 8 ? gp[w] : mask[(size_t)p * 2 * W + w];
        uint64_t mn = w < 8 ? gn[w] : mask[(size_t)p * 2 * W + W + w];
        plus = plus && ((hp & ~mp) | (hn & ~mn)) == 0;
        minus = minus && ((hp & ~mn) | (hn & ~mp)) == 0;
      }
      if (plus || minus) {
        const int8_t* h = keys + (size_t)(base + q) * stride;
        if (magnitude_below(h, g, n)) dead = true;
      }
    }
  }
  if (valid) alive[p] = dead ? 0u : 1u;
}

hipError_t launch_filter(hipStream_t s, graver_ctx* ctx, int n, const int8_t* in, int64_t count_in,
                         int8_t* out, int64_t cap, int64_t* count_out, graver_status* st) {
  *count_out = 0;
  const int stride = key_stride(n);
  const int W = (n + 63) / 64;
  const uint32_t cnt = (uint32_t)count_in;
  if (cnt == 0) return hipStreamSynchronize(s);
  uint32_t p2 = 1024;
  while (p2 < cnt) p2 <<= 1;
  int8_t* canon = (int8_t*)ws_get(ctx, WS_F_CANON, (size_t)cnt * stride, st);
  uint32_t* idx = (uint32_t*)ws_get(ctx, WS_SORT_IDX, (size_t)p2 * 4, st);
  uint32_t* flag = (uint32_t*)ws_get(ctx, WS_FLAGS, (size_t)cnt * 4 + 64, st);
  uint32_t* pos = (uint32_t*)ws_get(ctx, WS_SCAN, (size_t)cnt * 4 + 64, st);
  uint32_t* scr = (uint32_t*)ws_get(ctx, WS_SCAN2, ((size_t)cnt / 512 + 256) * 4, st);
  int8_t* uniq = (int8_t*)ws_get(ctx, WS_F_UNIQ, (size_t)cnt * stride, st);
  int32_t* l1 = (int32_t*)ws_get(ctx, WS_F_L1, (size_t)cnt * 8, st);
  uint64_t* msk = (uint64_t*)ws_get(ctx, WS_F_MASK, (size_t)cnt * 4 * W * 8, st);
  uint32_t* lo = (uint32_t*)ws_get(ctx, WS_F_LO, (size_t)cnt * 4, st);
  uint32_t* alive = (uint32_t*)ws_get(ctx, WS_F_ALIVE, (size_t)cnt * 4 + 64, st);
  int8_t* surv = (int8_t*)ws_get(ctx, WS_F_OUT, (size_t)cnt * stride, st);
  if (!canon || !idx || !flag || !pos || !scr || !uniq || !l1 || !msk || !lo || !alive || !surv)
    return hipSuccess;
  const unsigned b256 = (cnt + 255) / 256;
  hipLaunchKernelGGL(k_canon, dim3(b256), dim3(256), 0, s, in, (int64_t)cnt, n, stride, canon);
  launch_sort_keys(s, canon, stride, n, cnt, idx, nullptr, 0, nullptr);
  hipLaunchKernelGGL(k_mark_unique, dim3(b256), dim3(256), 0, s, canon, stride, idx, cnt, flag);
  scan_exclusive(s, flag, pos, cnt, scr);
  uint32_t hlast[2] = {0, 0};
  hipMemcpyAsync(&hlast[0], pos + cnt - 1, 4, hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(&hlast[1], flag + cnt - 1, 4, hipMemcpyDeviceToHost, s);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const uint32_t U = hlast[0] + hlast[1];
  if (U == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact_rows, dim3(b256), dim3(256), 0, s, canon, stride, idx, flag, pos, cnt, uniq);
  const unsigned u256 = (U + 255) / 256;
  int32_t* l1b = l1 + cnt;
  uint64_t* mskb = msk + (size_t)cnt * 2 * W;
  hipLaunchKernelGGL(k_prep, dim3(u256), dim3(256), 0, s, uniq, stride, n, U, W, l1, msk);
  launch_sort_keys(s, uniq, stride, n, U, idx, nullptr, 1, l1);
  hipLaunchKernelGGL(k_gather_rows, dim3(u256), dim3(256), 0, s, uniq, stride, idx, U, canon, l1, l1b,
                     msk, mskb, W);
  hipLaunchKernelGGL(k_level_start, dim3(u256), dim3(256), 0, s, l1b, U, lo);
  size_t shmem = (size_t)kTile * 2 * W * sizeof(uint64_t);
  hipLaunchKernelGGL(k_pairs, dim3(u256), dim3(256), shmem, s, canon, stride, n, U, W, mskb, lo, alive);
  scan_exclusive(s, alive, pos, U, scr);
  hipMemcpyAsync(&hlast[0], pos + U - 1, 4, hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(&hlast[1], alive + U - 1, 4, hipMemcpyDeviceToHost, s);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const uint32_t R = hlast[0] + hlast[1];
  hipLaunchKernelGGL(k_compact_rows, dim3(u256), dim3(256), 0, s, canon, stride, (const uint32_t*)nullptr,
                     alive, pos, U, surv);
  *count_out = R;
  if ((int64_t)R > cap) {
    *st = set_error(GRAVER_E_CAPACITY, "keys_cap too small for the filtered set");
    return hipSuccess;
  }
  launch_sort_keys(s, surv, stride, n, R, idx, nullptr, 0, nullptr);
  launch_gather_keys(s, surv, stride, n, idx, R, out, n);
  return hipStreamSynchronize(s);
}

}  // namespace graver
