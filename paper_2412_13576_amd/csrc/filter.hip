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

#include <algorithm>
#include <vector>

#include "graver_internal.h"
#include "pool_device.h"

namespace graver {

__global__ void k_zero32(uint32_t* a, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// Tiles of consecutive rows are staged through LDS: the rows of a tile are
// one contiguous byte range in both layouts (n bytes per row in, stride
// bytes out), so loads and stores are coalesced and each thread then works
// on one row inside LDS.  A block has kTileRows threads; a tile holds up to
// kTileRows rows and at most kTileBytes bytes.
constexpr int kTileRows = 256;
constexpr int kTileBytes = 32768;
inline int tile_rows_for(int stride) {
  const int r = kTileBytes / stride;
  return r < 1 ? 1 : (r > kTileRows ? kTileRows : r);
}

// each key -> the representative of {g, -g} whose first nonzero is positive,
// written at the padded stride with zero padding
__global__ __launch_bounds__(kTileRows) void k_canon(const int8_t* in, int64_t count, int n, int stride,
                                                     int tile_rows, int8_t* out) {
  extern __shared__ __align__(16) int8_t ctile[];  // tile_rows x stride
  const int64_t r0 = (int64_t)blockIdx.x * tile_rows;
  const int rows = (int)min((int64_t)tile_rows, count - r0);
  const int8_t* src = in + r0 * n;
  if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(in) & 3) == 0) {
    const int words = rows * n / 4;
    const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src);
    for (int w = threadIdx.x; w < words; w += blockDim.x) {
      const int b = 4 * w, r = b / n;
      *reinterpret_cast<uint32_t*>(ctile + r * stride + (b - r * n)) = s32[w];
    }
  } else {
    for (int b = threadIdx.x; b < rows * n; b += blockDim.x) {
      const int r = b / n;
      ctile[r * stride + (b - r * n)] = src[b];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < rows) {
    int8_t* g = ctile + threadIdx.x * stride;
    int first = 0;
    for (int i = 0; i < n && first == 0; ++i) first = g[i];
    if (first < 0)
      for (int i = 0; i < n; ++i) g[i] = (int8_t)(-g[i]);
    for (int i = n; i < stride; ++i) g[i] = 0;
  }
  __syncthreads();
  const int words = rows * stride / 8;
  const uint64_t* t64 = reinterpret_cast<const uint64_t*>(ctile);
  uint64_t* o64 = reinterpret_cast<uint64_t*>(out + r0 * stride);
  for (int w = threadIdx.x; w < words; w += blockDim.x) o64[w] = t64[w];
}

// (64 bytes per round trip: rows with equal prefixes often share long runs)
__device__ __forceinline__ bool rows_equal(const int8_t* keys, int stride, uint32_t a, uint32_t b) {
  const uint4* ka = reinterpret_cast<const uint4*>(keys + (size_t)a * stride);
  const uint4* kb = reinterpret_cast<const uint4*>(keys + (size_t)b * stride);
  const int nc = stride / 16;
  for (int c0 = 0; c0 < nc; c0 += 4) {
    uint32_t diff = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c0 + u < nc) {
        const uint4 x = ka[c0 + u], y = kb[c0 + u];
        diff |= (x.x ^ y.x) | (x.y ^ y.y) | (x.z ^ y.z) | (x.w ^ y.w);
      }
    }
    if (diff) return false;
  }
  return true;
}

// flag[i] = 1 when sorted row i is nonzero and differs from row i - 1; pk
// holds the sorted 8-byte prefixes, so rows are read only on a prefix tie
// (or when the prefix is that of a zero row)
__global__ void k_mark_unique(const int8_t* keys, int stride, const uint32_t* idx, const uint64_t* pk,
                              uint32_t count, uint32_t* flag) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  constexpr uint64_t kZeroPrefix = 0x8080808080808080ull;
  const uint64_t p = pk[i];
  bool nz = p != kZeroPrefix;
  if (!nz) {
    const uint64_t* k = reinterpret_cast<const uint64_t*>(keys + (size_t)idx[i] * stride);
    for (int w = 1; w < stride / 8; ++w) nz |= k[w] != 0;
  }
  const bool first = i == 0 || p != pk[i - 1] || !rows_equal(keys, stride, idx[i], idx[i - 1]);
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

// Row movers run a thread per 8-byte word, so the lanes that copy one row
// read and write whole cache lines.
// (grid-stride: count rows of stride / 8 words can exceed the 2^32 - 1
// work-items of one dispatch)
__global__ void k_compact_rows(const int8_t* src, int stride, const uint32_t* idx, const uint32_t* flag,
                               const uint32_t* pos, uint32_t count, int8_t* dst) {
  const int L = stride / 8;
  const uint64_t total = (uint64_t)count * L;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = t / L;
    const int w = (int)(t - i * L);
    if (!flag[i]) continue;
    const uint64_t* a = reinterpret_cast<const uint64_t*>(src + (size_t)(idx ? idx[i] : (uint32_t)i) * stride);
    reinterpret_cast<uint64_t*>(dst + (size_t)pos[i] * stride)[w] = a[w];
  }
}

// ---- LSD radix sort of 64-bit keys, 4 bits per pass ----------------------
// A block owns a tile of kRadixTile consecutive elements, taken in rounds of
// 256 in element order; the rank of an element among equal digits of its
// round comes from wave ballots, so every pass is stable.
constexpr uint32_t kRadixTile = 2048;

__global__ void k_radix_hist(const uint64_t* keys, uint32_t n, int shift, uint32_t nblocks, uint32_t* hist) {
  __shared__ uint32_t c[16];
  if (threadIdx.x < 16) c[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kRadixTile;
  for (uint32_t r = 0; r < kRadixTile / 256; ++r) {
    const uint32_t e = base + r * 256 + threadIdx.x;
    if (e < n) atomicAdd(&c[(keys[e] >> shift) & 15], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 16) hist[threadIdx.x * nblocks + blockIdx.x] = c[threadIdx.x];
}

__global__ void k_radix_scatter(const uint64_t* keys, uint64_t* out, uint32_t n, int shift, uint32_t nblocks,
                                const uint32_t* off) {
  __shared__ uint32_t wc[4][16];
  __shared__ uint32_t run[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (threadIdx.x < 16) run[threadIdx.x] = off[threadIdx.x * nblocks + blockIdx.x];
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t base = blockIdx.x * kRadixTile;
  for (uint32_t r = 0; r < kRadixTile / 256; ++r) {
    const uint32_t e = base + r * 256 + threadIdx.x;
    const bool valid = e < n;
    const uint64_t k = valid ? keys[e] : 0ull;
    const int d = valid ? (int)((k >> shift) & 15) : 16;
    uint32_t rank = 0;
    for (int v = 0; v < 16; ++v) {
      const uint64_t m = __ballot(d == v);
      if (lane == 0) wc[wid][v] = (uint32_t)__popcll(m);
      if (d == v) rank = (uint32_t)__popcll(m & lt);
    }
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int w = 0; w < wid; ++w) pos += wc[w][d];
      out[pos] = k;
    }
    __syncthreads();
    if (threadIdx.x < 16) run[threadIdx.x] += wc[0][threadIdx.x] + wc[1][threadIdx.x] + wc[2][threadIdx.x] + wc[3][threadIdx.x];
    __syncthreads();
  }
}

__global__ void k_l1_keys(const int32_t* l1, uint32_t count, int bits_pos, uint64_t* keys) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) keys[k] = ((uint64_t)(uint32_t)l1[k] << bits_pos) | k;
}

__global__ void k_low_bits(const uint64_t* keys, uint32_t count, int bits_pos, uint32_t* idx) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) idx[i] = (uint32_t)(keys[i] & ((1ull << bits_pos) - 1ull));
}

__global__ void k_scatter_flags(const uint32_t* idx, const uint32_t* alive, uint32_t count, uint32_t* flag_lex) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < count) flag_lex[idx[p]] = alive[p];
}

// rows with flag set, in order, into out (n bytes per row); one thread per
// 4-byte word of a row, so consecutive threads touch consecutive bytes
__global__ void k_compact_out(const int8_t* src, int stride, const uint32_t* flag, const uint32_t* pos,
                              uint32_t count, int n, int8_t* out) {
  const int nw = (n + 3) / 4;
  const uint64_t total = (uint64_t)count * nw;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = t / nw;
    const int w = (int)(t % nw);
    if (!flag[i]) continue;
    const int8_t* a = src + (size_t)i * stride + 4 * w;
    int8_t* b = out + (size_t)pos[i] * n + 4 * w;
    if ((n & 3) == 0) {
      *reinterpret_cast<uint32_t*>(b) = *reinterpret_cast<const uint32_t*>(a);
    } else {
      for (int j = 0; j < 4 && 4 * w + j < n; ++j) b[j] = a[j];
    }
  }
}

// Sorts keys[0..n) by bits [0, nbits); tmp is scratch of n entries; returns
// the buffer that holds the result.
static uint64_t* radix_sort_u64(hipStream_t s, uint64_t* keys, uint64_t* tmp, uint32_t n, int nbits, uint32_t* hist,
                                uint32_t* off, uint32_t* scratch) {
  const uint32_t nblocks = (n + kRadixTile - 1) / kRadixTile;
  for (int shift = 0; shift < nbits; shift += 4) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(256), 0, s, keys, n, shift, nblocks, hist);
    scan_exclusive(s, hist, off, 16 * nblocks, scratch);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(256), 0, s, keys, tmp, n, shift, nblocks, off);
    uint64_t* t = keys;
    keys = tmp;
    tmp = t;
  }
  return keys;
}

// l1 norm and support masks (W words of positive support, then W of negative).
// l1 norm and the positive / negative support bit masks of every key
__global__ __launch_bounds__(kTileRows) void k_prep(const int8_t* keys, int stride, int n, uint32_t count, int W,
                                                    int tile_rows, int32_t* l1, uint64_t* mask) {
  extern __shared__ __align__(16) int8_t ptile[];  // tile_rows x stride
  const uint32_t r0 = blockIdx.x * (uint32_t)tile_rows;
  const int rows = (int)min((uint32_t)tile_rows, count - r0);
  const uint64_t* s64 = reinterpret_cast<const uint64_t*>(keys + (size_t)r0 * stride);
  for (int w = threadIdx.x; w < rows * stride / 8; w += blockDim.x) reinterpret_cast<uint64_t*>(ptile)[w] = s64[w];
  __syncthreads();
  if ((int)threadIdx.x >= rows) return;
  const int8_t* g = ptile + threadIdx.x * stride;
  const uint32_t k = r0 + threadIdx.x;
  int32_t s = 0;
  uint64_t* mk = mask + (size_t)k * 2 * W;
  for (int w = 0; w < W; ++w) {
    uint64_t p = 0, q = 0;
    const int hi = min(64, n - w * 64);
    for (int b = 0; b < hi; ++b) {
      const int v = g[w * 64 + b];
      s += v < 0 ? -v : v;
      p |= (uint64_t)(v > 0) << b;
      q |= (uint64_t)(v < 0) << b;
    }
    mk[w] = p;
    mk[W + w] = q;
  }
  l1[k] = s;
}

// dst row i = src row idx[i] with its l1 and masks (2W <= stride / 8 words)
__global__ void k_gather_rows(const int8_t* src, int stride, const uint32_t* idx, uint32_t count,
                              int8_t* dst, const int32_t* l1src, int32_t* l1dst, const uint64_t* msrc,
                              uint64_t* mdst, int W) {
  const int L = stride / 8;
  const uint64_t total = (uint64_t)count * L;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = t / L;
    const int w = (int)(t - i * L);
    const uint32_t j = idx[i];
    reinterpret_cast<uint64_t*>(dst + (size_t)i * stride)[w] =
        reinterpret_cast<const uint64_t*>(src + (size_t)j * stride)[w];
    if (w == 0) l1dst[i] = l1src[j];
    if (w < 2 * W) mdst[(size_t)i * 2 * W + w] = msrc[(size_t)j * 2 * W + w];
  }
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

// ---- witness search through a sign-pattern index -------------------------
// A witness h of g (h conformally below g, or -h below g) must agree with
// g's sign pattern wherever it is nonzero.  On a chosen set C of k
// coordinates, every key gets the base-3 code of its signs (0 zero, 1
// positive, 2 negative).  The witnesses of g for the relation "h below g"
// can only have codes whose digits are 0 or g's digit, and for "-h below
// g" digits that are 0 or the swapped digit; g enumerates these 2^z codes
// (z = nonzeros of g on C) and tests only the keys of those buckets.  The
// result is the same predicate as testing every pair.
constexpr int kMaxC = 18;
constexpr int kJoinThreads = 64;  // one wave
struct Coords {
  int k;
  int c[kMaxC];
  int pow3[kMaxC];
};

// |x| of four int8 lanes in [-127, 127], as four bytes in [0, 127]:
// one's complement of the negative lanes plus one (no carry between lanes)
__device__ __forceinline__ uint32_t abs8x4(uint32_t x) {
  const uint32_t neg = (x >> 7) & 0x01010101u;
  return (x ^ (neg * 0xFFu)) + neg;
}

// |h_i| <= |g_i| for every byte of two zero-padded rows, 16 bytes per
// step: (|g| | 0x80) - |h| keeps bit 7 of a lane exactly when |g| >= |h|
__device__ __forceinline__ bool magnitude_below(const int8_t* h, const int8_t* g, int stride) {
  const uint4* h4 = reinterpret_cast<const uint4*>(h);
  const uint4* g4 = reinterpret_cast<const uint4*>(g);
  for (int c = 0; c < stride / 16; ++c) {
    const uint4 a = h4[c], b = g4[c];
    const uint32_t keep = ((abs8x4(b.x) | 0x80808080u) - abs8x4(a.x)) & ((abs8x4(b.y) | 0x80808080u) - abs8x4(a.y)) &
                          ((abs8x4(b.z) | 0x80808080u) - abs8x4(a.z)) & ((abs8x4(b.w) | 0x80808080u) - abs8x4(a.w));
    if ((keep & 0x80808080u) != 0x80808080u) return false;
  }
  return true;
}

// nonzero count of every coordinate over the rows r = i * step, i < rows
// (they only rank the coordinates for the index, so an evenly spaced,
// deterministic sample of the keys serves); block = 64 sampled rows,
// thread = column
constexpr uint32_t kNnzSampleRows = 65536;
__global__ void k_col_nnz(const int8_t* keys, int stride, int n, uint32_t rows, uint32_t step, uint32_t* cnt) {
  const uint32_t i0 = blockIdx.x * 64u;
  const uint32_t i1 = min(rows, i0 + 64u);
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    uint32_t local = 0;
    for (uint32_t i = i0; i < i1; ++i) local += keys[(size_t)i * step * stride + c] != 0;
    if (local) atomicAdd(&cnt[c], local);
  }
}

// base-3 sign code of every key on the index coordinates (row tiles in LDS)
__global__ __launch_bounds__(kTileRows) void k_codes(const int8_t* keys, int stride, uint32_t count, Coords C,
                                                     int tile_rows, uint32_t* code, uint32_t* hist) {
  extern __shared__ __align__(16) int8_t dtile[];  // tile_rows x stride
  const uint32_t r0 = blockIdx.x * (uint32_t)tile_rows;
  const int rows = (int)min((uint32_t)tile_rows, count - r0);
  const uint64_t* s64 = reinterpret_cast<const uint64_t*>(keys + (size_t)r0 * stride);
  for (int w = threadIdx.x; w < rows * stride / 8; w += blockDim.x) reinterpret_cast<uint64_t*>(dtile)[w] = s64[w];
  __syncthreads();
  if ((int)threadIdx.x >= rows) return;
  const uint32_t p = r0 + threadIdx.x;
  const int8_t* g = dtile + threadIdx.x * stride;
  uint32_t cd = 0;
  for (int i = 0; i < C.k; ++i) {
    int v = g[C.c[i]];
    cd += (v > 0 ? 1u : (v < 0 ? 2u : 0u)) * (uint32_t)C.pow3[i];
  }
  code[p] = cd;
  atomicAdd(&hist[cd], 1u);
}

// masks in bucket order: bmask row e = mask row bl[e] (a thread per word)
// (and the first word of each half again, as one 16-byte pair per member:
// the join's fast test reads only those)
__global__ void k_bucket_masks(const uint32_t* bl, const uint64_t* mask, uint32_t count, int W, uint64_t* bmask,
                               uint64_t* bfirst) {
  const uint64_t total = (uint64_t)count * 2 * W;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t e = t / (2 * W);
    const int w = (int)(t - e * 2 * W);
    const uint64_t v = mask[(size_t)bl[e] * 2 * W + w];
    bmask[e * 2 * W + w] = v;
    if (w == 0) bfirst[2 * e] = v;
    if (w == W) bfirst[2 * e + 1] = v;
  }
}

// (code << bits_pos) | p: sorting these puts every bucket's members in
// increasing position, i.e. increasing l1
__global__ void k_code_keys(const uint32_t* code, uint32_t count, int bits_pos, uint64_t* keys) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < count) keys[p] = ((uint64_t)code[p] << bits_pos) | p;
}

// Witness search as a tiled join over the sign-pattern index.  A work item
// is a chunk of at most kJoinThreads keys g of one bucket G, one g per lane
// of a one-wave block.  The candidate buckets H (digits 0 or G's digit for
// "h below g", 0 or the swapped digit for "-h below g") are the same for
// every g of the item.  The wave enumerates them in rounds of kListCap codes
// (2 * 2^z codes for z nonzero digits of G), keeps the non-empty ones of a
// round in an LDS list with an exclusive prefix of their sizes, and streams
// the concatenation of their members through LDS in tiles; every member is
// compared against every g of the chunk.  Only existence of a witness
// matters, so the order of the list is free.
constexpr int kListCap = 256;
constexpr int kListPerLane = kListCap / kJoinThreads;
constexpr uint32_t kPolBit = 0x80000000u;

// bit c of bits: bucket c is non-empty (the join tests it before reading
// the bucket's offsets)
__global__ void k_bucket_bits(const uint32_t* hist, uint32_t ncode, uint32_t* bits) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w * 32u >= ncode) return;
  uint32_t v = 0;
  for (uint32_t b = 0; b < 32u && w * 32u + b < ncode; ++b) v |= (hist[w * 32u + b] != 0 ? 1u : 0u) << b;
  bits[w] = v;
}

// Work items of the join: bucket G is cut into ceil(size / kJoinThreads)
// chunks of consecutive members; owner[w] = bucket of chunk w, and the
// chunks of G start at item choff[G].
__global__ void k_chunk_count(const uint32_t* hist, uint32_t ncode, uint32_t* nch) {
  uint32_t G = blockIdx.x * blockDim.x + threadIdx.x;
  if (G > ncode) return;
  nch[G] = G < ncode ? (hist[G] + kJoinThreads - 1) / kJoinThreads : 0u;
}
__global__ void k_chunk_owner(const uint32_t* nch, const uint32_t* choff, uint32_t ncode, uint32_t* owner) {
  uint32_t G = blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= ncode) return;
  for (uint32_t c = 0; c < nch[G]; ++c) owner[choff[G] + c] = G;
}

__global__ __launch_bounds__(kJoinThreads) void k_pairs_join(const int8_t* keys, int stride, int n, int W,
                                                           const uint64_t* __restrict__ mask,
                                                           const uint32_t* __restrict__ lo,
                                                           const uint32_t* __restrict__ off,
                                                           const uint32_t* __restrict__ bl,
                                                           const uint64_t* __restrict__ bmask,
                                                           const ulonglong2* __restrict__ bfirst, Coords C,
                                                           const uint32_t* __restrict__ choff,
                                                           const uint32_t* __restrict__ owner, uint32_t ncode,
                                                           const uint32_t* __restrict__ bits, uint32_t* alive) {
  extern __shared__ uint64_t smem_join[];
  // a tile holds one member per lane (small tiles keep more one-wave blocks
  // resident and let an item stop sooner once its keys are dead: on the
  // quartic headline's keys 32 / 64 / 96 / 128 / 256 / 512 / 1024 members
  // gave 0.94 / 0.92 / 0.92 / 0.97 / 1.08 / 1.45 / 2.12 s for the whole filter)
  constexpr uint32_t tile_n = kJoinThreads;
  ulonglong2* tfirst = reinterpret_cast<ulonglong2*>(smem_join);          // tile_n: first positive / negative words
  uint32_t* tpos = reinterpret_cast<uint32_t*>(tfirst + tile_n);          // tile_n: position
  uint32_t* teb = tpos + tile_n;                                          // tile_n: bucket-order index | polarity
  __shared__ uint32_t lst_b[kListCap];       // bl offset of a non-empty candidate bucket | polarity
  __shared__ uint32_t lst_pre[kListCap + 1];  // sizes, then their exclusive prefix (total at [L])
  // the item's candidate codes: code(j) = tcode[pol][0][j & 63] +
  // tcode[pol][1][(j >> 6) & 63] + tcode[pol][2][j >> 12] for subset j of
  // the item's nonzero digits
  __shared__ uint32_t tcode[2][3][64];
  const uint32_t lane = threadIdx.x;
  const uint32_t nwork = choff[ncode];
  for (uint32_t wk = blockIdx.x; wk < nwork; wk += gridDim.x) {
    const uint32_t G = owner[wk];
    const uint32_t gb = off[G] + (wk - choff[G]) * kJoinThreads;
    const uint32_t ge = min(off[G + 1], gb + kJoinThreads);
    int dg[kMaxC];
    {
      uint32_t rem = G;
#pragma unroll
      for (int i = 0; i < kMaxC; ++i) {
        dg[i] = i < C.k ? (int)(rem % 3u) : 0;
        rem /= 3u;
      }
    }
    int z = 0;
#pragma unroll
    for (int i = 0; i < kMaxC; ++i) z += dg[i] != 0;
    const uint32_t nsub = 1u << z;
    __syncthreads();  // the previous item's code tables are no longer read
    for (uint32_t e = lane; e < 6u * 64u; e += kJoinThreads) {
      const uint32_t pol = e / 192u, part = (e / 64u) % 3u, sub = e & 63u;
      uint32_t code = 0;
      int bit = 0;
#pragma unroll
      for (int i = 0; i < kMaxC; ++i) {
        if (dg[i]) {
          const int b6 = bit - 6 * (int)part;
          if (b6 >= 0 && b6 < 6 && ((sub >> b6) & 1u)) code += (uint32_t)((pol ? 3 - dg[i] : dg[i]) * C.pow3[i]);
          ++bit;
        }
      }
      tcode[pol][part][sub] = code;
    }
    __syncthreads();
    const uint32_t e = gb + lane;
    const bool valid = e < ge;
    const uint32_t p = valid ? bl[e] : 0u;
    const uint32_t my_lo = valid ? lo[p] : 0u;
    // members at positions >= every key's level start cannot be witnesses;
    // bucket lists are in increasing position, so each is cut there
    uint32_t maxlo = my_lo;
    for (int o = 32; o > 0; o >>= 1) maxlo = max(maxlo, (uint32_t)__shfl_xor((int)maxlo, o, 64));
    const uint64_t* gm = mask + (size_t)p * 2 * W;
    const uint64_t ngp0 = ~(valid ? gm[0] : 0ull), ngn0 = ~(valid ? gm[W] : 0ull);
    const bool idle = !valid || my_lo == 0;  // nothing of smaller l1 to test
    const int8_t* g = keys + (size_t)p * stride;
    bool dead = false;
    for (uint32_t j0 = 0; j0 < 2 * nsub; j0 += kListCap) {
      if (__ballot(!idle && !dead) == 0) break;
      __syncthreads();  // the previous round's list and tiles are no longer read
      // non-empty candidate buckets of codes j0 .. j0 + kListCap - 1
      uint32_t L = 0;
      for (int r = 0; r < kListPerLane; ++r) {
        const uint32_t j = j0 + (uint32_t)r * kJoinThreads + lane;
        uint32_t hb = 0, he = 0, pol = 0;
        if (j < 2 * nsub) {
          pol = j >= nsub ? 1u : 0u;
          const uint32_t sidx = j - pol * nsub;
          const uint32_t code = tcode[pol][0][sidx & 63u] + tcode[pol][1][(sidx >> 6) & 63u] + tcode[pol][2][sidx >> 12];
          if ((bits[code >> 5] >> (code & 31u)) & 1u) {
            hb = off[code];
            he = off[code + 1];
            // first member at position >= maxlo
            uint32_t a = hb, b = he;
            while (a < b) {
              const uint32_t mid = (a + b) >> 1;
              if (bl[mid] < maxlo) a = mid + 1; else b = mid;
            }
            he = a;
          }
        }
        const bool keep = he > hb;
        const uint64_t km = __ballot(keep);
        if (keep) {
          const uint32_t slot =
              L + __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
          lst_b[slot] = hb | (pol ? kPolBit : 0u);
          lst_pre[slot] = he - hb;
        }
        L += (uint32_t)__popcll(km);
      }
      if (L == 0) continue;
      __syncthreads();
      // exclusive prefix of the sizes: lane t sums entries [t * kListPerLane, ...)
      uint32_t total;
      {
        const uint32_t a0 = min(L, lane * kListPerLane), a1 = min(L, a0 + kListPerLane);
        uint32_t loc = 0;
        for (uint32_t i = a0; i < a1; ++i) loc += lst_pre[i];
        uint32_t v = loc;
        for (int o = 1; o < kJoinThreads; o <<= 1) {
          const uint32_t t = __shfl_up(v, o, kJoinThreads);
          if ((int)lane >= o) v += t;
        }
        uint32_t run = v - loc;
        for (uint32_t i = a0; i < a1; ++i) {
          const uint32_t sz = lst_pre[i];
          lst_pre[i] = run;
          run += sz;
        }
        total = __shfl(v, kJoinThreads - 1, kJoinThreads);
        if (lane == 0) lst_pre[L] = total;
      }
      __syncthreads();
      // this lane's member of a tile: list entry, then its first mask words
      // (polarity applied: -h below g is tested as h with its sign words
      // swapped), position and bucket-order index; read one tile ahead so
      // the loads are in flight while the current tile is tested
      ulonglong2 nf = make_ulonglong2(~0ull, ~0ull);
      uint32_t npos = 0xFFFFFFFFu, neb = 0;
      auto fetch = [&](uint32_t q) {
        if (q >= total) return;
        uint32_t a = 0, b = L - 1;  // last list entry whose prefix is <= q (prefixes strictly increase)
        while (a < b) {
          const uint32_t mid = (a + b + 1) / 2;
          if (lst_pre[mid] <= q) a = mid; else b = mid - 1;
        }
        const uint32_t hb = lst_b[a];
        const uint32_t eb = (hb & ~kPolBit) + (q - lst_pre[a]);
        const ulonglong2 f = bfirst[eb];
        nf = (hb & kPolBit) ? make_ulonglong2(f.y, f.x) : f;
        npos = bl[eb];
        neb = eb | (hb & kPolBit);
      };
      fetch(lane);
      for (uint32_t t0 = 0; t0 < total; t0 += tile_n) {
        if (__ballot(!idle && !dead) == 0) break;
        const uint32_t cnt = min(tile_n, total - t0);
        __syncthreads();  // the previous tile is no longer read
        if (lane < cnt) {
          tfirst[lane] = nf;
          tpos[lane] = npos;
          teb[lane] = neb;
        }
        // pad the tile to a multiple of 4 members that never match
        for (uint32_t t = cnt + lane; t < ((cnt + 3u) & ~3u); t += kJoinThreads) {
          tpos[t] = 0xFFFFFFFFu;
          tfirst[t] = make_ulonglong2(~0ull, ~0ull);
        }
        __syncthreads();
        fetch(t0 + tile_n + lane);
        if (idle || dead) continue;
        // Fast test on the first 64 coordinates of the sign masks, four
        // members at a time; the other words and the magnitudes are read only
        // for members that pass it (for unrelated dense keys, almost none).
        for (uint32_t t = 0; t < cnt && !dead; t += 4) {
          bool cand[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const ulonglong2 f = tfirst[t + u];
            cand[u] = ((f.x & ngp0) | (f.y & ngn0)) == 0 && tpos[t + u] < my_lo;
          }
          if (__ballot(cand[0] || cand[1] || cand[2] || cand[3]) == 0) continue;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (!cand[u] || dead) continue;
            const uint32_t hv = teb[t + u];
            const bool pol = (hv & kPolBit) != 0;
            const uint64_t* hm = bmask + (size_t)(hv & ~kPolBit) * 2 * W;
            bool ok = true;
            for (int w = 1; w < W && ok; ++w) {
              const uint64_t hp = hm[w], hn = hm[W + w];
              const uint64_t gpw = gm[w], gnw = gm[W + w];
              ok = pol ? ((hp & ~gnw) | (hn & ~gpw)) == 0 : ((hp & ~gpw) | (hn & ~gnw)) == 0;
            }
            if (ok && magnitude_below(keys + (size_t)tpos[t + u] * stride, g, stride)) dead = true;
          }
        }
      }
    }
    if (valid) alive[p] = dead ? 0u : 1u;
  }
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
  // The two key-sized buffers take the slots of the extraction's pool and
  // candidate log (dead once an extraction has returned its keys), so a
  // filter that follows an extraction of the same size allocates nothing
  // for them and the pair fits in device memory together.
  int8_t* canon = (int8_t*)ws_get(ctx, WS_POOL_KEYS, (size_t)cnt * stride, st);
  uint32_t* idx = (uint32_t*)ws_get(ctx, WS_SORT_IDX, (size_t)p2 * 4, st);
  uint32_t* flag = (uint32_t*)ws_get(ctx, WS_FLAGS, (size_t)cnt * 4 + 64, st);
  uint32_t* pos = (uint32_t*)ws_get(ctx, WS_SCAN, (size_t)cnt * 4 + 64, st);
  uint32_t* scr = (uint32_t*)ws_get(ctx, WS_SCAN2, ((size_t)cnt / 512 + 256) * 4, st);
  int8_t* uniq = (int8_t*)ws_get(ctx, WS_LOG, (size_t)cnt * stride, st);
  int32_t* l1 = (int32_t*)ws_get(ctx, WS_F_L1, (size_t)cnt * 8, st);
  uint64_t* msk = (uint64_t*)ws_get(ctx, WS_F_MASK, (size_t)cnt * 4 * W * 8, st);
  uint32_t* lo = (uint32_t*)ws_get(ctx, WS_F_LO, (size_t)cnt * 4, st);
  uint32_t* alive = (uint32_t*)ws_get(ctx, WS_F_ALIVE, (size_t)cnt * 4 + 64, st);
  if (!canon || !idx || !flag || !pos || !scr || !uniq || !l1 || !msk || !lo || !alive)
    return hipSuccess;
  const unsigned b256 = (cnt + 255) / 256;
  const int trows = tile_rows_for(stride);
  hipLaunchKernelGGL(k_canon, dim3((cnt + trows - 1) / trows), dim3(kTileRows), (size_t)trows * stride, s, in,
                     (int64_t)cnt, n, stride, trows, canon);
  HIP_RET(hipGetLastError());
  uint64_t* spk = (uint64_t*)ws_get(ctx, WS_SORT_TMP, (size_t)p2 * 8, st);
  if (!spk) return hipSuccess;
  HIP_RET(launch_sort_keys(s, canon, stride, cnt, idx, spk));
  hipLaunchKernelGGL(k_mark_unique, dim3(b256), dim3(256), 0, s, canon, stride, idx, spk, cnt, flag);
  HIP_RET(hipGetLastError());
  scan_exclusive(s, flag, pos, cnt, scr);
  uint32_t hlast[2] = {0, 0};
  HIP_RET(hipMemcpyAsync(&hlast[0], pos + cnt - 1, 4, hipMemcpyDeviceToHost, s));
  HIP_RET(hipMemcpyAsync(&hlast[1], flag + cnt - 1, 4, hipMemcpyDeviceToHost, s));
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const uint32_t U = hlast[0] + hlast[1];
  if (U == 0) return hipSuccess;
  const uint64_t rw = (uint64_t)stride / 8;
  hipLaunchKernelGGL(k_compact_rows, dim3(stride_grid((uint64_t)cnt * rw)), dim3(256), 0, s, canon, stride, idx,
                     flag, pos, cnt, uniq);
  HIP_RET(hipGetLastError());
  const unsigned u256 = (U + 255) / 256;
  int32_t* l1b = l1 + cnt;
  uint64_t* mskb = msk + (size_t)cnt * 2 * W;
  hipLaunchKernelGGL(k_prep, dim3((U + trows - 1) / trows), dim3(kTileRows), (size_t)trows * stride, s, uniq, stride,
                     n, U, W, trows, l1, msk);
  HIP_RET(hipGetLastError());
  // (l1, lex) order: uniq is lexicographic, so sorting the distinct keys
  // (l1 << bits_pos) | lex position is a stable reorder by l1
  {
    int bits_pos = 1;
    while (bits_pos < 32 && ((uint64_t)1 << bits_pos) < U) ++bits_pos;
    int bits_l1 = 1;
    while (((uint64_t)1 << bits_l1) <= (uint64_t)127 * n) ++bits_l1;
    const uint32_t nblocks = (U + kRadixTile - 1) / kRadixTile;
    uint64_t* rk = (uint64_t*)ws_get(ctx, WS_R_KEYS, (size_t)U * 16, st);
    uint32_t* rh = (uint32_t*)ws_get(ctx, WS_R_HIST, (size_t)nblocks * 16 * 4 * 2 + 64, st);
    if (!rk || !rh) return hipSuccess;
    hipLaunchKernelGGL(k_l1_keys, dim3(u256), dim3(256), 0, s, l1, U, bits_pos, rk);
    HIP_RET(hipGetLastError());
    uint64_t* sorted = radix_sort_u64(s, rk, rk + U, U, bits_l1 + bits_pos, rh, rh + (size_t)nblocks * 16, scr);
    hipLaunchKernelGGL(k_low_bits, dim3(u256), dim3(256), 0, s, sorted, U, bits_pos, idx);
    HIP_RET(hipGetLastError());
  }
  hipLaunchKernelGGL(k_gather_rows, dim3(stride_grid((uint64_t)U * rw)), dim3(256), 0, s, uniq, stride, idx, U,
                     canon, l1, l1b,
                     msk, mskb, W);
  HIP_RET(hipGetLastError());
  hipLaunchKernelGGL(k_level_start, dim3(u256), dim3(256), 0, s, l1b, U, lo);
  HIP_RET(hipGetLastError());
  // sign-pattern index on the k most frequently nonzero coordinates.  A work
  // item enumerates up to 2 * 2^k codes, while the members it tests shrink
  // geometrically with k (for dense keys by about half per coordinate), so
  // k grows with log2 U: about log2(U) / 2 + 3, at most kMaxC (on 9.6e7 dense
  // keys of n = 400, k = 13 / 14 / 15 / 16 / 17 / 18 measured 2.72 / 1.79 /
  // 1.37 / 1.23 / 1.18 / 1.55 s for the whole filter: past 16 the work
  // items, chunks of one bucket, get smaller and each enumerates 2 * 2^k
  // codes, and the code-indexed arrays grow as 3^k; on 1.5e6 keys of
  // n = 100, k = 11 ... 14 all took 5-7 ms).
  Coords C{};
  {
    int k = 0;
    if (U >= 64) {
      int lg = 0;
      while ((1u << (lg + 1)) <= U) ++lg;
      k = (lg + 1) / 2 + 3;
    }
    k = k < kMaxC ? k : kMaxC;
    k = k < n ? k : n;
    std::vector<uint32_t> hc(n, 0);
    if (k > 0) {
      uint32_t* cnt = (uint32_t*)ws_get(ctx, WS_F_CODE, ((size_t)U + n + 64) * 4, st);
      if (!cnt) return hipSuccess;
      hipLaunchKernelGGL(k_zero32, dim3((n + 255) / 256), dim3(256), 0, s, cnt, (uint32_t)n);
      HIP_RET(hipGetLastError());
      const uint32_t step = (U + kNnzSampleRows - 1) / kNnzSampleRows;
      const uint32_t rows = (U + step - 1) / step;
      hipLaunchKernelGGL(k_col_nnz, dim3((rows + 63) / 64), dim3(128), 0, s, canon, stride, n, rows, step, cnt);
      HIP_RET(hipGetLastError());
      HIP_RET(hipMemcpyAsync(hc.data(), cnt, (size_t)n * 4, hipMemcpyDeviceToHost, s));
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hc[a] > hc[b]; });
    C.k = k;
    int pw = 1;
    for (int i = 0; i < k; ++i) {
      C.c[i] = order[i];
      C.pow3[i] = pw;
      pw *= 3;
    }
  }
  uint32_t ncode = 1;
  for (int i = 0; i < C.k; ++i) ncode *= 3;
  uint32_t* code = (uint32_t*)ws_get(ctx, WS_F_CODE, ((size_t)U + n + 64) * 4, st);
  uint32_t* hist = (uint32_t*)ws_get(ctx, WS_F_HIST, ((size_t)ncode + 64) * 4, st);
  uint32_t* boff = (uint32_t*)ws_get(ctx, WS_F_OFF, ((size_t)ncode + 64) * 4, st);
  uint32_t* bl = (uint32_t*)ws_get(ctx, WS_F_BL, (size_t)U * 4 + 64, st);
  uint32_t* scr2 = (uint32_t*)ws_get(ctx, WS_SCAN2, (((size_t)cnt > ncode ? cnt : ncode) / 512 + 256) * 4, st);
  if (!code || !hist || !boff || !bl || !scr2) return hipSuccess;
  const unsigned c256 = (ncode + 1 + 255) / 256;
  hipLaunchKernelGGL(k_zero32, dim3(c256), dim3(256), 0, s, hist, ncode + 1);
  HIP_RET(hipGetLastError());
  hipLaunchKernelGGL(k_codes, dim3((U + trows - 1) / trows), dim3(kTileRows), (size_t)trows * stride, s, canon, stride,
                     U, C, trows, code, hist);
  HIP_RET(hipGetLastError());
  scan_exclusive(s, hist, boff, ncode + 1, scr2);
  {
    // bucket lists in increasing position (stable radix sort by code)
    int bits_pos = 1;
    while (bits_pos < 32 && ((uint64_t)1 << bits_pos) < U) ++bits_pos;
    int bits_code = 1;
    while (((uint64_t)1 << bits_code) < ncode) ++bits_code;
    const uint32_t nblocks = (U + kRadixTile - 1) / kRadixTile;
    uint64_t* rk = (uint64_t*)ws_get(ctx, WS_R_KEYS, (size_t)U * 16, st);
    uint32_t* rh = (uint32_t*)ws_get(ctx, WS_R_HIST, (size_t)nblocks * 16 * 4 * 2 + 64, st);
    if (!rk || !rh) return hipSuccess;
    hipLaunchKernelGGL(k_code_keys, dim3(u256), dim3(256), 0, s, code, U, bits_pos, rk);
    HIP_RET(hipGetLastError());
    uint64_t* sorted = radix_sort_u64(s, rk, rk + U, U, bits_code + bits_pos, rh, rh + (size_t)nblocks * 16, scr2);
    hipLaunchKernelGGL(k_low_bits, dim3(u256), dim3(256), 0, s, sorted, U, bits_pos, bl);
    HIP_RET(hipGetLastError());
  }
  // the masks in bucket order go to the first half of the mask buffer (its
  // lexicographic-order masks are no longer read)
  uint64_t* bmsk = msk;
  uint64_t* bfirst = (uint64_t*)ws_get(ctx, WS_F_FIRST, (size_t)U * 16 + 64, st);
  if (!bfirst) return hipSuccess;
  hipLaunchKernelGGL(k_bucket_masks, dim3(stride_grid((uint64_t)U * 2 * W)), dim3(256), 0, s, bl, mskb, U,
                     W, bmsk, bfirst);
  HIP_RET(hipGetLastError());
  // join work items: chunks of at most kJoinThreads members of one bucket
  const size_t max_items = (size_t)(U < ncode ? U : ncode) + U / kJoinThreads + 1;
  uint32_t* chk = (uint32_t*)ws_get(ctx, WS_F_CHUNK, ((size_t)2 * (ncode + 1) + max_items + 64) * 4, st);
  if (!chk) return hipSuccess;
  uint32_t* nch = chk;
  uint32_t* choff = chk + (ncode + 1);
  uint32_t* owner = chk + 2 * (size_t)(ncode + 1);
  hipLaunchKernelGGL(k_chunk_count, dim3(c256), dim3(256), 0, s, hist, ncode, nch);
  HIP_RET(hipGetLastError());
  scan_exclusive(s, nch, choff, ncode + 1, scr2);
  hipLaunchKernelGGL(k_chunk_owner, dim3((ncode + 255) / 256), dim3(256), 0, s, nch, choff, ncode, owner);
  HIP_RET(hipGetLastError());
  uint32_t* bits = (uint32_t*)ws_get(ctx, WS_F_BITS, ((size_t)ncode / 32 + 64) * 4, st);
  if (!bits) return hipSuccess;
  hipLaunchKernelGGL(k_bucket_bits, dim3((ncode / 32 + 1 + 255) / 256), dim3(256), 0, s, hist, ncode, bits);
  HIP_RET(hipGetLastError());
  // one tile member per lane, 24 bytes each in LDS
  const size_t jshm = (size_t)kJoinThreads * (sizeof(ulonglong2) + 2 * sizeof(uint32_t));
  const unsigned jgrid = (unsigned)(max_items < (1u << 20) ? max_items : (1u << 20));
  hipLaunchKernelGGL(k_pairs_join, dim3(jgrid), dim3(kJoinThreads), jshm, s, canon, stride, n, W, mskb, lo, boff, bl,
                     bmsk, reinterpret_cast<const ulonglong2*>(bfirst), C, choff, owner, ncode, bits, alive);
  HIP_RET(hipGetLastError());
  // survivors back in lexicographic order: flags to lex positions, then compact uniq
  hipLaunchKernelGGL(k_scatter_flags, dim3(u256), dim3(256), 0, s, idx, alive, U, flag);
  HIP_RET(hipGetLastError());
  scan_exclusive(s, flag, pos, U, scr2);  // (scr2: the scan slot as last sized)
  HIP_RET(hipMemcpyAsync(&hlast[0], pos + U - 1, 4, hipMemcpyDeviceToHost, s));
  HIP_RET(hipMemcpyAsync(&hlast[1], flag + U - 1, 4, hipMemcpyDeviceToHost, s));
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const uint32_t R = hlast[0] + hlast[1];
  *count_out = R;
  if ((int64_t)R > cap) {
    *st = set_error(GRAVER_E_CAPACITY, "keys_cap too small for the filtered set");
    return hipSuccess;
  }
  const uint64_t words = (uint64_t)U * ((n + 3) / 4);
  hipLaunchKernelGGL(k_compact_out, dim3(stride_grid(words)), dim3(256), 0, s, uniq, stride, flag, pos,
                     U, n, out);
  HIP_RET(hipGetLastError());
  return hipStreamSynchronize(s);
}

}  // namespace graver
