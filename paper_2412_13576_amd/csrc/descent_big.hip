// Descent of eq. loss with Parallel Extraction (Algorithm 2) on gfx950 matrix
// cores for large bases (n up to 1024, d up to 1024).
//
// A start group is 16 starts.  Its coordinates are split over CS waves of a
// block (column slices of DBPW 16-column blocks each), so the per-wave
// register state stays bounded as d grows; a block is 4 waves (one per
// SIMD), i.e. 4 / CS start groups.  The basis is streamed through LDS one
// 16-row block at a time (double buffered: the next block is loaded from
// HBM/L2 straight into LDS while the current one is used).  z and the gradient
// accumulators stay in registers; Adam's m and v stay in LDS for the whole
// launch where they fit beside the two basis chunks, and are otherwise read
// and written once per iteration in the wave-native layout.  Per row block ib
// each wave computes
//   y_ib   = B_ib z      over its own columns (binary32 MFMA, or the exact
//                        three-part bf16 split of z), summed over the slices
//                        through LDS
//   G     += B_ib^T sign(y_ib)           (exact bf16 operands, fp32 sums)
//   g_ib   = B_ib r      for the previous iterate r = round(z) (exact bf16
//                        operands, integer partial sums, summed over slices)
// so the exact candidate of iterate t is formed during iteration t+1 (and a
// final pass forms the last one).  The infinity norm, its ties, the change
// flag and the exact-range flag of a start are combined over its slices
// once per iteration.  Rounded coordinates beyond |r| <= 256 are not exact
// bf16 operands: such an iterate yields no candidate (counted as out of
// range).  The first slice of a start group stages candidate rows in a
// global scratch row and appends those that pass the box test to the
// candidate log.
//
// The LDS image of a row block holds B as bf16 only (every |B_ij| <= 256 is
// exact in bf16); the binary32 forward widens the operands in registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "graver_internal.h"

namespace graver {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kWaves = 4;
constexpr int kBigLogChunk = 64;

inline int blk16(int x) { return (x + 15) / 16; }

// Shapes with an instantiated kernel, in order of preference: the smallest
// split whose waves hold at most 12 column blocks (wider waves exceed the
// register file); 16 blocks per wave only beyond d = 768.  The 6-block
// shapes run two waves per SIMD: (4, 6) is preferred up to d = 384 (0.81x
// the time of (2, 12) at d = 350); (2, 6) is an autotuner candidate.
constexpr BigShape kShapes[] = {{1, 8}, {1, 12}, {2, 6}, {2, 8}, {4, 6}, {2, 12}, {4, 8}, {4, 12}, {4, 16}};

inline int64_t big_waves(int64_t N) {
  int64_t w = (N + 15) / 16;
  return (w + kWaves - 1) / kWaves * kWaves;
}

__device__ __forceinline__ short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }
__device__ __forceinline__ short sign_bf16(float y) {
  return y > 0.f ? (short)0x3F80 : (y < 0.f ? (short)0xBF80 : (short)0);
}
__device__ __forceinline__ short int_bf16(float v) { return (short)(__float_as_uint(v) >> 16); }  // |v| <= 256, integer

// v_mfma_f32_16x16x32_bf16 contracts over 32 indices, lane group l/16
// supplying the same 8 of them for both operands.  Two 16-column blocks run
// as one instruction: elements 0-3 of a lane carry the indices it holds in
// the first block and elements 4-7 those of the second, in both operands, so
// the sum runs over the union of the two blocks.
__device__ __forceinline__ floatx4 mfma_pair(shortx4 a0, shortx4 a1, shortx4 b0, shortx4 b1, floatx4 c) {
  const shortx8 a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
  const shortx8 b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

__device__ __forceinline__ float xmax4(float x) {
  x = fmaxf(x, __shfl_xor(x, 16, 64));
  return fmaxf(x, __shfl_xor(x, 32, 64));
}
__device__ __forceinline__ float xsum4(float x) {
  x += __shfl_xor(x, 16, 64);
  return x + __shfl_xor(x, 32, 64);
}
__device__ __forceinline__ int xor4(int x) {
  x |= __shfl_xor(x, 16, 64);
  return x | __shfl_xor(x, 32, 64);
}
__device__ __forceinline__ int xand4(int x) {
  x &= __shfl_xor(x, 16, 64);
  return x & __shfl_xor(x, 32, 64);
}

// Per row block ib (16 rows), for DBT column blocks:
//   FB[jb*64 + l] 4 x bf16 (B[16ib + l%16][16jb + 4(l/16) + r])
//   BT[jb*64 + l] 4 x bf16 (B[16ib + 4(l/16) + r][16jb + l%16])
// laid out as [FB | BT], chunk_bytes = DBT * 64 * 16 bytes.
__global__ void k_pack_big(int n, int d, int NB, int DBT, const int64_t* B, unsigned char* img) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int per = DBT * 64;
  if (t >= NB * per) return;
  int ib = t / per, rest = t % per, jb = rest / 64, l = rest % 64;
  unsigned char* chunk = img + (size_t)ib * per * 16;
  short* FB = reinterpret_cast<short*>(chunk);
  short* BT = reinterpret_cast<short*>(chunk + (size_t)per * 8);
  int i = 16 * ib + l % 16;
  for (int r = 0; r < 4; ++r) {
    int j = 16 * jb + 4 * (l / 16) + r;
    int64_t b = (i < n && j < d) ? B[(size_t)i * d + j] : 0;
    FB[(size_t)rest * 4 + r] = (short)(__float_as_uint((float)b) >> 16);
  }
  int j2 = 16 * jb + l % 16;
  for (int r = 0; r < 4; ++r) {
    int i2 = 16 * ib + 4 * (l / 16) + r;
    int64_t b = (i2 < n && j2 < d) ? B[(size_t)i2 * d + j2] : 0;
    BT[(size_t)rest * 4 + r] = (short)(__float_as_uint((float)b) >> 16);
  }
}

// After the NB chunks the image holds one 64-bit mask per row block: bit jb
// is set when the 16 x 16 block (ib, jb) of B has a nonzero entry.  The
// kernel skips the products of zero blocks (they add exact zeros).
__global__ void k_pack_big_masks(int n, int d, int NB, int DBT, const int64_t* B, uint64_t* masks) {
  const int ib = blockIdx.x * blockDim.x + threadIdx.x;
  if (ib >= NB) return;
  uint64_t m = 0;
  for (int i = 16 * ib; i < min(n, 16 * ib + 16); ++i)
    for (int j = 0; j < d && j < 16 * DBT; ++j)
      if (B[(size_t)i * d + j] != 0) m |= 1ull << (j / 16);
  masks[ib] = m;
}

// Row-block chunk (kU4 uint4) from HBM straight into LDS: each wave moves
// its 64-lane runs of 16 bytes with global_load_lds_dwordx4 (no registers
// held).  The caller waits for vmcnt(0) before the barrier that publishes it.
template <int kU4>
__device__ __forceinline__ void dma_chunk(const uint4* src, uint4* dst) {
  const int wbase = threadIdx.x & ~63;
#pragma unroll
  for (int t = 0; t < kU4 / 256; ++t)
    __builtin_amdgcn_global_load_lds(src + threadIdx.x + t * 256,
                                     (__attribute__((address_space(3))) void*)(dst + wbase + t * 256), 16, 0, 0);
}

__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// Global-memory view of a pointer read from the descriptor table.  Such
// pointers are generic, and accesses through them compile to flat
// instructions, which also count against the LDS wait counter: every wait
// for an LDS operand would then wait for the stores in flight as well.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

struct BigArgs {
  DescentArgs a;
  int NB;
  const unsigned char* img;
  float* z;  // wave-native state (z, then m, then v, each `per` floats)
  int64_t per;
  int8_t* scratch;  // one key row per start
  int stride;
  unsigned long long* counters;
};

inline size_t desc_table_bytes(int count) { return ((size_t)count * sizeof(BigArgs) + 255) / 256 * 256; }

// Adam's m and v stay in LDS for the whole launch (instead of streaming
// through HBM every iteration) when they fit beside the double-buffered
// basis chunks: 8 KB per column block of a wave for the four waves of a
// block, with up to 4 KB left for the box widths.
// Shapes that run two waves per SIMD (two blocks per CU): registers within
// 256 per lane and LDS within half the CU's, so Adam's m and v stay in HBM.
// (8 column blocks per wave need more than 256 registers.)
template <int CS, int DBPW>
constexpr int waves_per_simd() { return DBPW == 6 ? 2 : 1; }

template <int CS, int DBPW, bool BF16F>
constexpr bool mv_in_lds() {
  if (waves_per_simd<CS, DBPW>() > 1 || DBPW % 4 != 0) return false;
  const int kb = 2 * CS * DBPW + 8 * DBPW + (CS > 1 ? 8 : 0) + (BF16F && DBPW <= 12 ? 2 * DBPW : 0) + 1;
  return kb <= 156;
}
template <int DBPW>
constexpr size_t mv_lds_bytes() { return (size_t)kWaves * 2 * DBPW * 4 * 64 * sizeof(float); }

__device__ __forceinline__ void zero_rows_big(const LogDev& log, uint32_t first, uint32_t rows, int lane) {
  const int dw = log.stride / 4;
  auto base = gmem(reinterpret_cast<uint32_t*>(log.rows + (size_t)first * log.stride));
  for (uint32_t t = lane; t < rows * (uint32_t)dw; t += 64) base[t] = 0u;
}

// The grid covers the start groups of every instance of the launch: block
// b belongs to the instance i with cum[i] <= b < cum[i + 1].
template <int CS, int DBPW, bool BF16F>
__global__ __launch_bounds__(64 * kWaves, (waves_per_simd<CS, DBPW>())) void k_descent_big(const BigArgs* __restrict__ descs,
                                                                const int64_t* __restrict__ cum, int count) {
  int inst = 0;
  {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cum[mid] <= (int64_t)blockIdx.x) lo = mid;
      else hi = mid - 1;
    }
    inst = lo;
  }
  const BigArgs& g = descs[inst];
  const int64_t bx = (int64_t)blockIdx.x - cum[inst];
  unsigned long long* counters = g.counters;
  const DescentArgs& a = g.a;
  constexpr int DBT = CS * DBPW;                        // column blocks of the image
  constexpr int kChunkU4 = DBT * 64;                    // uint4 per row-block chunk
  constexpr bool kMvLds = mv_in_lds<CS, DBPW, BF16F>();
  extern __shared__ __align__(16) unsigned char smem[];
  uint4* buf0 = reinterpret_cast<uint4*>(smem);
  uint4* buf1 = buf0 + kChunkU4;
  // [chunk 0 | chunk 1 | m, v of the four waves (when in LDS) | box widths]
  float* sMV = reinterpret_cast<float*>(buf1 + kChunkU4);
  int* sLim = reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(sMV) + (kMvLds ? mv_lds_bytes<DBPW>() : 0));
  // slice partial sums (forward, candidate) and the per-iteration exchange
  // With LDS to spare (m and v not in LDS) the partial sums of consecutive
  // row blocks alternate between two slots, so one barrier per row block
  // both publishes them and the next basis chunk; otherwise a second barrier
  // ends their reads before they are rewritten.
  constexpr bool kOneBar = CS > 1 && !kMvLds;
  constexpr int kRedSlots = kOneBar ? 2 : 1;
  __shared__ floatx4 redY[kRedSlots][CS > 1 ? kWaves : 1][64];
  __shared__ floatx4 redG[kRedSlots][CS > 1 ? kWaves : 1][64];
  __shared__ float xmu[kWaves][16], xcnt[kWaves][16];
  __shared__ int xflag[kWaves][16];
  __shared__ int xwave[kWaves];
  // low bf16 parts of z, per lane, in LDS while they fit next to the
  // double-buffered basis chunks (widest shape: in registers)
  constexpr bool kLoLds = BF16F && DBPW <= 12;
  __shared__ shortx4 sLo[kLoLds ? kWaves : 1][kLoLds ? DBPW : 1][64];

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int q = lane >> 4, sl = lane & 15;
  const int cs = wid % CS;       // column slice of this wave
  const int gw0 = wid - cs;      // first wave of this start group
  const bool lead = cs == 0;     // the slice that emits candidates
  const int64_t sgroup = bx * (kWaves / CS) + wid / CS;
  const int64_t w = bx * kWaves + wid;  // = sgroup * CS + cs
  const int64_t sidx = sgroup * 16 + sl;
  const bool svalid = sidx < a.N;
  const int NB = g.NB;
  const int stride = g.stride;
  const int jb0 = cs * DBPW;     // first image column block of this wave
  for (int i = threadIdx.x; i < 16 * NB; i += blockDim.x) sLim[i] = i < a.n ? (int)(a.u[i] - a.l[i]) : 0;

  float z[DBPW][4];
  // per-wave base pointers (uniform) with 32-bit lane offsets
  const size_t wbase = (size_t)w * 4 * DBPW * 64;
  auto Z = gmem(g.z + wbase);
  auto M = gmem(g.z + g.per + wbase);
  auto V = gmem(g.z + 2 * g.per + wbase);
  const int base = lane;
#pragma unroll
  for (int jb = 0; jb < DBPW; ++jb)
#pragma unroll
    for (int r = 0; r < 4; ++r) z[jb][r] = Z[base + (4 * jb + r) * 64];

  const float lam1 = (float)a.lambda1, lam2 = (float)a.lambda2;
  const float b1 = (float)a.beta1, b2 = (float)a.beta2, omb1 = (float)a.one_minus_b1, omb2 = (float)a.one_minus_b2;
  const float eps = (float)a.eps;
  // this wave's m and v in LDS (same element order as the wave-native state)
  float* sM = sMV + (size_t)wid * 2 * DBPW * 4 * 64;
  float* sV = sM + DBPW * 4 * 64;
  if constexpr (kMvLds) {
    // (a rolled loop: the copy holds few registers at a time)
#pragma unroll 1
    for (int t = 0; t < 4 * DBPW; ++t) {
      sM[t * 64 + lane] = M[base + t * 64];
      sV[t * 64 + lane] = V[base + t * 64];
    }
  }
  const uint4* img = reinterpret_cast<const uint4*>(g.img);
  const uint64_t* bmask = reinterpret_cast<const uint64_t*>(g.img + (size_t)NB * kChunkU4 * 16);
  // (binary32 forward only: with the three-part bf16 forward the branches
  // cost more than the skipped products on the headline basis, 2.35 vs
  // 2.25 s)
  constexpr bool kSkipZero = DBPW <= 8 && !BF16F;
  auto srow = gmem(reinterpret_cast<uint32_t*>(g.scratch + (size_t)sidx * stride));
  const int lim_uniform = a.lim_uniform;

  int changed = 0;       // the current iterate's rounding differs from the previous one
  unsigned long long n_emit = 0, n_inbox = 0, n_range = 0;
  uint32_t lbase = 0, lused = 0;
  int lleft = 0;
  bool log_full = false;
  const LogDev& log = a.log;

  const bool collect = a.collect != 0;
  int par = 0;  // buffer of row block 0 in the current pass
  dma_chunk<kChunkU4>(img, buf0);
  wait_vmem();
  for (int k = 0; k <= a.T; ++k) {
    const bool descend = k < a.T;
    // infinity norm and its ties, change and exact-range flags of the
    // current iterate, over this wave's coordinates, then over the slices
    float mu = 0.f;
#pragma unroll
    for (int jb = 0; jb < DBPW; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) mu = fmaxf(mu, fabsf(z[jb][r]));
    mu = xmax4(mu);
    // the tie count matters only while the start's norm is in (0, 1); this
    // wave's part of the norm bounds it from below, so the count is skipped
    // in waves where no start has this part in (0, 1)
    float cnt = 0.f;
    if (__ballot(mu > 0.f && mu < 1.f) != 0) {
#pragma unroll
      for (int jb = 0; jb < DBPW; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) cnt += fabsf(z[jb][r]) == mu ? 1.f : 0.f;
      cnt = xsum4(cnt);
    }
    float rmax = 0.f;
#pragma unroll
    for (int jb = 0; jb < DBPW; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) rmax = fmaxf(rmax, fabsf(rintf(z[jb][r])));
    int inrange = xmax4(rmax) <= 256.f;
    // One barrier per pass exchanges the slices' parts of the norm and the
    // flags, and every wave's "some start of mine changed" flag, so that
    // whether the candidates are formed is block-uniform (the row-block loop
    // below has block barriers, and the final pass exits the loop when no
    // wave of the block needs it).  It also publishes row block 0, staged
    // during the previous pass's last row block (or before the loop).
    if constexpr (CS > 1) {
      if (q == 0) {
        xmu[wid][sl] = mu;
        xcnt[wid][sl] = cnt;
        xflag[wid][sl] = (changed ? 1 : 0) | (inrange ? 2 : 0);
      }
    }
    const int wchg = __ballot(changed && svalid) != 0 ? 1 : 0;
    if (lane == 0) xwave[wid] = wchg;
    __syncthreads();
    if constexpr (CS > 1) {
      float gm = xmu[gw0][sl];
#pragma unroll
      for (int c = 1; c < CS; ++c) gm = fmaxf(gm, xmu[gw0 + c][sl]);
      float gc = 0.f;
      int f_or = 0, f_and = 2;
#pragma unroll
      for (int c = 0; c < CS; ++c) {
        if (xmu[gw0 + c][sl] == gm) gc += xcnt[gw0 + c][sl];
        const int f = xflag[gw0 + c][sl];
        f_or |= f & 1;
        f_and &= f & 2;
      }
      mu = gm;
      cnt = gc;
      changed = f_or;
      inrange = f_and ? 1 : 0;
    }
    int anyw = 0;
#pragma unroll
    for (int w2 = 0; w2 < kWaves; ++w2) anyw |= xwave[w2];
    const bool needg = collect && k > 0 && anyw != 0;
    if (!descend && !needg) break;
    // rounded coordinates of the current iterate as exact bf16 operands
    shortx4 rp[DBPW];
    if (needg) {
#pragma unroll
      for (int jb = 0; jb < DBPW; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) rp[jb][r] = int_bf16(rintf(z[jb][r]));
    }
    // bf16 forward: z = hi + mid + lo exactly, each part the next 8 bits of
    // the binary32 significand (the residues are exact binary32 differences
    // of numbers within a factor of two, and the last has at most 8
    // significant bits); products with the integer entries of B are exact and
    // the sums are binary32
    // (the low part waits in this lane's LDS slots: registers hold z, hi, mid)
    shortx4 hi[BF16F ? DBPW : 1], mid[BF16F ? DBPW : 1], rlo[BF16F && !kLoLds ? DBPW : 1];
    if constexpr (BF16F) {
#pragma unroll
      for (int jb = 0; jb < DBPW; ++jb) {
        shortx4 lo;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const short h = bf16_rne(z[jb][r]);
          const float r1 = z[jb][r] - bf16_to_f(h);
          const short m = bf16_rne(r1);
          hi[jb][r] = h;
          mid[jb][r] = m;
          lo[r] = bf16_rne(r1 - bf16_to_f(m));
        }
        if constexpr (kLoLds)
          sLo[wid][jb][lane] = lo;
        else
          rlo[jb] = lo;
      }
    }
    floatx4 G[DBPW];
#pragma unroll
    for (int jb = 0; jb < DBPW; ++jb) G[jb] = floatx4{0.f, 0.f, 0.f, 0.f};
    int inbox = 1, nonzero = 0;

    for (int ib = 0; ib < NB; ++ib) {
      const int pb = (par + ib) & 1;
      uint4* cur = pb ? buf1 : buf0;
      uint4* nxt = pb ? buf0 : buf1;
      // the other buffer was last read before the previous row block's final
      // barrier: the next row block streams into it during this one, and
      // during the last one row block 0 of the next pass does
      if (ib + 1 < NB || descend) dma_chunk<kChunkU4>(img + (size_t)(ib + 1 < NB ? ib + 1 : 0) * kChunkU4, nxt);
      // this wave's operands of the row block, read from LDS once: B's
      // columns (forward and candidate) and B^T's (backward); the B^T reads
      // complete under the forward products
      // this wave's nonzero column blocks of the row block (uniform; the
      // 12- and 16-block tiles run every block: the conditional products
      // would cost them registers they do not have).  The quartic headline's
      // basis has 234 nonzero blocks of 550 (binary32 descent 3.07 -> 2.76 s).
      const uint32_t wm = kSkipZero ? __builtin_amdgcn_readfirstlane((uint32_t)(bmask[ib] >> jb0) & ((1u << DBPW) - 1u))
                                    : ((1u << DBPW) - 1u);
      const shortx4* FB = reinterpret_cast<const shortx4*>(cur) + jb0 * 64;
      const shortx4* BT = reinterpret_cast<const shortx4*>(cur) + (DBT + jb0) * 64;
      shortx4 fb[DBPW], bt[DBPW];
#pragma unroll
      for (int jb = 0; jb < DBPW; ++jb) fb[jb] = FB[jb * 64 + lane];
#pragma unroll
      for (int jb = 0; jb < DBPW; ++jb) bt[jb] = BT[jb * 64 + lane];
      floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
      floatx4 gx = floatx4{0.f, 0.f, 0.f, 0.f};
      if (descend) {
        // independent accumulators shorten the dependent MFMA chains
        if constexpr (BF16F) {
          // column blocks in pairs through the 32-deep instruction, one
          // accumulator per part
          floatx4 a1 = floatx4{0.f, 0.f, 0.f, 0.f}, a2 = a1;
#pragma unroll
          for (int jb = 0; jb < DBPW; jb += 2) {
            if (!((wm >> jb) & 3u)) continue;
            acc = mfma_pair(fb[jb], fb[jb + 1], hi[jb], hi[jb + 1], acc);
            a1 = mfma_pair(fb[jb], fb[jb + 1], mid[jb], mid[jb + 1], a1);
            if constexpr (kLoLds)
              a2 = mfma_pair(fb[jb], fb[jb + 1], sLo[wid][jb][lane], sLo[wid][jb + 1][lane], a2);
            else
              a2 = mfma_pair(fb[jb], fb[jb + 1], rlo[jb], rlo[jb + 1], a2);
          }
          acc += a1 + a2;
        } else {
          floatx4 a4[4] = {acc, acc, acc, acc};
#pragma unroll
          for (int jb = 0; jb < DBPW; ++jb) {
            if (!((wm >> jb) & 1u)) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
              a4[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf16_to_f(fb[jb][r]), z[jb][r], a4[r], 0, 0, 0);
          }
          acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        }
      }
      if (needg) {
        // two chains; the partial sums are integers below 2^24, so their
        // sum is exact in any order
        floatx4 g1 = gx;
#pragma unroll
        for (int jb = 0; jb < DBPW; jb += 4) {
          if ((wm >> jb) & 3u) gx = mfma_pair(fb[jb], fb[jb + 1], rp[jb], rp[jb + 1], gx);
          if (jb + 2 < DBPW && ((wm >> (jb + 2)) & 3u))
            g1 = mfma_pair(fb[jb + 2], fb[jb + 3], rp[jb + 2], rp[jb + 3], g1);
        }
        gx += g1;
      }
      const int rs = kOneBar ? (ib & 1) : 0;
      if constexpr (CS > 1) {
        if (descend) redY[rs][wid][lane] = acc;
        if (needg) redG[rs][wid][lane] = gx;
        if constexpr (kOneBar) {
          // publishes the partial sums and the next row block (every read of
          // this row block's chunk ended: its operands are in registers)
          wait_vmem();
        }
        __syncthreads();
        // sum the slices' partial products in slice order (the same order in
        // every wave of the group, so all of them hold the same y and g)
        if (descend) {
          acc = redY[rs][gw0][lane];
#pragma unroll
          for (int c = 1; c < CS; ++c) acc += redY[rs][gw0 + c][lane];
        }
        if (needg) {
          gx = redG[rs][gw0][lane];
#pragma unroll
          for (int c = 1; c < CS; ++c) gx += redG[rs][gw0 + c][lane];
        }
      }
      {
        // (also in the final pass, where y = 0 leaves G unchanged: the
        // accumulators then stay in the matrix-core registers across the loop)
        shortx4 sg;
#pragma unroll
        for (int r = 0; r < 4; ++r) sg[r] = sign_bf16(acc[r]);
#pragma unroll
        for (int jb = 0; jb < DBPW; ++jb)
          if ((wm >> jb) & 1u) G[jb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bt[jb], sg, G[jb], 0, 0, 0);
      }
      uint32_t wd = 0;
      if (needg) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gv = (int)gx[r];
          const int lim = lim_uniform >= 0 ? lim_uniform : sLim[16 * ib + 4 * q + r];
          inbox &= (gv <= lim) & (gv >= -lim);
          nonzero |= gv != 0;
          wd |= ((uint32_t)(uint8_t)(int8_t)gv) << (8 * r);
        }
      }
      if constexpr (!kOneBar) {
        // publishes the next row block, and (CS > 1) ends the reads of the
        // partial sums before they are rewritten
        wait_vmem();
        __syncthreads();
      }
      // (stored after the wait: the next row block's wait for its loads then
      // finds the store long completed)
      if (needg && svalid && lead) srow[4 * ib + q] = wd;
    }
    par = (par + NB) & 1;

    __builtin_amdgcn_sched_barrier(0);
    if (needg) {
      inbox = xand4(inbox);
      nonzero = xor4(nonzero);
      const bool em = changed && svalid;
      const bool emit = em && inrange;
      const bool put = lead && emit && inbox && nonzero;
      n_emit += (lead && q == 0 && emit) ? 1 : 0;
      n_inbox += (q == 0 && put) ? 1 : 0;
      const uint64_t pm = __ballot(put && q == 0);
      if (pm != 0) {
        const int npu = __popcll(pm);
        if (npu > lleft && !log_full) {
          if (lleft > 0) {
            zero_rows_big(log, lbase + lused, (uint32_t)lleft, lane);
            lleft = 0;
          }
          uint32_t nb = 0;
          if (lane == 0) nb = atomicAdd(log.count, (uint32_t)kBigLogChunk);
          nb = __builtin_amdgcn_readfirstlane(nb);
          if (nb < log.cap) {
            const uint32_t end = min(log.cap, nb + (uint32_t)kBigLogChunk);
            lbase = nb;
            lused = 0;
            lleft = (int)(end - nb);
          }
        }
        if (npu > lleft) {
          if (!log_full && lane == 0) atomicOr(log.count + 1, 1u);
          log_full = true;
        } else {
          const uint32_t rank = (uint32_t)__popcll(pm & ((1ull << sl) - 1ull));
          if (put) {
            // the four lanes of the start copy the staged row in 16-byte
            // pieces, four loads issued before their stores (one round trip
            // per 256 bytes of row); the staging stores of every lane of the
            // wave have completed first
            wait_vmem();
            auto row4 = gmem(reinterpret_cast<u32x4*>(log.rows + (size_t)(lbase + lused + rank) * stride));
            auto src4 = gmem(reinterpret_cast<u32x4*>(g.scratch + (size_t)sidx * stride));
            const int nc = stride / 16;
            for (int c0 = 0; c0 < nc; c0 += 16) {
              u32x4 t[4];
#pragma unroll
              for (int u = 0; u < 4; ++u)
                if (c0 + 4 * u + q < nc) t[u] = src4[c0 + 4 * u + q];
#pragma unroll
              for (int u = 0; u < 4; ++u)
                if (c0 + 4 * u + q < nc) row4[c0 + 4 * u + q] = t[u];
            }
          }
          lused += (uint32_t)npu;
          lleft -= npu;
        }
      }
    }
    // an iterate beyond the exact range yields no candidate; the next one
    // is formed from its own r again (B r is recomputed every iteration)
    if (needg && changed && svalid && !inrange && lead && q == 0) ++n_range;
    if (!descend) break;

    __builtin_amdgcn_sched_barrier(0);
    // barrier term, Adam, and the change flag of the new iterate
    const bool bar = mu > 0.f && mu < 1.f;
    const float wbar = bar ? lam2 / ((mu * mu) * cnt) : 0.f;
    const double bc1 = a.bc[2 * k], bc2 = a.bc[2 * k + 1];
    const float step = (float)(a.lr / bc1), ib2 = (float)(1.0 / bc2);
    int ch = 0;
    if constexpr (kMvLds) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int g0 = 0; g0 < DBPW; g0 += 4) {
        // one group of 4 column blocks: load its m and v, update, store
        float mm[4][4], vv[4][4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (4 * (g0 + jj) + r) * 64 + lane;
            mm[jj][r] = sM[e];
            vv[jj][r] = sV[e];
          }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int jb = g0 + jj;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (4 * jb + r) * 64 + lane;
            const float zj = z[jb][r];
            float gg = G[jb][r] + lam1 * ((ceilf(zj) + floorf(zj)) - 2.f * zj);
            if (bar && fabsf(zj) == mu) gg -= zj > 0.f ? wbar : -wbar;
            const float mj = b1 * mm[jj][r] + omb1 * gg;
            const float vj = b2 * vv[jj][r] + omb2 * (gg * gg);
            const float zn = zj - (step * mj) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vj * ib2) + eps);
            ch |= (rintf(zn) != rintf(zj)) | (k == 0);
            z[jb][r] = zn;
            sM[e] = mj;
            sV[e] = vj;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      changed = xor4(ch);
      continue;
    }
    // Opaque per-iteration copies of the base pointers: stops the compiler
    // from hoisting every element address out of the loop (each 64-bit
    // address would stay live in two VGPRs).
    auto Mi = M;
    auto Vi = V;
    asm volatile("" : "+v"(Mi), "+v"(Vi));
    // m and v stream through registers in groups of GW column blocks; the
    // next group's loads are issued before the current group is computed
    // (two register stages), and scheduling barriers keep the compiler from
    // hoisting every load of the iteration at once.
    constexpr int GW = DBPW % 4 == 0 ? 4 : 2;
    constexpr int NG = DBPW / GW;
    float mv[2][GW][4][2];
#pragma unroll
    for (int jb = 0; jb < GW; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = base + (4 * jb + r) * 64;
        mv[0][jb][r][0] = Mi[e];
        mv[0][jb][r][1] = Vi[e];
      }
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int cur = gi & 1, nx = cur ^ 1;
      if (gi + 1 < NG) {
#pragma unroll
        for (int jj = 0; jj < GW; ++jj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = base + (4 * (GW * (gi + 1) + jj) + r) * 64;
            mv[nx][jj][r][0] = Mi[e];
            mv[nx][jj][r][1] = Vi[e];
          }
      }
#pragma unroll
      for (int jj = 0; jj < GW; ++jj) {
        const int jb = GW * gi + jj;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float zj = z[jb][r];
          float gg = G[jb][r] + lam1 * ((ceilf(zj) + floorf(zj)) - 2.f * zj);
          if (bar && fabsf(zj) == mu) gg -= zj > 0.f ? wbar : -wbar;
          const float mj = b1 * mv[cur][jj][r][0] + omb1 * gg;
          const float vj = b2 * mv[cur][jj][r][1] + omb2 * (gg * gg);
          const float zn = zj - (step * mj) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vj * ib2) + eps);
          ch |= (rintf(zn) != rintf(zj)) | (k == 0);
          z[jb][r] = zn;
          const int e = base + (4 * jb + r) * 64;
          Mi[e] = mj;
          Vi[e] = vj;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    changed = xor4(ch);
  }
#pragma unroll
  for (int jb = 0; jb < DBPW; ++jb)
#pragma unroll
    for (int r = 0; r < 4; ++r) Z[base + (4 * jb + r) * 64] = z[jb][r];
  if constexpr (kMvLds) {
#pragma unroll 1
    for (int t = 0; t < 4 * DBPW; ++t) {
      M[base + t * 64] = sM[t * 64 + lane];
      V[base + t * 64] = sV[t * 64 + lane];
    }
  }
  if (lleft > 0) zero_rows_big(log, lbase + lused, (uint32_t)lleft, lane);
  for (int o = 32; o > 0; o >>= 1) {
    n_emit += __shfl_xor(n_emit, o, 64);
    n_inbox += __shfl_xor(n_inbox, o, 64);
    n_range += __shfl_xor(n_range, o, 64);
  }
  if (lane == 0) {
    if (n_emit) atomicAdd(&counters[C_EMIT], n_emit);
    if (n_inbox) atomicAdd(&counters[C_INBOX], n_inbox);
    if (n_range) atomicAdd(&counters[C_RANGE], n_range);
  }
}

template <int CS, int DBPW, bool BF16F>
hipError_t launch_big_t(hipStream_t s, const void* dev_desc, int count, int64_t total_blocks, int max_nb) {
  const size_t shmem = (size_t)2 * CS * DBPW * 64 * 16 + (mv_in_lds<CS, DBPW, BF16F>() ? mv_lds_bytes<DBPW>() : 0) +
                       (size_t)16 * max_nb * sizeof(int);
  auto kern = k_descent_big<CS, DBPW, BF16F>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  const BigArgs* descs = static_cast<const BigArgs*>(dev_desc);
  const int64_t* cum = reinterpret_cast<const int64_t*>(static_cast<const unsigned char*>(dev_desc) +
                                                         desc_table_bytes(count));
  hipLaunchKernelGGL(kern, dim3((unsigned)total_blocks), dim3(64 * kWaves), shmem, s, descs, cum, count);
  return hipGetLastError();
}

template <bool BF16F>
hipError_t launch_big_shape(hipStream_t s, BigShape sh, const void* dev_desc, int count, int64_t total_blocks,
                            int max_nb) {
  switch (sh.cs * 100 + sh.dbpw) {
    case 108: return launch_big_t<1, 8, BF16F>(s, dev_desc, count, total_blocks, max_nb);
    case 112: return launch_big_t<1, 12, BF16F>(s, dev_desc, count, total_blocks, max_nb);
    case 208: return launch_big_t<2, 8, BF16F>(s, dev_desc, count, total_blocks, max_nb);
    case 212: return launch_big_t<2, 12, BF16F>(s, dev_desc, count, total_blocks, max_nb);
    case 406: return launch_big_t<4, 6, BF16F>(s, dev_desc, count, total_blocks, max_nb);
    case 206: return launch_big_t<2, 6, BF16F>(s, dev_desc, count, total_blocks, max_nb);
    case 408: return launch_big_t<4, 8, BF16F>(s, dev_desc, count, total_blocks, max_nb);
    case 412: return launch_big_t<4, 12, BF16F>(s, dev_desc, count, total_blocks, max_nb);
    case 416: return launch_big_t<4, 16, BF16F>(s, dev_desc, count, total_blocks, max_nb);
  }
  return hipErrorInvalidValue;
}

}  // namespace

BigShape big_shape_default(int d) {
  const int db = blk16(d);
  for (const BigShape& sh : kShapes)
    if (sh.cs * sh.dbpw >= db) return sh;
  return BigShape{};
}

bool big_shape_fits(BigShape sh, int d) {
  for (const BigShape& k : kShapes)
    if (k.cs == sh.cs && k.dbpw == sh.dbpw) return sh.cs * sh.dbpw >= blk16(d);
  return false;
}

// Instantiated shapes that hold d with at most twice the needed column
// blocks (the autotuner's choices), in order of preference.
int big_shape_candidates(int d, BigShape* out, int cap) {
  const int db = blk16(d);
  int k = 0;
  for (const BigShape& sh : kShapes)
    if (sh.cs * sh.dbpw >= db && sh.cs * sh.dbpw <= 2 * db + 8 && k < cap) out[k++] = sh;
  return k;
}

bool descent_big_supported(int n, int d) { return n <= 1024 && d <= n && big_shape_default(d).cs > 0; }
size_t big_image_bytes(int n, BigShape sh) {
  return (size_t)blk16(n) * sh.cs * sh.dbpw * 64 * 16 + (size_t)blk16(n) * sizeof(uint64_t);
}
size_t big_state_floats(BigShape sh, int64_t N) { return 3 * (size_t)big_waves(N) * 4 * sh.cs * sh.dbpw * 64; }

hipError_t launch_big_pack(hipStream_t s, int n, int d, BigShape sh, const int64_t* B, unsigned char* img) {
  int NB = blk16(n), DBT = sh.cs * sh.dbpw;
  int total = NB * DBT * 64;
  hipLaunchKernelGGL(k_pack_big, dim3((total + 255) / 256), dim3(256), 0, s, n, d, NB, DBT, B, img);
  hipLaunchKernelGGL(k_pack_big_masks, dim3((NB + 63) / 64), dim3(64), 0, s, n, d, NB, DBT, B,
                     reinterpret_cast<uint64_t*>(img + (size_t)NB * DBT * 64 * 16));
  return hipGetLastError();
}

size_t big_desc_prepare(BigShape sh, const BigJob* jobs, int count, std::vector<unsigned char>& host,
                        int64_t* total_blocks, int* max_nb) {
  const size_t tb = desc_table_bytes(count);
  host.assign(tb + (size_t)(count + 1) * sizeof(int64_t), 0);
  BigArgs* descs = reinterpret_cast<BigArgs*>(host.data());
  int64_t* cum = reinterpret_cast<int64_t*>(host.data() + tb);
  const int DBT = sh.cs * sh.dbpw;
  int64_t blocks = 0;
  int nbmax = 1;
  for (int i = 0; i < count; ++i) {
    const BigJob& j = jobs[i];
    BigArgs g{};
    g.a = j.a;
    g.NB = blk16(j.a.n);
    g.img = j.img;
    g.z = j.state;
    // the state layout is that of DBT column blocks per start group
    g.per = big_waves(j.a.N) * 4 * DBT * 64;
    g.scratch = j.scratch;
    g.stride = key_stride(j.a.n);
    g.counters = j.counters;
    descs[i] = g;
    cum[i] = blocks;
    const int64_t groups = ((int64_t)j.a.N + 15) / 16;
    blocks += (groups + kWaves / sh.cs - 1) / (kWaves / sh.cs);
    nbmax = std::max(nbmax, g.NB);
  }
  cum[count] = blocks;
  *total_blocks = blocks;
  *max_nb = nbmax;
  return host.size();
}

hipError_t launch_descent_big(hipStream_t s, BigShape sh, bool bf16_forward, const void* dev_desc, int count,
                              int64_t total_blocks, int max_nb) {
  if (count < 1 || total_blocks < 1) return hipSuccess;
  return bf16_forward ? launch_big_shape<true>(s, sh, dev_desc, count, total_blocks, max_nb)
                      : launch_big_shape<false>(s, sh, dev_desc, count, total_blocks, max_nb);
}

}  // namespace graver
