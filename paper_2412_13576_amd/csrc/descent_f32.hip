// Binary32 descent of eq. loss with Parallel Extraction (Algorithm 2) on
// gfx950 matrix cores.
//
// One wave owns 16 starts for the whole call; their z, m, v stay in
// registers.  Both contractions run on matrix cores in transposed form so
// that no data moves between them:
//   forward   Y^T (n x 16) = B   (n x d) * Z^T (d x 16)
//   backward  G^T (d x 16) = B^T (d x n) * sign(Y)^T (n x 16)
// In a 16x16x4 MFMA, lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// receives D[4*(l/16)+r][l%16], r = 0..3.  With the K index of the r-th
// MFMA of a 16-block mapped to rows 4k+r, the forward result held by lane l
// (rows 4*(l/16)+r of start l%16) is exactly the backward B operand it
// must supply, and the backward result has the layout of z.  The A
// operands (entries of B) come from LDS, pre-packed per 16x16 block.
//
// Backward: sign(y) is in {-1, 0, 1} and the entries of B are small
// integers (|B_ij| <= 256, checked by the host), so bf16 operands are exact
// and the fp32 sums are exact integers: v_mfma_f32_16x16x16_bf16 gives the
// same result as binary32 arithmetic.  Its 4-value K group per lane is one
// 16-row block, so the forward accumulator of block ib is the operand.
// Forward: binary32 (v_mfma_f32_16x16x4_f32) in FP32 mode; in BF16 mode
// z = hi + lo with hi = bf16(z), lo = bf16(z - hi) and B z = B hi + B lo on
// v_mfma_f32_16x16x16_bf16 (products exact, fp32 accumulation), except the
// last polish iterations, which use the binary32 forward.
//
// After the Adam step every coordinate is rounded (ties to even).  The
// exact candidate g = B r of every start is tracked incrementally:
// g += B (r - r_prev) runs on the same MFMA only for the 4-column groups in
// which some start's rounded coordinate moved; every partial sum is an
// integer of at most 2^24 as long as |r_j| <= floor(2^24 / max_i sum_j |B_ij|),
// so binary32 accumulation is exact.  An iterate outside that range yields
// no candidate (counted as out of range); g is formed from zero again at
// the first iterate back inside it.  When a start's r
// changed and g is nonzero and inside [l - u, u - l], its int8 key is
// assembled in LDS and appended to the candidate log (each wave reserves
// 64-row chunks with one atomic); a separate kernel moves the log into the
// device pool, which removes duplicates.
#include <hip/hip_runtime.h>

#include "graver_internal.h"
#include "pool_device.h"

namespace graver {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWavesPerBlock = 4;
constexpr int kMaxBlk = 8;  // n, d <= 128

bool descent_f32_supported(int n, int d) { return n <= 16 * kMaxBlk && d <= 16 * kMaxBlk && d <= n; }

static inline int blk(int x) { return (x + 15) / 16; }

// FA (float4 per lane and block) followed by FB (4 bf16 per lane and block).
size_t f32_pack_floats(int n, int d) { return (size_t)blk(n) * blk(d) * 64 * 6; }

static inline int64_t n_waves(int64_t N) {
  int64_t w = (N + 15) / 16;
  return (w + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock;
}

size_t f32_state_floats(int n, int d, int64_t N) {
  (void)n;
  return 3 * (size_t)n_waves(N) * 4 * blk(d) * 64;
}

// FA[(ib*DB + jb)*64 + l] = (B[16ib + l%16][16jb + 4(l/16) + r], r = 0..3)      float
// FB[(ib*DB + jb)*64 + l] = the same four entries                              bf16
// BT[(jb*NBP + ip)*64 + l] = (B[32ip + 4(l/16) + r][16jb + l%16], r = 0..3,
//                             then B[32ip + 16 + 4(l/16) + r][16jb + l%16])    8 x bf16
// (NBP = ceil(NB / 2) pairs of row blocks, rows past n zero).  The backward
// runs v_mfma_f32_16x16x32_bf16, whose lane group l/16 supplies 8 of the 32
// contraction indices for both operands: elements 0-3 of a lane carry the
// rows it holds in the first row block of the pair and elements 4-7 those of
// the second, in both operands, so one instruction sums over both blocks.
__device__ __forceinline__ short bf16_bits_exact_int(int64_t v) {
  // v is an integer with |v| <= 256: exactly representable in bf16
  float f = (float)v;
  return (short)(__float_as_uint(f) >> 16);
}

__global__ void k_pack(int n, int d, int NB, int DB, const int64_t* B, float* FA, short* FB, short* BT) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int total = NB * DB * 64;
  if (t >= total) return;
  int l = t % 64, blkid = t / 64;
  {
    int ib = blkid / DB, jb = blkid % DB;
    int i = 16 * ib + l % 16;
    for (int r = 0; r < 4; ++r) {
      int j = 16 * jb + 4 * (l / 16) + r;
      int64_t b = (i < n && j < d) ? B[(size_t)i * d + j] : 0;
      FA[(size_t)t * 4 + r] = (float)b;
      FB[(size_t)t * 4 + r] = bf16_bits_exact_int(b);
    }
  }
  const int NBP = (NB + 1) / 2;
  if (t < DB * NBP * 64) {
    int jb = blkid / NBP, ip = blkid % NBP;
    int j = 16 * jb + l % 16;
    for (int h = 0; h < 2; ++h)
      for (int r = 0; r < 4; ++r) {
        int i = 32 * ip + 16 * h + 4 * (l / 16) + r;
        int64_t b = (i < n && j < d) ? B[(size_t)i * d + j] : 0;
        BT[(size_t)t * 8 + 4 * h + r] = bf16_bits_exact_int(b);
      }
  }
}

// out[0] = max_i sum_j |B_ij|, out[1] = max |B_ij| (both clamped to 2^30)
__global__ void k_rowl1(int n, int d, const int64_t* B, int* out) {
  __shared__ int sh[256], sm[256];
  int best = 0, bmax = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int64_t s = 0;
    for (int j = 0; j < d; ++j) {
      int64_t b = B[(size_t)i * d + j];
      b = b < 0 ? -b : b;
      s += b;
      bmax = max(bmax, (int)min<int64_t>(b, 1 << 30));
    }
    best = max(best, (int)min<int64_t>(s, 1 << 30));
  }
  sh[threadIdx.x] = best;
  sm[threadIdx.x] = bmax;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + o]);
      sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sh[0];
    out[1] = sm[0];
  }
}

hipError_t launch_rowl1(hipStream_t s, int n, int d, const int64_t* B, int* rowl1) {
  hipLaunchKernelGGL(k_rowl1, dim3(1), dim3(256), 0, s, n, d, B, rowl1);
  return hipGetLastError();
}

hipError_t launch_f32_pack(hipStream_t s, int n, int d, const int64_t* B, float* Bp, float* BTp, int* rowl1) {
  int NB = blk(n), DB = blk(d);
  int total = NB * DB * 64;
  short* FB = reinterpret_cast<short*>(Bp + (size_t)total * 4);
  hipLaunchKernelGGL(k_pack, dim3((total + 255) / 256), dim3(256), 0, s, n, d, NB, DB, B, Bp, FB,
                     reinterpret_cast<short*>(BTp));
  hipLaunchKernelGGL(k_rowl1, dim3(1), dim3(256), 0, s, n, d, B, rowl1);
  return hipGetLastError();
}

// Conversion between N x d binary64 arrays and the wave-native layout:
// element (s, j) lives at ((w*4DB + 4*jb + r) * 64 + 16*q + s%16) with
// w = s/16, jb = j/16, q = (j%16)/4, r = j%4.
__global__ void k_state_io(int d, int DB, int64_t N, int64_t nw, float* state, double* z, double* m,
                           double* v, int to_device) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t per = nw * 4 * DB * 64;
  if (t >= per) return;
  int l = (int)(t % 64);
  int64_t rest = t / 64;
  int rho = (int)(rest % (4 * DB));
  int64_t w = rest / (4 * DB);
  int jb = rho / 4, r = rho % 4;
  int64_t s = w * 16 + (l % 16);
  int j = 16 * jb + 4 * (l / 16) + r;
  bool valid = s < N && j < d;
  size_t e = (size_t)s * d + j;
  if (to_device) {
    state[t] = valid ? (float)z[e] : 0.f;
    state[per + t] = valid && m ? (float)m[e] : 0.f;
    state[2 * per + t] = valid && v ? (float)v[e] : 0.f;
  } else if (valid) {
    z[e] = (double)state[t];
    if (m) m[e] = (double)state[per + t];
    if (v) v[e] = (double)state[2 * per + t];
  }
}

hipError_t launch_f32_state_io(hipStream_t s, int n, int d, int64_t N, float* state, double* z, double* m,
                               double* v, int to_device) {
  return launch_state_io_db(s, d, blk(d), N, state, z, m, v, to_device);
}

hipError_t launch_state_io_db(hipStream_t s, int d, int DB, int64_t N, float* state, double* z, double* m,
                              double* v, int to_device) {
  int64_t nw = n_waves(N);
  int64_t per = nw * 4 * DB * 64;
  hipLaunchKernelGGL(k_state_io, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, s, d, DB, N, nw, state, z,
                     m, v, to_device);
  return hipGetLastError();
}

__device__ __forceinline__ float sgnf(float y) { return y > 0.f ? 1.f : (y < 0.f ? -1.f : 0.f); }

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

__device__ __forceinline__ short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }
__device__ __forceinline__ short sign_bf16(float y) {
  return y > 0.f ? (short)0x3F80 : (y < 0.f ? (short)0xBF80 : (short)0);
}

constexpr int kLogChunk = 64;

// Zero `rows` consecutive log rows starting at `first` with the 64 lanes.
__device__ __forceinline__ void zero_rows(const LogDev& log, uint32_t first, uint32_t rows, int lane) {
  const int dw = log.stride / 4;
  uint32_t* base = reinterpret_cast<uint32_t*>(log.rows + (size_t)first * log.stride);
  for (uint32_t t = lane; t < rows * (uint32_t)dw; t += 64) base[t] = 0u;
}

template <int NB, int DB>
__global__ __launch_bounds__(64 * kWavesPerBlock, 1) void k_descent_f32(DescentArgs a, const floatx4* __restrict__ FA,
                                                                         const shortx4* __restrict__ FB,
                                                                         const shortx8* __restrict__ BT,
                                                                         float* __restrict__ state, PoolDev pool,
                                                                         unsigned long long* counters,
                                                                         float zrange, int64_t per,
                                                                         int lim_uniform, LogDev log,
                                                                         const float2* __restrict__ stepf) {
  extern __shared__ __align__(16) unsigned char smem[];
  floatx4* sFA = reinterpret_cast<floatx4*>(smem);
  constexpr int NBP = (NB + 1) / 2;
  shortx4* sFB = reinterpret_cast<shortx4*>(sFA + NB * DB * 64);
  shortx8* sBT = reinterpret_cast<shortx8*>(sFB + NB * DB * 64);
  int* sLim = reinterpret_cast<int*>(sBT + NBP * DB * 64);
  const int stride = pool.stride;

  for (int t = threadIdx.x; t < NB * DB * 64; t += blockDim.x) {
    sFA[t] = FA[t];
    sFB[t] = FB[t];
  }
  for (int t = threadIdx.x; t < NBP * DB * 64; t += blockDim.x) sBT[t] = BT[t];
  for (int i = threadIdx.x; i < 16 * NB; i += blockDim.x)
    sLim[i] = i < a.n ? (int)(a.u[i] - a.l[i]) : 0;
  __syncthreads();

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int q = lane >> 4, sl = lane & 15;
  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  const int64_t sidx = w * 16 + sl;
  const bool svalid = sidx < a.N;

  float z[DB][4], m[DB][4], v[DB][4], rp[DB][4];
  int gi[NB][4];
  const size_t base = (size_t)w * 4 * DB * 64 + lane;
#pragma unroll
  for (int jb = 0; jb < DB; ++jb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      size_t e = base + (size_t)(4 * jb + r) * 64;
      z[jb][r] = state[e];
      m[jb][r] = state[per + e];
      v[jb][r] = state[2 * per + e];
      rp[jb][r] = 0.f;
    }
#pragma unroll
  for (int ib = 0; ib < NB; ++ib)
#pragma unroll
    for (int r = 0; r < 4; ++r) gi[ib][r] = 0;

  bool exact = true;  // gi = B rp holds (it is not maintained while the iterate is out of range)
  unsigned long long n_emit = 0, n_inbox = 0, n_range = 0;
  uint32_t lbase = 0, lused = 0;
  int lleft = 0;
  bool log_full = false;
  const float lam1 = (float)a.lambda1, lam2 = (float)a.lambda2;
  const float b1 = (float)a.beta1, b2 = (float)a.beta2, omb1 = (float)a.one_minus_b1, omb2 = (float)a.one_minus_b2;
  const float eps = (float)a.eps;

  // Every load of the state is complete before the loop, whose only vector
  // memory operations are the log stores; a wait inside the loop would also
  // wait for those stores to reach memory.
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  for (int k = 0; k < a.T; ++k) {
    // ---- forward Y^T = B Z^T, then signs (kept in the accumulators) ----
    floatx4 acc[NB];
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) acc[ib] = floatx4{0.f, 0.f, 0.f, 0.f};
    if (k < a.bf16_iters) {
#pragma unroll
      for (int jb = 0; jb < DB; ++jb) {
        shortx4 hi, lo;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          short h = bf16_rne(z[jb][r]);
          hi[r] = h;
          lo[r] = bf16_rne(z[jb][r] - bf16_to_f(h));
        }
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
          const shortx4 A = sFB[(ib * DB + jb) * 64 + lane];
          acc[ib] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, hi, acc[ib], 0, 0, 0);
          acc[ib] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, lo, acc[ib], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int jb = 0; jb < DB; ++jb) {
        floatx4 A[NB];
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) A[ib] = sFA[(ib * DB + jb) * 64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int ib = 0; ib < NB; ++ib)
            acc[ib] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ib][r], z[jb][r], acc[ib], 0, 0, 0);
      }
    }
    // Scheduling barriers keep the phases (forward, backward, Adam,
    // collection) from being interleaved, which bounds live ranges: the
    // kernel then fits 2 waves per SIMD without spills.
    __builtin_amdgcn_sched_barrier(0);
    // ---- backward G^T = B^T sign(Y)^T on exact bf16 operands ----
    floatx4 gacc[DB];
#pragma unroll
    for (int jb = 0; jb < DB; ++jb) gacc[jb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ip = 0; ip < NBP; ++ip) {
      shortx8 sg;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sg[r] = sign_bf16(acc[2 * ip][r]);
        sg[4 + r] = 2 * ip + 1 < NB ? sign_bf16(acc[2 * ip + 1][r]) : (short)0;
      }
#pragma unroll
      for (int jb = 0; jb < DB; ++jb)
        gacc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, sBT[(jb * NBP + ip) * 64 + lane]),
                                                           __builtin_bit_cast(bf16x8, sg), gacc[jb], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- barrier term: ||z||_inf and ties, per start (4 lanes) ----
    float mu = 0.f;
#pragma unroll
    for (int jb = 0; jb < DB; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) mu = fmaxf(mu, fabsf(z[jb][r]));
    mu = xmax4(mu);
    const bool bar = mu > 0.f && mu < 1.f;
    // the barrier term acts only while ||z||_inf < 1, which is rare: its tie
    // count and its gradient run only in waves where some start needs them
    const bool wave_bar = __ballot(bar) != 0;
    float wbar = 0.f;
    if (wave_bar) {
      float cnt = 0.f;
#pragma unroll
      for (int jb = 0; jb < DB; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) cnt += fabsf(z[jb][r]) == mu ? 1.f : 0.f;
      cnt = xsum4(cnt);
      wbar = bar ? lam2 / ((mu * mu) * cnt) : 0.f;
    }
    // per-iteration Adam factors: a uniform read of data no launch writes,
    // which the compiler keeps off the vector memory counter (so the wait
    // for it does not also wait for this wave's log stores)
    const float2 sf = stepf[k];
    const float step = sf.x, ib2 = sf.y;
    // ---- gradient, Adam, rounding ----
    // the largest |z_j| and the largest rounding change decide the range and
    // change flags (the same tests as per coordinate, in fewer instructions)
    float zmax = 0.f, dmax = 0.f;
    floatx4 dr[DB];
#pragma unroll
    for (int jb = 0; jb < DB; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float zj = z[jb][r];
        float g = gacc[jb][r] + lam1 * ((ceilf(zj) + floorf(zj)) - 2.f * zj);
        if (bar && fabsf(zj) == mu) g -= zj > 0.f ? wbar : -wbar;
        const float mj = b1 * m[jb][r] + omb1 * g;
        const float vj = b2 * v[jb][r] + omb2 * (g * g);
        m[jb][r] = mj;
        v[jb][r] = vj;
        const float zn = zj - (step * mj) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vj * ib2) + eps);
        z[jb][r] = zn;
        const float rn = rintf(zn);
        const float d = rn - rp[jb][r];
        dmax = fmaxf(dmax, fabsf(d));
        zmax = fmaxf(zmax, fabsf(rn));
        dr[jb][r] = d;
        rp[jb][r] = rn;
      }
    int changed = (dmax > 0.f) | (k == 0);
    int inrange = zmax <= zrange;  // zmax: largest |r_j| of the new iterate
    int jump = dmax > zrange;      // a step too large for an exact update of g
    __builtin_amdgcn_sched_barrier(0);
    if (!a.collect) continue;
    // ---- per-start flags (the 4 lanes of a start agree afterwards) ----
    inrange = xand4(inrange);
    changed = xor4(changed);
    jump = xor4(jump);
    // An iterate beyond the exact range yields no candidate and g is not
    // updated; the first iterate back in range (or one that moved by more
    // than the range in one step) forms g = B r from zero, so every partial
    // sum stays within the range and the set does not depend on how the run
    // is split into launches.
    const bool fresh = inrange && (!exact || jump);
    if (!inrange) {
      n_range += (q == 0 && svalid && changed) ? 1 : 0;
#pragma unroll
      for (int jb = 0; jb < DB; ++jb) dr[jb] = floatx4{0.f, 0.f, 0.f, 0.f};
    } else if (fresh) {
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) gi[ib][r] = 0;
#pragma unroll
      for (int jb = 0; jb < DB; ++jb) dr[jb] = floatx4{rp[jb][0], rp[jb][1], rp[jb][2], rp[jb][3]};
    }
    exact = inrange;
    const bool emit = svalid && inrange && changed;
    // ---- exact candidate update g += B (r - r_prev) on changed blocks ----
    // After the first step |r - r_prev| is small (an Adam step moves z by
    // about lr), so the 4 differences of a block are exact bf16 operands; the
    // first step (r_prev = 0) and any larger jump use the binary32 product.
    floatx4 dg[NB];
    bool any = false;
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) dg[ib] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jb = 0; jb < DB; ++jb) {
      const bool nz = (dr[jb][0] != 0.f) | (dr[jb][1] != 0.f) | (dr[jb][2] != 0.f) | (dr[jb][3] != 0.f);
      if (__ballot(nz) == 0) continue;
      any = true;
      const bool small = fabsf(dr[jb][0]) <= 256.f && fabsf(dr[jb][1]) <= 256.f && fabsf(dr[jb][2]) <= 256.f &&
                         fabsf(dr[jb][3]) <= 256.f;
      if (k > 0 && __ballot(!small) == 0) {
        shortx4 dp;
#pragma unroll
        for (int r = 0; r < 4; ++r) dp[r] = (short)(__float_as_uint(dr[jb][r]) >> 16);
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
          dg[ib] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(sFB[(ib * DB + jb) * 64 + lane], dp, dg[ib], 0, 0, 0);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int ib = 0; ib < NB; ++ib)
            dg[ib] = __builtin_amdgcn_mfma_f32_16x16x4f32(sFA[(ib * DB + jb) * 64 + lane][r], dr[jb][r], dg[ib], 0,
                                                           0, 0);
      }
    }
    if (any) {
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) gi[ib][r] += (int)dg[ib][r];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (__ballot(emit) == 0) continue;
    // ---- box test (condition C4) and nonzero test ----
    int inbox = 1, nonzero = 0;
    if (lim_uniform >= 0) {
      // one width for every coordinate: the largest |g_i| decides both tests
      int amax = 0;
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) amax = max(amax, max(gi[ib][r], -gi[ib][r]));
      amax = max(amax, __shfl_xor(amax, 16, 64));
      amax = max(amax, __shfl_xor(amax, 32, 64));
      inbox = amax <= lim_uniform;
      nonzero = amax > 0;
    } else {
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int g = gi[ib][r];
          const int lim = sLim[16 * ib + 4 * q + r];
          inbox &= (g <= lim) & (g >= -lim);
          nonzero |= g != 0;
        }
      inbox = xand4(inbox);
      nonzero = xor4(nonzero);
    }
    const bool put = emit && inbox && nonzero;
    n_emit += (q == 0 && emit) ? 1 : 0;
    n_inbox += (q == 0 && put) ? 1 : 0;
    const uint64_t pm = __ballot(put && q == 0);  // bit s: start s of this wave logs a key
    if (pm == 0) continue;
    // ---- append the keys to the candidate log --------------------------
    // Each lane holds rows 16ib + 4q .. +3 of its start's g: one dword per
    // block.  Slots come from per-wave chunks of kLogChunk rows reserved with
    // one atomic; unused slots are zeroed (the log reader skips zero rows).
    const int npu = __popcll(pm);
    if (npu > lleft && !log_full) {
      if (lleft > 0) {
        zero_rows(log, lbase + lused, (uint32_t)lleft, lane);
        lleft = 0;
      }
      uint32_t nb = 0;
      if (lane == 0) nb = atomicAdd(log.count, (uint32_t)kLogChunk);
      nb = __builtin_amdgcn_readfirstlane(nb);
      if (nb < log.cap) {
        const uint32_t end = min(log.cap, nb + (uint32_t)kLogChunk);
        lbase = nb;
        lused = 0;
        lleft = (int)(end - nb);
      }
    }
    if (npu > lleft) {
      // the log is exhausted: flag it; the host replays this call in shorter
      // pieces, so no candidate is lost
      if (!log_full && lane == 0) atomicOr(log.count + 1, 1u);
      log_full = true;
      continue;
    }
    {
      const uint32_t rank = (uint32_t)__popcll(pm & ((1ull << sl) - 1ull));
      if (put) {
        uint32_t* row = reinterpret_cast<uint32_t*>(log.rows + (size_t)(lbase + lused + rank) * stride);
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
          uint32_t w = 0;
#pragma unroll
          for (int r = 0; r < 4; ++r) w |= ((uint32_t)(uint8_t)(int8_t)gi[ib][r]) << (8 * r);
          row[4 * ib + q] = w;
        }
      }
      lused += (uint32_t)npu;
      lleft -= npu;
    }
  }
  if (lleft > 0) zero_rows(log, lbase + lused, (uint32_t)lleft, lane);
#pragma unroll
  for (int jb = 0; jb < DB; ++jb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      size_t e = base + (size_t)(4 * jb + r) * 64;
      state[e] = z[jb][r];
      state[per + e] = m[jb][r];
      state[2 * per + e] = v[jb][r];
    }
  // wave-reduce the counters, one atomic per wave
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

template <int NB, int DB>
static hipError_t launch_nd(hipStream_t s, const DescentArgs& a, const float* FA, const float* BA, float* state,
                            PoolDev pool, unsigned long long* counters, float zrange) {
  const int lim_uniform = a.lim_uniform;
  const int64_t nw = n_waves(a.N);
  const int64_t per = nw * 4 * DB * 64;
  const size_t shmem = (size_t)NB * DB * 64 * (sizeof(floatx4) + sizeof(shortx4)) +
                       (size_t)((NB + 1) / 2) * DB * 64 * sizeof(shortx8) + 16 * NB * sizeof(int);
  auto kern = k_descent_f32<NB, DB>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  const size_t nblk64 = (size_t)NB * DB * 64;
  hipLaunchKernelGGL(kern, dim3((unsigned)(nw / kWavesPerBlock)), dim3(64 * kWavesPerBlock), shmem, s, a,
                     reinterpret_cast<const floatx4*>(FA), reinterpret_cast<const shortx4*>(FA + nblk64 * 4),
                     reinterpret_cast<const shortx8*>(BA), state, pool, counters, zrange, per, lim_uniform,
                     a.log, reinterpret_cast<const float2*>(a.stepf));
  return hipGetLastError();
}

template <int NB, int DB>
static hipError_t dispatch_d(int db, hipStream_t s, const DescentArgs& a, const float* FA, const float* BA,
                             float* st, PoolDev p, unsigned long long* c, float zr) {
  if constexpr (DB > NB) {
    return hipErrorInvalidValue;
  } else {
    if (db == DB) return launch_nd<NB, DB>(s, a, FA, BA, st, p, c, zr);
    if constexpr (DB > 1) return dispatch_d<NB, DB - 1>(db, s, a, FA, BA, st, p, c, zr);
    return hipErrorInvalidValue;
  }
}

template <int NB>
static hipError_t dispatch_n(int nb, int db, hipStream_t s, const DescentArgs& a, const float* FA, const float* BA,
                             float* st, PoolDev p, unsigned long long* c, float zr) {
  if (nb == NB) return dispatch_d<NB, NB>(db, s, a, FA, BA, st, p, c, zr);
  if constexpr (NB > 1) return dispatch_n<NB - 1>(nb, db, s, a, FA, BA, st, p, c, zr);
  return hipErrorInvalidValue;
}

hipError_t launch_descent_f32(hipStream_t s, const DescentArgs& a, const float* FA, const float* BA, float* state,
                              PoolDev pool, unsigned long long* counters, float zrange) {
  return dispatch_n<kMaxBlk>(blk(a.n), blk(a.d), s, a, FA, BA, state, pool, counters, zrange);
}

}  // namespace graver
