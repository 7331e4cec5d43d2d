// Descent of eq. loss with Parallel Extraction (Algorithm 2, Section 3.2) in
// binary32 for sparse kernel bases.
//
// A kernel basis of a sparse constraint matrix is itself sparse: the quartic
// workload's B (400 x 350) holds 702 nonzeros.  The matrix-core descent pays
// 4 n d flop per start-iteration whatever the sparsity; this kernel pays for
// the nonzeros only.  One wavefront runs one start (then the next, for grids
// capped below the start count).  Lane l holds coordinates j = l + 64 c,
// c < DC, of z, m and v in registers for the whole launch; B's rows, as
// slot-uniform row lists (descent_sparse.h), sit in LDS once per block.  Per
// iteration and slot of 64 rows (one row per lane):
//   y_i   = sum_j B_ij z_j        gathers of z from the wave's LDS copy, in a
//                                 fixed order per row (deterministic)
//   G_j  += B_ij sign(y_i)        integer LDS atomic adds of +-B_ij right
//                                 after the row's sum (exact in any order;
//                                 float atomic adds measured 4x slower)
//   g_i   = sum_j B_ij round(z_j) from the same gathers when the rounding
//                                 changed (exact: |round(z_j)| <= rlim keeps
//                                 every partial sum below 2^24)
// then the integrality and barrier terms and Adam, exactly as in the
// matrix-core kernels.  The infinity norm and its ties are needed only when
// every |z_j| < 1, so per iteration they cost two ballots; the exact
// reduction runs only then.  A candidate row is staged in LDS and appended
// to the candidate log when it is nonzero and inside the box.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "descent_sparse.h"

namespace graver {
namespace {

constexpr int kSpWaves = 4;       // starts (wavefronts) per block
constexpr int kSpLogChunk = 16;   // log rows reserved by a wave at a time (at most)
constexpr int kSpMaxSlots = 16;   // n <= 1024
constexpr int kSpMaxEntries = 128;  // row-list entries per lane (32 KB of LDS)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct SparseArgs {
  DescentArgs a;
  const uint32_t* ent;  // ew x 64 entry words
  const uint32_t* row;  // nc x 64 row words
  uint32_t slot[kSpMaxSlots];  // width | first entry << 16
  int nc, ew, DB, stride;
  uint32_t chunk;  // log rows a wave reserves at a time
  float* state;  // z, then m, then v, `per` floats each (wave-native layout)
  int64_t per;
  unsigned long long* counters;
  float rlim;
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// The wave-native layout (16 starts by DB column blocks per group) puts
// coordinate j of start s at start_base(s) + coord_off(j).
__device__ __forceinline__ int64_t start_base(int64_t s, int DB) { return (s >> 4) * 4 * DB * 64 + (s & 15); }
__device__ __forceinline__ int coord_off(int j) { return (4 * (j >> 4) + (j & 3)) * 64 + 16 * ((j >> 2) & 3); }

__device__ __forceinline__ float wave_max(float x) {
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ float wave_sum(float x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// waves per SIMD the register budget is cut for (8: 64 registers, 6: 80,
// 5: 96; the largest count that needs no spills)
template <int DC>
constexpr int sp_waves_per_simd() { return DC <= 4 ? 8 : (DC <= 6 ? 6 : (DC <= 8 ? 5 : 1)); }

template <int DC>
__global__ __launch_bounds__(64 * kSpWaves, (sp_waves_per_simd<DC>())) void k_descent_sparse(SparseArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const DescentArgs& a = g.a;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nc = g.nc;
  // [row words | entry words | per wave: z (64 DC), gradient (64 DC) | per wave: key row]
  uint32_t* sRow = reinterpret_cast<uint32_t*>(smem);
  uint32_t* sEnt = sRow + nc * 64;
  float* zb = reinterpret_cast<float*>(sEnt + g.ew * 64) + (size_t)wid * 2 * 64 * DC;
  int* gb = reinterpret_cast<int*>(zb + 64 * DC);  // B^T sign(y): integers
  int8_t* kr = reinterpret_cast<int8_t*>(reinterpret_cast<float*>(sEnt + g.ew * 64) + (size_t)kSpWaves * 2 * 64 * DC) +
               (size_t)wid * g.stride;
  for (int i = threadIdx.x; i < nc * 64; i += blockDim.x) sRow[i] = g.row[i];
  for (int i = threadIdx.x; i < g.ew * 64; i += blockDim.x) sEnt[i] = g.ent[i];
  for (int b = a.n + lane; b < g.stride; b += 64) kr[b] = 0;  // key bytes beyond n stay zero
  __syncthreads();

  const float lam1 = (float)a.lambda1, lam2 = (float)a.lambda2;
  const float b1 = (float)a.beta1, b2 = (float)a.beta2, omb1 = (float)a.one_minus_b1, omb2 = (float)a.one_minus_b2;
  const float eps = (float)a.eps;
  const float rlim = g.rlim;
  const bool collect = a.collect != 0;
  const LogDev& log = a.log;
  const int d = a.d;

  unsigned long long n_emit = 0, n_inbox = 0, n_range = 0;
  uint32_t lbase = 0, lused = 0;
  int lleft = 0;
  bool log_full = false;

  const int64_t wstep = (int64_t)gridDim.x * kSpWaves;
  for (int64_t s = (int64_t)blockIdx.x * kSpWaves + wid; s < a.N; s += wstep) {
    // this start's state: a uniform base and 32-bit lane offsets
    auto Zs = gmem(g.state + start_base(s, g.DB));
    auto Ms = Zs + g.per;
    auto Vs = Zs + 2 * g.per;
    float z[DC], m[DC], v[DC];
#pragma unroll
    for (int c = 0; c < DC; ++c) {
      const int j = lane + 64 * c;
      const bool ok = j < d;
      const int o = ok ? coord_off(j) : 0;
      z[c] = ok ? Zs[o] : 0.f;
      m[c] = ok ? Ms[o] : 0.f;
      v[c] = ok ? Vs[o] : 0.f;
    }
    bool changed = false;
    for (int k = 0; k <= a.T; ++k) {
      const bool descend = k < a.T;
      int oor = 0;
#pragma unroll
      for (int c = 0; c < DC; ++c) oor |= fabsf(rintf(z[c])) > rlim;
      const bool inrange = __ballot(oor) == 0;
      const bool needg = collect && k > 0 && changed;
      if (!descend && !needg) break;
      const bool cand = needg && inrange;
#pragma unroll
      for (int c = 0; c < DC; ++c) {
        zb[c * 64 + lane] = z[c];
        gb[c * 64 + lane] = 0;
      }
      wave_sync();
      int inbox = 1, nonzero = 0;
      // one slot of 64 rows at a time: the rows' forward sums (and candidate
      // sums), then the signed scatter of the same entries into the gradient
      for (int t = 0; t < nc; ++t) {
        const uint32_t sw = g.slot[t];
        const int w = (int)(sw & 0xFFFFu), e0 = (int)(sw >> 16);
        const uint32_t* E = sEnt + e0 * 64 + lane;
        float run = 0.f, grun = 0.f;
        if (cand) {
          for (int e = 0; e < w; ++e) {
            const uint32_t en = E[e * 64];
            const float zc = zb[en & 0xFFFFu];
            const float bvv = (float)((int32_t)en >> 16);
            run = fmaf(bvv, zc, run);
            grun = fmaf(bvv, rintf(zc), grun);
          }
          const uint32_t ri = sRow[t * 64 + lane];
          const int rowi = (int)(ri & 0xFFFFu), lim = (int)(ri >> 16);
          if (rowi != 0xFFFF) {
            const int gv = (int)grun;
            inbox &= (gv <= lim) & (gv >= -lim);
            nonzero |= gv != 0;
            kr[rowi] = (int8_t)gv;
          }
        } else {
          for (int e = 0; e < w; ++e) {
            const uint32_t en = E[e * 64];
            run = fmaf((float)((int32_t)en >> 16), zb[en & 0xFFFFu], run);
          }
        }
        // (padding entries, and rows with y = 0, add nothing and stay out of
        // the atomics: the padding entries of a slot all name column 0, and
        // same-address atomic adds serialize)
        if (descend && run != 0.f) {
          const bool neg = run < 0.f;
          for (int e = 0; e < w; ++e) {
            const uint32_t en = E[e * 64];
            const int b = (int32_t)en >> 16;
            if (b != 0) __hip_atomic_fetch_add(&gb[en & 0xFFFFu], neg ? -b : b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
          }
        }
      }
      wave_sync();
      if (needg) {
        if (!inrange) {
          ++n_range;
        } else {
          ++n_emit;
          const bool put = __ballot(!inbox) == 0 && __ballot(nonzero) != 0;
          if (put) {
            ++n_inbox;
            if (lleft == 0 && !log_full) {
              uint32_t nb = 0;
              if (lane == 0) nb = atomicAdd(log.count, g.chunk);
              nb = __builtin_amdgcn_readfirstlane(nb);
              if (nb < log.cap) {
                lbase = nb;
                lused = 0;
                lleft = (int)(min(log.cap, nb + g.chunk) - nb);
              }
            }
            if (lleft == 0) {
              if (!log_full && lane == 0) atomicOr(log.count + 1, 1u);
              log_full = true;
            } else {
              auto dst = gmem(reinterpret_cast<u32x4*>(log.rows + (size_t)(lbase + lused) * g.stride));
              const u32x4* src = reinterpret_cast<const u32x4*>(kr);
              for (int c = lane; c < g.stride / 16; c += 64) dst[c] = src[c];
              ++lused;
              --lleft;
            }
          }
        }
      }
      if (!descend) break;

      // integrality and barrier terms, Adam, and the change flag
      int big = 0, nzr = 0;
#pragma unroll
      for (int c = 0; c < DC; ++c) {
        big |= fabsf(z[c]) >= 1.f;
        nzr |= z[c] != 0.f;
      }
      const bool bar = __ballot(big) == 0 && __ballot(nzr) != 0;  // 0 < ||z||_inf < 1
      float mu = 0.f, wbar = 0.f;
      if (bar) {
        float mx = 0.f;
#pragma unroll
        for (int c = 0; c < DC; ++c) mx = fmaxf(mx, fabsf(z[c]));
        mu = wave_max(mx);
        float cnt = 0.f;
#pragma unroll
        for (int c = 0; c < DC; ++c) cnt += fabsf(z[c]) == mu ? 1.f : 0.f;
        cnt = wave_sum(cnt);
        wbar = lam2 / ((mu * mu) * cnt);
      }
      const float step = a.stepf[2 * k], ib2 = a.stepf[2 * k + 1];
      int ch = 0;
#pragma unroll
      for (int c = 0; c < DC; ++c) {
        const float zj = z[c];
        float gg = (float)gb[c * 64 + lane] + lam1 * ((ceilf(zj) + floorf(zj)) - 2.f * zj);
        if (bar && fabsf(zj) == mu) gg -= zj > 0.f ? wbar : -wbar;
        const float mj = b1 * m[c] + omb1 * gg;
        const float vj = b2 * v[c] + omb2 * (gg * gg);
        const float zn = zj - (step * mj) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vj * ib2) + eps);
        ch |= rintf(zn) != rintf(zj);
        z[c] = zn;
        m[c] = mj;
        v[c] = vj;
      }
      changed = k == 0 || __ballot(ch) != 0;
    }
#pragma unroll
    for (int c = 0; c < DC; ++c) {
      const int j = lane + 64 * c;
      if (j < d) {
        const int o = coord_off(j);
        Zs[o] = z[c];
        Ms[o] = m[c];
        Vs[o] = v[c];
      }
    }
  }
  if (lleft > 0) {
    const int dw = g.stride / 4;
    auto base = gmem(reinterpret_cast<uint32_t*>(log.rows + (size_t)(lbase + lused) * g.stride));
    for (uint32_t t = lane; t < (uint32_t)lleft * (uint32_t)dw; t += 64) base[t] = 0u;
  }
  if (lane == 0) {
    if (n_emit) atomicAdd(&g.counters[C_EMIT], n_emit);
    if (n_inbox) atomicAdd(&g.counters[C_INBOX], n_inbox);
    if (n_range) atomicAdd(&g.counters[C_RANGE], n_range);
  }
}

constexpr int kDC[] = {2, 4, 6, 8, 12, 16};

template <int DC>
hipError_t launch_t(hipStream_t s, const SparseArgs& g, size_t shmem, unsigned blocks) {
  auto kern = k_descent_sparse<DC>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * kSpWaves), shmem, s, g);
  return hipGetLastError();
}

int dc_of(int d) {
  for (int dc : kDC)
    if (64 * dc >= d) return dc;
  return 0;
}

}  // namespace

bool sparse_image_build(int n, int d, const int64_t* B, const int64_t* l, const int64_t* u, SparseImage& img) {
  img = SparseImage{};
  if (n < 1 || n > 64 * kSpMaxSlots || d < 1 || dc_of(d) == 0) return false;
  std::vector<std::vector<std::pair<int, int>>> rows((size_t)n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < d; ++j) {
      const int64_t b = B[(size_t)i * d + j];
      if (b == 0) continue;
      if (b < -32767 || b > 32767) return false;
      rows[(size_t)i].push_back({j, (int)b});
    }
  std::vector<int> order((size_t)n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return rows[(size_t)x].size() > rows[(size_t)y].size(); });
  const int nc = (n + 63) / 64;
  int ew = 0;
  for (int t = 0; t < nc; ++t) {
    const int w = (int)rows[(size_t)order[(size_t)(64 * t)]].size();
    img.slot[t] = (uint32_t)w | (uint32_t)ew << 16;
    ew += w;
  }
  if (ew > kSpMaxEntries) return false;
  img.ew = ew;
  img.nc = nc;
  img.ent.assign((size_t)std::max(ew, 1) * 64, 0u);
  img.row.assign((size_t)nc * 64, 0xFFFFu);
  // Within a slot, the entries of one position e are one LDS instruction
  // over the 64 lanes, and lanes that name the same column serialize in the
  // gradient's atomic adds.  Each row's entries are therefore placed, most
  // frequent columns first, at the free position where their column is
  // rarest so far (a greedy edge colouring of the slot's rows x columns).
  std::vector<int> colfreq((size_t)d, 0);
  for (const auto& r : rows)
    for (const auto& e : r) ++colfreq[(size_t)e.first];
  for (int t = 0; t < nc; ++t) {
    const int e0 = (int)(img.slot[t] >> 16), w = (int)(img.slot[t] & 0xFFFFu);
    std::vector<int> cnt((size_t)w * d, 0);
    for (int ln = 0; ln < 64; ++ln) {
      const int p = 64 * t + ln;
      if (p >= n) continue;
      const int i = order[(size_t)p];
      img.row[(size_t)t * 64 + ln] = (uint32_t)i | (uint32_t)(u[i] - l[i]) << 16;
      auto r = rows[(size_t)i];
      std::stable_sort(r.begin(), r.end(), [&](const std::pair<int, int>& x, const std::pair<int, int>& y) {
        return colfreq[(size_t)x.first] > colfreq[(size_t)y.first];
      });
      std::vector<char> used((size_t)w, 0);
      for (const auto& e : r) {
        int best = -1;
        for (int q = 0; q < w; ++q)
          if (!used[(size_t)q] && (best < 0 || cnt[(size_t)q * d + e.first] < cnt[(size_t)best * d + e.first])) best = q;
        used[(size_t)best] = 1;
        ++cnt[(size_t)best * d + e.first];
        img.ent[(size_t)(e0 + best) * 64 + ln] = (uint32_t)e.first | (uint32_t)(uint16_t)(int16_t)e.second << 16;
      }
    }
  }
  return true;
}

bool sparse_form_pays(const SparseImage& img, int n, int d) {
  return img.nc > 0 && (int64_t)img.ew * 64 * 8 <= (int64_t)n * d;
}

hipError_t launch_descent_sparse(hipStream_t s, const DescentArgs& a, const SparseImage& img, const uint32_t* dev_ent,
                                 const uint32_t* dev_row, float* state, int64_t per, unsigned long long* counters,
                                 float rlim) {
  const int dc = dc_of(a.d);
  if (dc == 0 || img.nc < 1 || img.nc > kSpMaxSlots || a.N < 1) return hipErrorInvalidValue;
  SparseArgs g{};
  g.a = a;
  g.ent = dev_ent;
  g.row = dev_row;
  for (int t = 0; t < img.nc; ++t) g.slot[t] = img.slot[t];
  g.nc = img.nc;
  g.ew = img.ew;
  g.DB = (a.d + 15) / 16;
  g.stride = a.log.stride;
  g.state = state;
  g.per = per;
  g.counters = counters;
  g.rlim = rlim;
  // A wave leaves up to chunk - 1 reserved rows unused, so the reservation
  // shrinks with the log's capacity per start: the unused rows of one launch
  // stay within a quarter of the log (a small log then still holds the
  // candidates of one iteration whenever it holds one row per start).
  g.chunk = (uint32_t)std::min<int64_t>(kSpLogChunk, std::max<int64_t>(1, (int64_t)a.log.cap / (4 * a.N)));
  if (g.stride % 16 != 0 || g.stride < a.n) return hipErrorInvalidValue;
  const size_t shmem = (size_t)(img.nc + img.ew) * 64 * 4 + (size_t)kSpWaves * 2 * 64 * dc * 4 +
                       (size_t)kSpWaves * g.stride;
  const int64_t want = (a.N + kSpWaves - 1) / kSpWaves;
  const unsigned blocks = (unsigned)std::min<int64_t>(want, (int64_t)1 << 20);
  switch (dc) {
    case 2: return launch_t<2>(s, g, shmem, blocks);
    case 4: return launch_t<4>(s, g, shmem, blocks);
    case 6: return launch_t<6>(s, g, shmem, blocks);
    case 8: return launch_t<8>(s, g, shmem, blocks);
    case 12: return launch_t<12>(s, g, shmem, blocks);
    case 16: return launch_t<16>(s, g, shmem, blocks);
  }
  return hipErrorInvalidValue;
}

}  // namespace graver
