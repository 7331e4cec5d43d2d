// Multi-start augmentation (Algorithm 1 from every start, MAPE Section 3.3)
// on gfx950.  One step for all active starts is three launches:
//   prepare : quadratic r = c + 2 Q x per start; separable p_i(x_i) per start
//   eval    : grid (direction blocks) x (starts); each thread scores one
//             direction g and its negation over lambda = 1..lambda_max and
//             the block keeps the best (Delta, position, lambda)
//   pick    : per start, the best over blocks (a total order, so the result
//             does not depend on the reduction order); x += lambda g when
//             Delta < 0, otherwise the start is finished.
// Every Delta is the fixed binary64 formula of the header with ascending
// sums over the support of g and no fused multiply-add (this file is
// compiled with -ffp-contract=off), so moves match a plain evaluation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "graver_internal.h"

namespace graver {

struct Move {
  double delta;
  uint32_t pos;  // position in D: 2k for row k, 2k+1 for its negation
  int32_t lam;
};

__device__ __forceinline__ bool better(const Move& a, const Move& b) {
  if (a.delta != b.delta) return a.delta < b.delta;
  if (a.pos != b.pos) return a.pos < b.pos;
  return a.lam < b.lam;
}

// start feasibility: thread t < S*m checks row t % m of A x = b for start
// t / m; the next S*n threads check l <= x <= u coordinate by coordinate
__global__ void k_check_starts(int n, int m, int S, const int64_t* A, const int64_t* b, const int64_t* l,
                               const int64_t* u, const int64_t* X, unsigned int* bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = (int64_t)S * m;
  bool ok = true;
  if (t < rows) {
    const int s = (int)(t / m), r = (int)(t % m);
    const int64_t* x = X + (size_t)s * n;
    int64_t acc = 0;
    for (int j = 0; j < n; ++j) acc += A[(size_t)r * n + j] * x[j];
    ok = acc == b[r];
  } else if (t < rows + (int64_t)S * n) {
    const int64_t k = t - rows;
    const int i = (int)(k % n);
    ok = X[k] >= l[i] && X[k] <= u[i];
  }
  if (!ok) atomicAdd(bad, 1u);
}

__global__ void k_copy_i64(const int64_t* a, int64_t* b, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}
__global__ void k_zero_u32(uint32_t* a, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}
__global__ void k_zero_i64(int64_t* a, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// tab[i * w + (v - l_i)] = p_i(v) by Horner from the top coefficient.
__global__ void k_poly_table(int n, int deg, int w, const double* coef, const int64_t* l, const int64_t* u,
                             double* tab) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  int i = t / w, o = t % w;
  int64_t v = l[i] + o;
  if (v > u[i]) return;
  const double* c = coef + (size_t)i * (deg + 1);
  double x = (double)v;
  double p = c[deg];
  for (int k = deg - 1; k >= 0; --k) p = p * x + c[k];
  tab[t] = p;
}

// quadratic: r[s, i] = c_i + 2 * (sum_j Q_ij x_j); separable: px[s, i] = p_i(x_i).
__global__ void k_prepare(AugArgs a, const int64_t* X, const uint32_t* done, const double* tab, int w,
                          double* R) {
  int s = blockIdx.y;
  if (done[s]) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t* x = X + (size_t)s * a.n;
  if (a.kind == GRAVER_F_QUADRATIC) {
    double acc = 0.0;
    for (int j = 0; j < a.n; ++j) acc = acc + a.Q[(size_t)i * a.n + j] * (double)x[j];
    R[(size_t)s * a.n + i] = a.c[i] + 2.0 * acc;
  } else {
    R[(size_t)s * a.n + i] = tab[(size_t)i * w + (x[i] - a.l[i])];
  }
}

constexpr int kEvalThreads = 256;
constexpr int kStartGroup = 16;  // 2 bits per start in a 32-bit feasibility mask

// q_g of one direction (ascending sums over its support), computed the
// first time some start can move along g and cached for the call.  The
// cache holds kQgUnset until then; a cached value is one 64-bit word read
// and written with relaxed atomics (q_g is a function of g and Q alone, so
// a thread that misses the cache computes the same bits).
constexpr uint64_t kQgUnset = 0x7FF4A3C5E1F00D01ull;  // a NaN payload no binary64 arithmetic produces
__device__ double qg_of(const int8_t* g, int n, const double* Q) {
  double q = 0.0;
  for (int i = 0; i < n; ++i) {
    if (g[i] == 0) continue;
    double t = 0.0;
    for (int j = 0; j < n; ++j) {
      if (g[j] == 0) continue;
      t = t + Q[(size_t)i * n + j] * (double)g[j];
    }
    q = q + (double)g[i] * t;
  }
  return q;
}

__device__ __forceinline__ void wave_best(Move& b) {
  // no lane holds a move: every lane already has the empty move
  if (__ballot(b.pos != 0xFFFFFFFFu) == 0) return;
  for (int o = 32; o > 0; o >>= 1) {
    Move o2;
    o2.delta = __shfl_xor(b.delta, o, 64);
    o2.pos = __shfl_xor(b.pos, o, 64);
    o2.lam = __shfl_xor(b.lam, o, 64);
    if (better(o2, b)) b = o2;
  }
}

// Thread = one direction g, looping over a group of starts.  A move along
// +g or -g exists only if lambda = 1 is feasible (the box is convex and x
// is inside it), which is tested first with an early exit; lambda_max,
// a_g and q_g are computed only for feasible directions.
__global__ void k_eval(AugArgs a, const int64_t* X, const uint32_t* done, const double* R, uint64_t* qg,
                       const double* tab, int w, int lds_r, Move* partial) {
  const int n = a.n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int s0 = blockIdx.y * kStartGroup;
  const int8_t* g = a.dirs + (size_t)(k < a.K ? k : 0) * n;
  __shared__ Move sh[kStartGroup][kEvalThreads / 64];
  // slacks of the group's starts as int8 (exact: every width u_i - l_i is
  // at most 127); x_i + g_i stays in [l_i, u_i] iff -dn_i <= g_i <= up_i.
  // With lds_r the group's r rows follow them.
  extern __shared__ __align__(16) int8_t slack[];  // [kStartGroup][2][n]: up, then dn
  double* sR = reinterpret_cast<double*>(slack + ((size_t)kStartGroup * 2 * n + 15) / 16 * 16);
  for (int t = threadIdx.x; t < kStartGroup * n; t += blockDim.x) {
    const int si = t / n, i = t % n, s = s0 + si;
    int64_t up = 0, dn = 0;
    if (s < a.S) {
      const int64_t xi = X[(size_t)s * n + i];
      up = a.u[i] - xi;
      dn = xi - a.l[i];
      if (lds_r) sR[t] = R[(size_t)s * n + i];
    }
    slack[(size_t)si * 2 * n + i] = (int8_t)up;
    slack[(size_t)si * 2 * n + n + i] = (int8_t)dn;
  }
  __syncthreads();
  // lambda = 1 feasibility of +g and -g for every start of the group in one
  // pass over g: bit 2 si is x + g, bit 2 si + 1 is x - g; the pass stops
  // when no (start, sign) is left (a direction infeasible at lambda = 1 is
  // infeasible for every lambda)
  uint32_t fmask = 0;
  bool any = false;
  if (k < a.K) {
    for (int si = 0; si < kStartGroup; ++si) {
      const int s = s0 + si;
      if (s < a.S && !done[s]) fmask |= 3u << (2 * si);
    }
    // g is read four bytes at a time when its rows are 4-byte aligned
    const bool words = (n & 3) == 0 && (reinterpret_cast<uintptr_t>(a.dirs) & 3) == 0;
    for (int i0 = 0; i0 < n && fmask; i0 += 4) {
      uint32_t quad = 0;
      if (words) {
        quad = *reinterpret_cast<const uint32_t*>(g + i0);
      } else {
        for (int b = 0; b < 4 && i0 + b < n; ++b) quad |= (uint32_t)(uint8_t)g[i0 + b] << (8 * b);
      }
      for (int b = 0; b < 4 && fmask; ++b) {
        const int gi = (int8_t)(quad >> (8 * b));
        if (gi == 0) continue;
        const int i = i0 + b;
        any = true;
#pragma unroll
        for (int si = 0; si < kStartGroup; ++si) {
          const int up = slack[(size_t)si * 2 * n + i], dn = slack[(size_t)si * 2 * n + n + i];
          const uint32_t ok = ((gi <= up && -gi <= dn) ? 1u : 0u) | ((-gi <= up && gi <= dn) ? 2u : 0u);
          fmask &= ~((3u & ~ok) << (2 * si));
        }
      }
    }
  }
  for (int si = 0; si < kStartGroup; ++si) {
    const int s = s0 + si;
    Move best{INFINITY, 0xFFFFFFFFu, 0};
    const bool fp = (fmask >> (2 * si)) & 1u, fn = (fmask >> (2 * si + 1)) & 1u;
    if (s < a.S && !done[s] && k < a.K) {
      const int64_t* x = X + (size_t)s * n;
      if (any && (fp || fn)) {
        // lambda_max of +g and -g and, for a quadratic, a_g = sum g_i r_i in
        // one pass over the support of g (ascending i)
        const double* r = lds_r ? sR + (size_t)si * n : R + (size_t)s * n;
        const bool quad = a.kind == GRAVER_F_QUADRATIC;
        // the slacks are exact: every width u_i - l_i is at most 127 (int8
        // keys; the entry points reject wider boxes)
        const int8_t* su = slack + (size_t)si * 2 * n;
        const int8_t* sd = su + n;
        int lpi = INT_MAX, lni = INT_MAX;
        double ag = 0.0;
        for (int i = 0; i < n; ++i) {
          const int gi = g[i];
          if (gi == 0) continue;
          const int up = su[i], dn = sd[i];
          if (gi > 0) {
            lpi = min(lpi, up / gi);
            lni = min(lni, dn / gi);
          } else {
            lpi = min(lpi, dn / (-gi));
            lni = min(lni, up / (-gi));
          }
          if (quad) ag = ag + (double)gi * r[i];
        }
        const int64_t lp = lpi, ln = lni;
        if (quad) {
          uint64_t qbits = __hip_atomic_load(&qg[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (qbits == kQgUnset) {
            qbits = __double_as_longlong(qg_of(g, n, a.Q));
            __hip_atomic_store(&qg[k], qbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          const double q = __longlong_as_double(qbits);
          for (int sg = 0; sg < 2; ++sg) {
            const int64_t lm = sg ? ln : lp;
            const double av = sg ? -ag : ag;
            for (int64_t lam = 1; lam <= lm; ++lam) {
              double lf = (double)lam;
              Move mv{(lf * av) + ((lf * lf) * q), (uint32_t)(2 * k + sg), (int32_t)lam};
              if (better(mv, best)) best = mv;
            }
          }
        } else {
          // the support of g in ascending order, gathered once for every
          // step length (the sums below run over it in the same order as a
          // scan of all n coordinates that skips zeros); a support longer
          // than kSupp is scanned in full
          constexpr int kSupp = 8;
          int sidx[kSupp];
          int ns = 0;
          for (int i = 0; i < n && ns <= kSupp; ++i)
            if (g[i] != 0) {
              if (ns < kSupp) sidx[ns] = i;
              ++ns;
            }
          const bool compact = ns <= kSupp;
          for (int sg = 0; sg < 2; ++sg) {
            const int64_t lm = sg ? ln : lp;
            const int sgn = sg ? -1 : 1;
            for (int64_t lam = 1; lam <= lm; ++lam) {
              double acc = 0.0;
              if (compact) {
                for (int t = 0; t < ns; ++t) {
                  const int i = sidx[t];
                  const int64_t v = x[i] + lam * sgn * g[i];
                  acc = acc + (tab[(size_t)i * w + (v - a.l[i])] - r[i]);
                }
              } else {
                for (int i = 0; i < n; ++i) {
                  const int gi = g[i];
                  if (gi == 0) continue;
                  const int64_t v = x[i] + lam * sgn * gi;
                  acc = acc + (tab[(size_t)i * w + (v - a.l[i])] - r[i]);
                }
              }
              Move mv{acc, (uint32_t)(2 * k + sg), (int32_t)lam};
              if (better(mv, best)) best = mv;
            }
          }
        }
      }
    }
    wave_best(best);
    if ((threadIdx.x & 63) == 0) sh[si][threadIdx.x >> 6] = best;
  }
  __syncthreads();
  if (threadIdx.x < kStartGroup) {
    const int s = s0 + threadIdx.x;
    if (s < a.S) {
      Move best = sh[threadIdx.x][0];
      for (int wv = 1; wv < kEvalThreads / 64; ++wv)
        if (better(sh[threadIdx.x][wv], best)) best = sh[threadIdx.x][wv];
      partial[(size_t)s * gridDim.x + blockIdx.x] = best;
    }
  }
}

__global__ void k_pick(AugArgs a, int nblk, const Move* partial, int64_t* X, uint32_t* done, int64_t* steps,
                       uint32_t* active) {
  const int s = blockIdx.x;
  if (done[s]) return;
  __shared__ Move sh[256];
  Move best{INFINITY, 0xFFFFFFFFu, 0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    Move mv = partial[(size_t)s * nblk + b];
    if (better(mv, best)) best = mv;
  }
  sh[threadIdx.x] = best;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o && better(sh[threadIdx.x + o], sh[threadIdx.x])) sh[threadIdx.x] = sh[threadIdx.x + o];
    __syncthreads();
  }
  best = sh[0];
  const bool take = best.pos != 0xFFFFFFFFu && best.delta < 0.0 && steps[s] < a.max_steps;
  if (!take) {
    if (threadIdx.x == 0) done[s] = 1;
    return;
  }
  const int k = (int)(best.pos / 2);
  const int64_t mult = (best.pos & 1) ? -(int64_t)best.lam : (int64_t)best.lam;
  const int8_t* g = a.dirs + (size_t)k * a.n;
  for (int i = threadIdx.x; i < a.n; i += blockDim.x) X[(size_t)s * a.n + i] += mult * (int64_t)g[i];
  if (threadIdx.x == 0) {
    steps[s] += 1;
    atomicOr(active, 1u);
  }
}

// f(x) with ascending sums and separate rounding: quadratic
// (sum_i x_i * (sum_j Q_ij x_j)) + (sum_i c_i x_i); separable sum_i p_i(x_i).
__global__ void k_fval(AugArgs a, const int64_t* X, double* T, double* fout) {
  const int s = blockIdx.x;
  const int n = a.n;
  const int64_t* x = X + (size_t)s * n;
  double* t = T + (size_t)s * n;
  if (a.kind == GRAVER_F_QUADRATIC) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc = acc + a.Q[(size_t)i * n + j] * (double)x[j];
      t[i] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s1 = 0.0, s2 = 0.0;
      for (int i = 0; i < n; ++i) s1 = s1 + (double)x[i] * t[i];
      for (int i = 0; i < n; ++i) s2 = s2 + a.c[i] * (double)x[i];
      fout[s] = s1 + s2;
    }
  } else if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
      const double* c = a.coef + (size_t)i * (a.degree + 1);
      double xv = (double)x[i];
      double p = c[a.degree];
      for (int k = a.degree - 1; k >= 0; --k) p = p * xv + c[k];
      acc = acc + p;
    }
    fout[s] = acc;
  }
}

__global__ void k_best(int S, const double* f, int32_t* best) {
  if (threadIdx.x != 0) return;
  int b = 0;
  for (int s = 1; s < S; ++s)
    if (f[s] < f[b]) b = s;
  *best = b;
}

// dst[r, :] = src[idx[r], :] for r < cnt (int64 rows of n).
__global__ void k_gather_rows_i64(const int64_t* src, int n, const int32_t* idx, int64_t cnt, int64_t* dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt * n) return;
  const int64_t r = t / n;
  const int j = (int)(t % n);
  dst[t] = src[(size_t)idx[r] * n + j];
}

hipError_t launch_gather_rows_i64(hipStream_t s, const int64_t* src, int n, const int32_t* idx, int64_t cnt,
                                  int64_t* dst) {
  if (cnt > 0)
    hipLaunchKernelGGL(k_gather_rows_i64, dim3((unsigned)((cnt * n + 255) / 256)), dim3(256), 0, s, src, n, idx,
                       cnt, dst);
  return hipGetLastError();
}

size_t aug_work_bytes(int n, int S, int64_t K, int w) {
  const int nblk = K > 0 ? (int)((K + kEvalThreads - 1) / kEvalThreads) : 1;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  return al(64) + al((size_t)S * 4 + 64) + al((size_t)S * n * 8) + al((size_t)S * nblk * sizeof(Move)) +
         al((size_t)(K > 0 ? K : 1) * 8) + al((size_t)n * w * 8) + al(64);
}

AugWork aug_work_carve(void* base, int n, int S, int64_t K, int w) {
  const int nblk = K > 0 ? (int)((K + kEvalThreads - 1) / kEvalThreads) : 1;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  char* p = static_cast<char*>(base);
  AugWork wk{};
  wk.flags = reinterpret_cast<unsigned int*>(p);
  p += al(64);
  wk.done = reinterpret_cast<uint32_t*>(p);
  p += al((size_t)S * 4 + 64);
  wk.R = reinterpret_cast<double*>(p);
  p += al((size_t)S * n * 8);
  wk.partial = p;
  p += al((size_t)S * nblk * sizeof(Move));
  wk.qg = reinterpret_cast<uint64_t*>(p);
  p += al((size_t)(K > 0 ? K : 1) * 8);
  wk.tab = reinterpret_cast<double*>(p);
  p += al((size_t)n * w * 8);
  wk.best = reinterpret_cast<int32_t*>(p);
  return wk;
}

// Checks done on the device for callers that cannot copy the instance to
// the host: flag bit 0 when some l_i > u_i, bit 1 when some u_i - l_i > 127,
// bit 2 when Q (quadratic, may be NULL) is not symmetric.
__global__ void k_aug_validate(int n, const int64_t* l, const int64_t* u, const double* Q, unsigned int* flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned int bits = 0;
  if (t < n) {
    if (l[t] > u[t]) bits |= 1u;
    else if (u[t] - l[t] > 127) bits |= 2u;
  }
  if (Q && t < (int64_t)n * n) {
    const int64_t i = t / n, j = t % n;
    if (j < i && Q[i * n + j] != Q[j * n + i]) bits |= 4u;
  }
  if (bits) atomicOr(flag, bits);
}

hipError_t launch_aug_validate(hipStream_t s, int n, const int64_t* l, const int64_t* u, const double* Q,
                               unsigned int* flag) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, flag, (size_t)1);
  const int64_t cnt = Q ? (int64_t)n * n : n;
  hipLaunchKernelGGL(k_aug_validate, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, n, l, u, Q, flag);
  return hipGetLastError();
}

graver_status run_augment(graver_ctx* ctx, const AugArgs& a, int w, const int64_t* x_starts, int64_t* x_out,
                          double* f_out, int64_t* steps_out, int32_t* best_out) {
  graver_status st = GRAVER_OK;
  void* base = ws_get(ctx, WS_A_R, aug_work_bytes(a.n, a.S, a.K, w), &st);
  if (!base) return st;
  return run_augment_ws(ctx->stream, a, w, aug_work_carve(base, a.n, a.S, a.K, w), x_starts, x_out, f_out,
                        steps_out, best_out);
}

graver_status run_augment_ws(hipStream_t s, const AugArgs& a, int w, const AugWork& wk, const int64_t* x_starts,
                             int64_t* x_out, double* f_out, int64_t* steps_out, int32_t* best_out) {
  const int n = a.n, S = a.S, K = a.K;
  unsigned int* bad = wk.flags;
  uint32_t* done = wk.done;
  double* R = wk.R;
  const int nblk = K > 0 ? (K + kEvalThreads - 1) / kEvalThreads : 1;
  Move* partial = static_cast<Move*>(wk.partial);
  uint64_t* qg = wk.qg;
  int32_t* dbest = wk.best;

  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, bad, (size_t)16);
  const int64_t checks = (int64_t)S * (a.m + n);
  hipLaunchKernelGGL(k_check_starts, dim3((unsigned)((checks + 255) / 256)), dim3(256), 0, s, n, a.m, S, a.A, a.b,
                     a.l, a.u, x_starts, bad);
  unsigned int hbad = 0;
  HIP_TRY(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s), "augment start check");
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "augment start check");
  if (hbad) return set_error(GRAVER_E_INFEASIBLE_START, "a start violates A x = b or l <= x <= u");

  // value table for separable objectives: tab[i * w + (v - l_i)] = p_i(v),
  // w > max(u - l)
  const double* tab = nullptr;
  if (a.kind == GRAVER_F_SEPARABLE_POLY) {
    hipLaunchKernelGGL(k_poly_table, dim3((n * w + 255) / 256), dim3(256), 0, s, n, a.degree, w, a.coef, a.l,
                       a.u, wk.tab);
    tab = wk.tab;
  }
  size_t sn = (size_t)S * n;
  hipLaunchKernelGGL(k_copy_i64, dim3((unsigned)((sn + 255) / 256)), dim3(256), 0, s, x_starts, x_out, sn);
  hipLaunchKernelGGL(k_zero_u32, dim3((S + 255) / 256), dim3(256), 0, s, done, (size_t)S);
  hipLaunchKernelGGL(k_zero_i64, dim3((S + 255) / 256), dim3(256), 0, s, steps_out, (size_t)S);
  if (K > 0) HIP_TRY(launch_fill_u64(s, qg, (uint64_t)K, kQgUnset), "q_g cache");
  // the group's r rows go to LDS next to the slacks while they fit
  const int lds_r = a.kind == GRAVER_F_QUADRATIC && n <= 256 ? 1 : 0;
  const size_t eval_shm = ((size_t)kStartGroup * 2 * n + 15) / 16 * 16 + (lds_r ? (size_t)kStartGroup * n * 8 : 0);

  uint32_t* active = bad + 4;
  if (K > 0) {
    for (;;) {
      hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, active, (size_t)1);
      hipLaunchKernelGGL(k_prepare, dim3((n + 127) / 128, S), dim3(128), 0, s, a, x_out, done, tab, w, R);
      hipLaunchKernelGGL(k_eval, dim3(nblk, (S + kStartGroup - 1) / kStartGroup), dim3(kEvalThreads),
                         eval_shm, s, a, x_out, done, R, qg, tab, w, lds_r, partial);
      hipLaunchKernelGGL(k_pick, dim3(S), dim3(256), 0, s, a, nblk, partial, x_out, done, steps_out, active);
      uint32_t hact = 0;
      HIP_TRY(hipMemcpyAsync(&hact, active, 4, hipMemcpyDeviceToHost, s), "augment step");
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_error(e, "augment step");
      if (!hact) break;
    }
  }
  hipLaunchKernelGGL(k_fval, dim3(S), dim3(256), 0, s, a, x_out, R, f_out);
  hipLaunchKernelGGL(k_best, dim3(1), dim3(64), 0, s, S, f_out, dbest);
  int32_t hb = 0;
  HIP_TRY(hipMemcpyAsync(&hb, dbest, 4, hipMemcpyDeviceToHost, s), "augment objective");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "augment objective");
  if (best_out) *best_out = hb;
  return GRAVER_OK;
}

}  // namespace graver
