// Binary64 descent of eq. loss with Parallel Extraction (Algorithm 2) on
// gfx950, one thread per start.  This is the bit-reproducible mode: every
// sum runs in ascending index order from 0.0, products and sums are
// separately rounded (this file is compiled with -ffp-contract=off), and
// sqrt / division are the correctly rounded IEEE operations, so iterates
// equal a plain binary64 evaluation of the same formulas.
//
// Also holds the start generator of Algorithm 2: g ~ Uniform(l-u, u-l) by
// Philox4x32-10 (Salmon et al., SC'11) and z = P g.
#include <hip/hip_runtime.h>

#include "graver_internal.h"
#include "pool_device.h"

namespace graver {

// ---- Philox4x32-10 -------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)M0 * c.x;
    uint64_t p1 = (uint64_t)M1 * c.z;
    U4 o;
    o.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    o.y = (uint32_t)p1;
    o.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    o.w = (uint32_t)p0;
    c = o;
  }
  return c;
}

// g[s, j] (stored j-major: g[j * N + s]) for start s = first + local index:
// mode 0: g ~ U(l - u, u - l) (extraction starts); mode 1: x ~ U(l, u)
// (starting points of the initial-solution search).
__global__ void k_box_points(int n, int64_t N, const int64_t* l, const int64_t* u, uint64_t seed,
                             int64_t first, double* g, int mode) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  uint64_t sg = (uint64_t)(first + s);
  for (int p = 0; p < (n + 1) / 2; ++p) {
    U4 c{(uint32_t)p, (uint32_t)sg, (uint32_t)(sg >> 32), 0u};
    U4 w = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int h = 0; h < 2; ++h) {
      int j = 2 * p + h;
      if (j >= n) break;
      uint32_t wa = h ? w.z : w.x, wb = h ? w.w : w.y;
      double U = ((double)(wa >> 5) * 67108864.0 + (double)(wb >> 6)) * (1.0 / 9007199254740992.0);
      double lo = mode ? (double)l[j] : (double)(l[j] - u[j]);
      double width = mode ? (double)(u[j] - l[j]) : (double)(2 * (u[j] - l[j]));
      g[(size_t)j * N + s] = lo + U * width;
    }
  }
}

__global__ void k_zero_nfeas(unsigned int* p) {
  if (threadIdx.x == 0) *p = 0u;
}

// X[s, j] = G[j * N + s] (j-major to row-major).
__global__ void k_transpose_f64(int n, int64_t N, const double* G, double* X) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * n) return;
  int64_t s = t / n;
  int j = (int)(t % n);
  X[t] = G[(size_t)j * N + s];
}

// z[s, i] = sum_j P[i, j] g[s, j], ascending j from 0.0; z row-major N x d.
// A thread forms kProjCols outputs of its start per pass over g, so g
// (column-major n x N, coalesced across threads) is read ceil(d / kProjCols)
// times.
constexpr int kProjCols = 16;
__global__ void k_project(int n, int d, int64_t N, const double* __restrict__ P,
                          const double* __restrict__ g, double* z) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  for (int i0 = 0; i0 < d; i0 += kProjCols) {
    double acc[kProjCols];
#pragma unroll
    for (int t = 0; t < kProjCols; ++t) acc[t] = 0.0;
    for (int j = 0; j < n; ++j) {
      const double gj = g[(size_t)j * N + s];
#pragma unroll
      for (int t = 0; t < kProjCols; ++t)
        if (i0 + t < d) acc[t] = acc[t] + P[(size_t)(i0 + t) * n + j] * gj;
    }
#pragma unroll
    for (int t = 0; t < kProjCols; ++t)
      if (i0 + t < d) z[(size_t)s * d + i0 + t] = acc[t];
  }
}

hipError_t launch_init_box(hipStream_t s, int n, int d, int64_t N, const double* P,
                           const int64_t* l, const int64_t* u, uint64_t seed, int64_t first_start,
                           double* g_scratch, double* z_out) {
  unsigned blocks = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(k_box_points, dim3(blocks), dim3(256), 0, s, n, N, l, u, seed, first_start,
                     g_scratch, 0);
  hipLaunchKernelGGL(k_project, dim3(blocks), dim3(256), 0, s, n, d, N, P, g_scratch, z_out);
  return hipGetLastError();
}

// ---- the descent ---------------------------------------------------------
// State (z, m, v, rprev) is row-major N x d binary64; sign scratch is n x N
// int8; key scratch is N x stride bytes.  Exactness range of the candidate
// map: iterates with |z_j| >= 2^30 yield no candidate.
__global__ void k_descent_fp64(DescentArgs a, double* __restrict__ Z, double* __restrict__ M,
                               double* __restrict__ V, double* __restrict__ RP,
                               int8_t* __restrict__ SG, int8_t* __restrict__ KS, PoolDev pool,
                               unsigned long long* counters) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.N) return;
  const int n = a.n, d = a.d;
  const int64_t N = a.N;
  double* z = Z + (size_t)s * d;
  double* m = M + (size_t)s * d;
  double* v = V + (size_t)s * d;
  double* rp = RP + (size_t)s * d;
  uint64_t* key = reinterpret_cast<uint64_t*>(KS + (size_t)s * pool.stride);
  const int64_t* B = a.B;
  unsigned long long n_emit = 0, n_inbox = 0, n_range = 0;
  const double zrange = 1073741824.0;  // 2^30

  for (int k = 0; k < a.T; ++k) {
    // forward y = B z and its sign
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = 0; j < d; ++j) acc = acc + (double)B[(size_t)i * d + j] * z[j];
      SG[(size_t)i * N + s] = (int8_t)((acc > 0.0) - (acc < 0.0));
    }
    // infinity norm and ties (before the update)
    double mu = 0.0;
    for (int j = 0; j < d; ++j) mu = fmax(mu, fabs(z[j]));
    double cnt = 0.0;
    for (int j = 0; j < d; ++j) cnt = cnt + (fabs(z[j]) == mu ? 1.0 : 0.0);
    const bool bar = (mu > 0.0) && (mu < 1.0);
    const double w = bar ? a.lambda2 / ((mu * mu) * cnt) : 0.0;
    const double bc1 = a.bc[2 * k], bc2 = a.bc[2 * k + 1];
    for (int j = 0; j < d; ++j) {
      double gb = 0.0;
      for (int i = 0; i < n; ++i)
        gb = gb + (double)SG[(size_t)i * N + s] * (double)B[(size_t)i * d + j];
      const double zj = z[j];
      double t = ceil(zj) + floor(zj);
      t = t - 2.0 * zj;
      double g = gb + a.lambda1 * t;
      if (bar && fabs(zj) == mu) g = g - (zj > 0.0 ? w : -w);
      double mj = a.beta1 * m[j] + a.one_minus_b1 * g;
      double vj = a.beta2 * v[j] + a.one_minus_b2 * (g * g);
      m[j] = mj;
      v[j] = vj;
      double mhat = mj / bc1;
      double vhat = vj / bc2;
      z[j] = zj - (a.lr * mhat) / (sqrt(vhat) + a.eps);
    }
    if (!a.collect) continue;
    // rounding, change detection, exact candidate, box test, pool insert
    bool changed = false, inrange = true;
    for (int j = 0; j < d; ++j) {
      double r = rint(z[j]);
      if (!(fabs(z[j]) < zrange)) inrange = false;
      if (r != rp[j]) changed = true;
      rp[j] = r;
    }
    if (!inrange) {
      ++n_range;
      continue;
    }
    if (!changed) continue;
    ++n_emit;
    bool nonzero = false, inbox = true;
    int8_t* kb = reinterpret_cast<int8_t*>(key);
    for (int i = 0; i < n; ++i) {
      int64_t gi = 0;
      for (int j = 0; j < d; ++j) gi += B[(size_t)i * d + j] * (int64_t)rp[j];
      int64_t lim = a.u[i] - a.l[i];
      if (gi > lim || gi < -lim) {
        inbox = false;
        break;
      }
      nonzero |= gi != 0;
      kb[i] = (int8_t)gi;
    }
    if (!inbox || !nonzero) continue;
    for (int i = n; i < pool.stride; ++i) kb[i] = 0;
    ++n_inbox;
    uint64_t h = hash_key_words(key, pool.stride / 8);
    pool_insert(pool, key, h);
  }
  if (n_emit) atomicAdd(&counters[C_EMIT], n_emit);
  if (n_inbox) atomicAdd(&counters[C_INBOX], n_inbox);
  if (n_range) atomicAdd(&counters[C_RANGE], n_range);
}

hipError_t launch_descent_fp64(hipStream_t s, const DescentArgs& a, double* z, double* m, double* v,
                               double* rprev, int8_t* sign_scratch, int8_t* key_scratch,
                               PoolDev pool, unsigned long long* counters) {
  unsigned blocks = (unsigned)((a.N + 63) / 64);
  hipLaunchKernelGGL(k_descent_fp64, dim3(blocks), dim3(64), 0, s, a, z, m, v, rprev, sign_scratch,
                     key_scratch, pool, counters);
  return hipGetLastError();
}

// ---- initial feasible solutions (eq. init_sol) ---------------------------
// One block per start, binary64 with the oracle's operation order.  Each
// iteration: thread i forms res_i = (sum_j A_ij x_j) - b_i (j ascending from
// 0.0); after a barrier thread j forms grad_j = 2 (sum_i A_ij res_i)
// + lam3 ((ceil x_j + floor x_j) - 2 x_j) (i ascending), takes the Adam step
// and projects onto [l, u].  x and res live in LDS; m and v (row-major
// S x n) stay in HBM, one coalesced read and write per iteration.  Finally
// r = round(x) and the exact test A r = b, l <= r <= u.
__global__ void k_init_sol(InitArgs a, double* __restrict__ X, double* __restrict__ M, double* __restrict__ V,
                           int64_t* __restrict__ xr, int32_t* __restrict__ feas, unsigned int* nfeas) {
  extern __shared__ double ish[];
  const int n = a.n, m = a.m;
  const int64_t s = blockIdx.x;
  double* xs = ish;       // n
  double* rs = ish + n;   // m
  double* x = X + (size_t)s * n;
  double* mm = M + (size_t)s * n;
  double* vv = V + (size_t)s * n;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    xs[j] = x[j];
    mm[j] = 0.0;
    vv[j] = 0.0;
  }
  __syncthreads();
  for (int k = 0; k < a.T; ++k) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc = acc + (double)a.A[(size_t)i * n + j] * xs[j];
      rs[i] = acc - (double)a.b[i];
    }
    __syncthreads();
    const double bc1 = a.bc[2 * k], bc2 = a.bc[2 * k + 1];
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      double g = 0.0;
      for (int i = 0; i < m; ++i) g = g + (double)a.A[(size_t)i * n + j] * rs[i];
      const double xj = xs[j];
      double t = ceil(xj) + floor(xj);
      t = t - 2.0 * xj;
      const double grad = 2.0 * g + a.lambda3 * t;
      const double mj = a.beta1 * mm[j] + a.one_minus_b1 * grad;
      const double vj = a.beta2 * vv[j] + a.one_minus_b2 * (grad * grad);
      mm[j] = mj;
      vv[j] = vj;
      const double mhat = mj / bc1;
      const double vhat = vj / bc2;
      double xn = xj - (a.lr * mhat) / (sqrt(vhat) + a.eps);
      xs[j] = fmin(fmax(xn, (double)a.l[j]), (double)a.u[j]);
    }
    __syncthreads();
  }
  int64_t* r = xr + (size_t)s * n;
  int ok = 1;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double xj = xs[j];
    x[j] = xj;
    const double rj = rint(xj);  // |rj| < 2^53 (bounds checked by the host)
    r[j] = (int64_t)rj;
    xs[j] = rj;
    ok &= (rj >= (double)a.l[j] && rj <= (double)a.u[j]) ? 1 : 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    int64_t acc = 0;
    for (int j = 0; j < n; ++j) acc += a.A[(size_t)i * n + j] * (int64_t)xs[j];
    ok &= acc == a.b[i] ? 1 : 0;
  }
  ok = __syncthreads_and(ok);
  if (threadIdx.x == 0) {
    feas[s] = ok;
    if (ok) atomicAdd(nfeas, 1u);
  }
}

hipError_t launch_init_sol(hipStream_t s, const InitArgs& a, const double* x0, uint64_t seed, int64_t first,
                           double* X, double* M, double* V, double* R, double* gscratch, int64_t* xr,
                           int32_t* feas, unsigned int* nfeas) {
  (void)R;
  if (x0) {
    HIP_RET(hipMemcpyAsync(X, x0, (size_t)a.S * a.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    hipLaunchKernelGGL(k_box_points, dim3((unsigned)((a.S + 255) / 256)), dim3(256), 0, s, a.n, a.S, a.l, a.u,
                       seed, first, gscratch, 1);
    hipLaunchKernelGGL(k_transpose_f64, dim3((unsigned)((a.S * a.n + 255) / 256)), dim3(256), 0, s, a.n, a.S,
                       gscratch, X);
  }
  hipLaunchKernelGGL(k_zero_nfeas, dim3(1), dim3(64), 0, s, nfeas);
  const size_t shmem = (size_t)(a.n + a.m) * sizeof(double);
  hipLaunchKernelGGL(k_init_sol, dim3((unsigned)a.S), dim3(128), shmem, s, a, X, M, V, xr, feas, nfeas);
  return hipGetLastError();
}

}  // namespace graver
