// MAPE end to end (Section 3.3): kernel basis, Parallel Extraction
// (Algorithm 2), minimality filter, initial feasible solutions (eq.
// init_sol) and augmentation (Algorithm 1) from every feasible initial
// solution, with a per-context cache of bases and filtered sets keyed by
// (A, u - l): the extracted set depends on A and on the box widths only, so
// instances that share them reuse one extraction.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <vector>

#include "graver_internal.h"

namespace graver {

namespace {

struct SolveEntry {
  int m = 0, n = 0, d = 0;
  std::vector<int64_t> A, width;
  int64_t* B = nullptr;  // device n x d
  double* P = nullptr;   // device d x n
  int8_t* F = nullptr;   // device K x n
  int64_t K = 0;
};

struct SolveCache {
  std::vector<SolveEntry> entries;
};

SolveCache* cache_of(graver_ctx* ctx) {
  if (!ctx->solve_cache) ctx->solve_cache = new SolveCache();
  return static_cast<SolveCache*>(ctx->solve_cache);
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

template <class T>
graver_status to_host(graver_ctx* ctx, std::vector<T>& dst, const T* src, size_t count) {
  dst.resize(count);
  if (count == 0) return GRAVER_OK;
  hipError_t e = hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? GRAVER_OK : hip_error(e, "device to host copy");
}

template <class T>
graver_status dev_alloc(T** p, size_t count) {
  *p = nullptr;
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(GRAVER_E_NOMEM, "device allocation failed");
  }
  return GRAVER_OK;
}

}  // namespace

void solve_cache_free(graver_ctx* ctx) {
  if (!ctx->solve_cache) return;
  auto* c = static_cast<SolveCache*>(ctx->solve_cache);
  for (auto& e : c->entries) {
    (void)hipFree(e.B);
    (void)hipFree(e.P);
    (void)hipFree(e.F);
  }
  delete c;
  ctx->solve_cache = nullptr;
}

}  // namespace graver

using namespace graver;

extern "C" graver_status graver_solve(graver_ctx* ctx, const graver_problem* prob, const graver_objective* f,
                                      const graver_solve_params* prm, int64_t* x_best, double* f_best,
                                      graver_solve_stats* stats) {
  if (!ctx || !prob || !f || !prm || !x_best || !f_best) return set_error(GRAVER_E_INVALID, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  Phase ph("graver_solve (MAPE)");
  if (prob->m < 1 || prob->n < 1 || prob->n > 4096)
    return set_error(GRAVER_E_INVALID, "need m >= 1 and 1 <= n <= 4096");
  if (!prob->A || !prob->b || !prob->l || !prob->u)
    return set_error(GRAVER_E_INVALID, "A, b, l, u must be device pointers");
  if (!prm->extract.collect) return set_error(GRAVER_E_INVALID, "extract.collect must be 1");
  if (prm->max_steps < 0) return set_error(GRAVER_E_INVALID, "max_steps < 0");
  const int m = prob->m, n = prob->n;
  hipStream_t s = ctx->stream;
  graver_solve_stats st{};
  graver_status rc = GRAVER_OK;
  std::vector<int64_t> hA, hl, hu;
  if ((rc = to_host(ctx, hA, prob->A, (size_t)m * n)) != GRAVER_OK) return rc;
  if ((rc = to_host(ctx, hl, prob->l, (size_t)n)) != GRAVER_OK) return rc;
  if ((rc = to_host(ctx, hu, prob->u, (size_t)n)) != GRAVER_OK) return rc;
  std::vector<int64_t> width(n);
  for (int j = 0; j < n; ++j) width[j] = hu[j] - hl[j];

  // ---- basis, extraction and filter (or the cached set) --------------------
  SolveEntry* hit = nullptr;
  if (prm->reuse) {
    for (auto& e : cache_of(ctx)->entries)
      if (e.m == m && e.n == n && e.A == hA && e.width == width) hit = &e;
  }
  const int8_t* F = nullptr;
  int64_t K = 0;
  int d = 0;
  if (hit) {
    F = hit->F;
    K = hit->K;
    d = hit->d;
    st.reused = 1;
  } else {
    auto t0 = std::chrono::steady_clock::now();
    graver_problem p = *prob;
    if (!p.B) {
      std::vector<int64_t> hB((size_t)n * n);
      std::vector<double> hP((size_t)n * n);
      int32_t dd = 0;
      if ((rc = kernel_basis_host(m, n, hA.data(), prm->lll, hB.data(), &dd, hP.data())) != GRAVER_OK) return rc;
      if (dd < 1) return set_error(GRAVER_E_INVALID, "A has full column rank: the kernel is {0}");
      auto* dB = (int64_t*)ws_get(ctx, WS_S_B, (size_t)n * dd * sizeof(int64_t), &rc);
      if (!dB) return rc;
      auto* dP = (double*)ws_get(ctx, WS_S_P, (size_t)dd * n * sizeof(double), &rc);
      if (!dP) return rc;
      HIP_TRY(hipMemcpyAsync(dB, hB.data(), (size_t)n * dd * sizeof(int64_t), hipMemcpyHostToDevice, s), "basis");
      HIP_TRY(hipMemcpyAsync(dP, hP.data(), (size_t)dd * n * sizeof(double), hipMemcpyHostToDevice, s), "basis");
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_error(e, "copy basis");
      p.B = dB;
      p.P = dP;
      p.d = dd;
    }
    d = p.d;
    st.ms_basis = ms_since(t0);

    t0 = std::chrono::steady_clock::now();
    const int64_t cap = prm->extract.pool_capacity;
    auto* keys = (int8_t*)ws_get(ctx, WS_S_KEYS, (size_t)std::max<int64_t>(cap, 1) * n, &rc);
    if (!keys) return rc;
    int64_t count = 0;
    graver_extract_stats es{};
    graver_extract_params ex = prm->extract;
    ex.any_order = 1;  // the filter sorts
    if ((rc = graver_extract(ctx, &p, &ex, nullptr, keys, cap, &count, &es)) != GRAVER_OK) return rc;
    st.unique = count;
    st.ms_extract = ms_since(t0);

    t0 = std::chrono::steady_clock::now();
    auto* Fbuf = (int8_t*)ws_get(ctx, WS_S_F, (size_t)std::max<int64_t>(count, 1) * n, &rc);
    if (!Fbuf) return rc;
    if ((rc = graver_filter(ctx, n, count ? keys : nullptr, count, Fbuf, count, &K)) != GRAVER_OK) return rc;
    F = Fbuf;
    st.ms_filter = ms_since(t0);

    if (prm->reuse) {
      SolveEntry e;
      e.m = m;
      e.n = n;
      e.d = d;
      e.A = hA;
      e.width = width;
      e.K = K;
      if ((rc = dev_alloc(&e.B, (size_t)n * d)) != GRAVER_OK) return rc;
      if ((rc = dev_alloc(&e.P, p.P ? (size_t)d * n : 1)) != GRAVER_OK) return rc;
      if ((rc = dev_alloc(&e.F, (size_t)K * n)) != GRAVER_OK) return rc;
      HIP_TRY(hipMemcpyAsync(e.B, p.B, (size_t)n * d * sizeof(int64_t), hipMemcpyDeviceToDevice, s), "cache");
      if (p.P) HIP_TRY(hipMemcpyAsync(e.P, p.P, (size_t)d * n * sizeof(double), hipMemcpyDeviceToDevice, s), "cache");
      if (K) HIP_TRY(hipMemcpyAsync(e.F, F, (size_t)K * n, hipMemcpyDeviceToDevice, s), "cache");
      hipError_t err = hipStreamSynchronize(s);
      if (err != hipSuccess) return hip_error(err, "cache copy");
      cache_of(ctx)->entries.push_back(std::move(e));
      F = cache_of(ctx)->entries.back().F;
    }
  }
  st.d = d;
  st.filtered = K;

  // ---- initial feasible solutions -----------------------------------------
  auto t0 = std::chrono::steady_clock::now();
  const int64_t S = prm->init.n_starts;
  auto* sol = (int64_t*)ws_get(ctx, WS_S_SOL, (size_t)std::max<int64_t>(S, 1) * n * sizeof(int64_t), &rc);
  if (!sol) return rc;
  auto* feas = (int32_t*)ws_get(ctx, WS_S_FEAS, (size_t)std::max<int64_t>(S, 1) * sizeof(int32_t), &rc);
  if (!feas) return rc;
  int64_t nfeas = 0;
  if ((rc = graver_init_solutions(ctx, prob, &prm->init, nullptr, nullptr, sol, feas, &nfeas)) != GRAVER_OK)
    return rc;
  st.feasible_starts = nfeas;
  const int64_t nx = prm->x_starts ? prm->n_x_starts : 0;
  if (nx < 0) return set_error(GRAVER_E_INVALID, "n_x_starts < 0");
  if (nfeas + nx == 0) {
    if (stats) *stats = st;
    return set_error(GRAVER_E_INFEASIBLE_START, "no initial solution is feasible and no x_starts were given");
  }
  if (nfeas + nx > (1 << 30)) return set_error(GRAVER_E_INVALID, "too many starts");
  std::vector<int32_t> hf;
  if ((rc = to_host(ctx, hf, feas, (size_t)S)) != GRAVER_OK) return rc;
  std::vector<int32_t> idx;
  idx.reserve((size_t)nfeas);
  for (int64_t r = 0; r < S; ++r)
    if (hf[r]) idx.push_back((int32_t)r);
  auto* didx = (int32_t*)ws_get(ctx, WS_S_IDX, std::max<size_t>(idx.size(), 1) * sizeof(int32_t), &rc);
  if (!didx) return rc;
  const int32_t S2 = (int32_t)(idx.size() + nx);
  auto* starts = (int64_t*)ws_get(ctx, WS_S_STARTS, (size_t)S2 * n * sizeof(int64_t), &rc);
  if (!starts) return rc;
  HIP_TRY(hipMemcpyAsync(didx, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice, s), "start indices");
  hipError_t e = launch_gather_rows_i64(s, sol, n, didx, (int64_t)idx.size(), starts);
  if (e != hipSuccess) return hip_error(e, "gather starts");
  if (nx)
    HIP_TRY(hipMemcpyAsync(starts + idx.size() * n, prm->x_starts, (size_t)nx * n * sizeof(int64_t),
                           hipMemcpyDeviceToDevice, s),
            "caller starts");
  st.ms_init = ms_since(t0);

  // ---- augmentation and best-of -------------------------------------------
  t0 = std::chrono::steady_clock::now();
  auto* xo = (int64_t*)ws_get(ctx, WS_S_X, (size_t)S2 * n * sizeof(int64_t), &rc);
  if (!xo) return rc;
  auto* fo = (double*)ws_get(ctx, WS_S_FV, (size_t)S2 * sizeof(double), &rc);
  if (!fo) return rc;
  auto* so = (int64_t*)ws_get(ctx, WS_S_STEPS, (size_t)S2 * sizeof(int64_t), &rc);
  if (!so) return rc;
  graver_augment_params ap{prm->max_steps};
  int32_t best = -1;
  if ((rc = graver_augment(ctx, prob, f, K ? F : nullptr, K, S2, starts, &ap, xo, fo, so, &best)) != GRAVER_OK)
    return rc;
  std::vector<int64_t> hs;
  if ((rc = to_host(ctx, hs, so, (size_t)S2)) != GRAVER_OK) return rc;
  for (int64_t v : hs) st.augment_steps += v;
  double fb = 0.0;
  HIP_TRY(hipMemcpyAsync(&fb, fo + best, sizeof(double), hipMemcpyDeviceToHost, s), "best-of");
  HIP_TRY(hipMemcpyAsync(x_best, xo + (size_t)best * n, (size_t)n * sizeof(int64_t), hipMemcpyDeviceToDevice, s),
          "best-of");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "best-of");
  *f_best = fb;
  st.best_start = best;
  st.ms_augment = ms_since(t0);
  if (stats) *stats = st;
  return GRAVER_OK;
}
