// C ABI entry points of the gfx950 library: argument validation, device
// workspace, and the orchestration of the kernels of each hot-path stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "graver_internal.h"

namespace graver {

static thread_local std::string g_last_error = "no error";

graver_status set_error(graver_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

graver_status hip_error(hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return set_error(GRAVER_E_NOMEM, msg);
  return set_error(GRAVER_E_DEVICE, msg);
}

void* ws_get(graver_ctx* ctx, int slot, size_t bytes, graver_status* st) {
  if (bytes == 0) bytes = 256;
  if (ctx->cap[slot] >= bytes) return ctx->buf[slot];
  if (ctx->buf[slot]) {
    hipStreamSynchronize(ctx->stream);
    hipFree(ctx->buf[slot]);
    ctx->buf[slot] = nullptr;
    ctx->cap[slot] = 0;
  }
  size_t want = bytes + bytes / 4;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *st = set_error(GRAVER_E_NOMEM, "device workspace allocation failed");
    return nullptr;
  }
  ctx->buf[slot] = p;
  ctx->cap[slot] = want;
  return p;
}

namespace {

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_error(e_, what); \
  } while (0)

template <class T>
graver_status copy_to_host(graver_ctx* ctx, std::vector<T>& dst, const T* src, size_t count) {
  dst.resize(count);
  if (count == 0) return GRAVER_OK;
  HIP_TRY(hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, ctx->stream),
          "device to host copy");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "stream synchronize");
  return GRAVER_OK;
}

struct EventTimer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit EventTimer(hipStream_t st) : s(st) {
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipEventRecord(a, s);
  }
  double stop_ms() {
    float ms = 0.f;
    hipEventRecord(b, s);
    hipEventSynchronize(b);
    hipEventElapsedTime(&ms, a, b);
    return ms;
  }
  ~EventTimer() {
    hipEventDestroy(a);
    hipEventDestroy(b);
  }
};

graver_status validate_problem(graver_ctx* ctx, const graver_problem* p, bool need_b,
                               std::vector<int64_t>& hl, std::vector<int64_t>& hu) {
  if (!p) return set_error(GRAVER_E_INVALID, "problem is NULL");
  if (p->m < 1 || p->n < 1 || p->n > 4096)
    return set_error(GRAVER_E_INVALID, "need m >= 1 and 1 <= n <= 4096");
  if (!p->A || !p->l || !p->u) return set_error(GRAVER_E_INVALID, "A, l, u must be device pointers");
  if (need_b && !p->b) return set_error(GRAVER_E_INVALID, "b must be a device pointer");
  graver_status st = copy_to_host(ctx, hl, p->l, (size_t)p->n);
  if (st != GRAVER_OK) return st;
  st = copy_to_host(ctx, hu, p->u, (size_t)p->n);
  if (st != GRAVER_OK) return st;
  for (int i = 0; i < p->n; ++i) {
    if (hl[i] > hu[i]) return set_error(GRAVER_E_INVALID, "l <= u violated");
    if (hu[i] - hl[i] > 127) return set_error(GRAVER_E_INVALID, "u - l must be <= 127 (int8 keys)");
  }
  return GRAVER_OK;
}

}  // namespace
}  // namespace graver

using namespace graver;

extern "C" {

const char* graver_last_error(void) { return g_last_error.c_str(); }

const char* graver_status_string(graver_status s) {
  switch (s) {
    case GRAVER_OK: return "ok";
    case GRAVER_E_INVALID: return "invalid argument";
    case GRAVER_E_INFEASIBLE_START: return "infeasible start";
    case GRAVER_E_NOT_KERNEL: return "not in the integer kernel";
    case GRAVER_E_OVERFLOW: return "integer overflow";
    case GRAVER_E_POOL_FULL: return "candidate pool full";
    case GRAVER_E_NOMEM: return "out of device memory";
    case GRAVER_E_DEVICE: return "device error";
    case GRAVER_E_CAPACITY: return "output buffer too small";
  }
  return "unknown status";
}

graver_status graver_ctx_create(graver_ctx** out, int32_t device) {
  if (!out) return set_error(GRAVER_E_INVALID, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (device < 0 || device >= count) return set_error(GRAVER_E_INVALID, "no such device");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(GRAVER_E_DEVICE, std::string("library is built for gfx950, device is ") +
                                          prop.gcnArchName);
  graver_ctx* c = new graver_ctx();
  c->device = device;
  *out = c;
  return GRAVER_OK;
}

void graver_ctx_destroy(graver_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  for (int i = 0; i < graver_ctx::kSlots; ++i)
    if (ctx->buf[i]) hipFree(ctx->buf[i]);
  solve_cache_free(ctx);
  delete ctx;
}

graver_status graver_ctx_set_stream(graver_ctx* ctx, void* hip_stream) {
  if (!ctx) return set_error(GRAVER_E_INVALID, "ctx is NULL");
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return GRAVER_OK;
}

graver_status graver_kernel_basis(int32_t m, int32_t n, const int64_t* A, int32_t lll,
                                  int64_t* B_out, int32_t* d_out, double* P_out) {
  if (m < 1 || n < 1 || n > 4096 || !A || !B_out || !d_out)
    return set_error(GRAVER_E_INVALID, "graver_kernel_basis: bad arguments");
  return kernel_basis_host(m, n, A, lll, B_out, d_out, P_out);
}

graver_status graver_extract(graver_ctx* ctx, const graver_problem* prob,
                             const graver_extract_params* prm, graver_state* state,
                             int8_t* keys_out, int64_t keys_cap, int64_t* count_out,
                             graver_extract_stats* stats) {
  if (!ctx || !prm || !count_out) return set_error(GRAVER_E_INVALID, "NULL argument");
  hipSetDevice(ctx->device);
  std::vector<int64_t> hl, hu;
  graver_status st = validate_problem(ctx, prob, false, hl, hu);
  if (st != GRAVER_OK) return st;
  const int n = prob->n, d = prob->d, m = prob->m;
  const int64_t N = prm->n_starts;
  const int T = prm->iters;
  if (d < 1 || d > n || !prob->B) return set_error(GRAVER_E_INVALID, "need a basis B with 1 <= d <= n");
  if (N < 1 || N > (int64_t)1 << 30 || T < 0) return set_error(GRAVER_E_INVALID, "bad n_starts / iters");
  if (prm->precision != GRAVER_FP64 && prm->precision != GRAVER_FP32 && prm->precision != GRAVER_BF16)
    return set_error(GRAVER_E_INVALID, "unknown precision");
  if (prm->polish_iters < 0) return set_error(GRAVER_E_INVALID, "polish_iters < 0");
  if (prm->init_mode == 0 && !prob->P) return set_error(GRAVER_E_INVALID, "init_mode 0 needs P");
  if (prm->init_mode == 1 && (!state || !state->z))
    return set_error(GRAVER_E_INVALID, "init_mode 1 needs state->z");
  if (prm->init_mode != 0 && prm->init_mode != 1) return set_error(GRAVER_E_INVALID, "bad init_mode");
  if (prm->collect && (prm->pool_capacity < 1 || prm->pool_capacity > ((int64_t)1 << 31)))
    return set_error(GRAVER_E_INVALID, "pool_capacity must be in [1, 2^31]");
  if (prm->t0 < 0 || !(prm->beta1 >= 0 && prm->beta1 < 1) || !(prm->beta2 >= 0 && prm->beta2 < 1))
    return set_error(GRAVER_E_INVALID, "bad Adam parameters");
  if (prm->collect && (keys_cap < 0 || (keys_cap > 0 && !keys_out)))
    return set_error(GRAVER_E_INVALID, "bad output buffer");

  // B must be a kernel basis: A B = 0 exactly.  A's nonzeros (CSR) serve
  // the exact check of the collected candidates.
  std::vector<int32_t> csr_rp((size_t)m + 1, 0), csr_col;
  std::vector<int64_t> csr_val;
  {
    std::vector<int64_t> hA, hB;
    if ((st = copy_to_host(ctx, hA, prob->A, (size_t)m * n)) != GRAVER_OK) return st;
    for (int i = 0; i < m; ++i) {
      for (int j = 0; j < n; ++j) {
        const int64_t av = hA[(size_t)i * n + j];
        if (av <= -((int64_t)1 << 31) || av >= ((int64_t)1 << 31))
          return set_error(GRAVER_E_OVERFLOW, "|A_ij| must be below 2^31");
        if (av != 0) {
          csr_col.push_back(j);
          csr_val.push_back(av);
        }
      }
      csr_rp[i + 1] = (int32_t)csr_col.size();
    }
    if ((st = copy_to_host(ctx, hB, prob->B, (size_t)n * d)) != GRAVER_OK) return st;
    for (int i = 0; i < m; ++i)
      for (int c = 0; c < d; ++c) {
        __int128 s = 0;
        for (int j = 0; j < n; ++j) s += (__int128)hA[(size_t)i * n + j] * hB[(size_t)j * d + c];
        if (s != 0) return set_error(GRAVER_E_NOT_KERNEL, "A B != 0: B is not a kernel basis");
      }
  }

  hipStream_t s = ctx->stream;
  graver_extract_stats stt{};
  stt.start_iterations = N * (int64_t)T;

  // Bias corrections 1 - beta^t for t = t0+1 .. t0+T (host libm pow).
  std::vector<double> hbc(2 * (size_t)std::max(T, 1));
  for (int k = 0; k < T; ++k) {
    double t = (double)prm->t0 + k + 1;
    hbc[2 * k] = 1.0 - std::pow(prm->beta1, t);
    hbc[2 * k + 1] = 1.0 - std::pow(prm->beta2, t);
  }
  double* dbc = (double*)ws_get(ctx, WS_BC, hbc.size() * sizeof(double), &st);
  if (!dbc) return st;
  HIP_TRY(hipMemcpyAsync(dbc, hbc.data(), hbc.size() * sizeof(double), hipMemcpyHostToDevice, s),
          "copy bias corrections");

  const size_t nd = (size_t)N * d;
  double* z = (double*)ws_get(ctx, WS_Z, nd * sizeof(double), &st);
  if (!z) return st;
  double* mm = (double*)ws_get(ctx, WS_M, nd * sizeof(double), &st);
  if (!mm) return st;
  double* vv = (double*)ws_get(ctx, WS_V, nd * sizeof(double), &st);
  if (!vv) return st;

  // Pool.
  PoolDev pool{};
  pool.n = n;
  pool.stride = key_stride(n);
  uint64_t cap = prm->collect ? (uint64_t)prm->pool_capacity : 1;
  uint64_t tsize = 1024;
  while (tsize < 2 * cap) tsize <<= 1;
  pool.cap = (uint32_t)std::min<uint64_t>(cap, 0xFFFFFFF0u);
  pool.tmask = tsize - 1;
  pool.keys = (int8_t*)ws_get(ctx, WS_POOL_KEYS, (size_t)pool.cap * pool.stride, &st);
  if (!pool.keys) return st;
  pool.table = (uint64_t*)ws_get(ctx, WS_POOL_TABLE, tsize * sizeof(uint64_t), &st);
  if (!pool.table) return st;
  pool.count = (uint32_t*)ws_get(ctx, WS_POOL_COUNT, 64, &st);
  if (!pool.count) return st;
  auto* counters = (unsigned long long*)ws_get(ctx, WS_COUNTERS, 64, &st);
  if (!counters) return st;

  {
    EventTimer tm(s);
    if (prm->init_mode == 0) {
      double* g0 = (double*)ws_get(ctx, WS_G0, (size_t)N * n * sizeof(double), &st);
      if (!g0) return st;
      HIP_TRY(launch_init_box(s, n, d, N, prob->P, prob->l, prob->u, prm->seed, prm->first_start, g0, z),
              "init kernels");
      HIP_TRY(hipMemsetAsync(mm, 0, nd * sizeof(double), s), "clear m");
      HIP_TRY(hipMemsetAsync(vv, 0, nd * sizeof(double), s), "clear v");
    } else {
      HIP_TRY(hipMemcpyAsync(z, state->z, nd * sizeof(double), hipMemcpyDeviceToDevice, s), "copy z");
      if (state->m)
        HIP_TRY(hipMemcpyAsync(mm, state->m, nd * sizeof(double), hipMemcpyDeviceToDevice, s), "copy m");
      else
        HIP_TRY(hipMemsetAsync(mm, 0, nd * sizeof(double), s), "clear m");
      if (state->v)
        HIP_TRY(hipMemcpyAsync(vv, state->v, nd * sizeof(double), hipMemcpyDeviceToDevice, s), "copy v");
      else
        HIP_TRY(hipMemsetAsync(vv, 0, nd * sizeof(double), s), "clear v");
    }
    HIP_TRY(launch_pool_clear(s, pool), "pool clear");
    HIP_TRY(hipMemsetAsync(counters, 0, 64, s), "clear counters");
    stt.ms_init = tm.stop_ms();
  }

  DescentArgs da{};
  da.n = n;
  da.d = d;
  da.N = (int32_t)N;
  da.T = T;
  da.B = prob->B;
  da.l = prob->l;
  da.u = prob->u;
  da.lr = prm->lr;
  da.beta1 = prm->beta1;
  da.beta2 = prm->beta2;
  da.eps = prm->eps;
  da.lambda1 = prm->lambda1;
  da.lambda2 = prm->lambda2;
  da.one_minus_b1 = 1.0 - prm->beta1;
  da.one_minus_b2 = 1.0 - prm->beta2;
  da.bc = dbc;
  da.collect = prm->collect;
  da.bf16_iters = prm->precision == GRAVER_BF16 ? std::max(0, T - prm->polish_iters) : 0;
  da.lim_uniform = (int32_t)(hu[0] - hl[0]);
  for (int i = 1; i < n; ++i)
    if (hu[i] - hl[i] != hu[0] - hl[0]) da.lim_uniform = -1;

  {
    if (prm->precision == GRAVER_FP64) {
      double* rp = (double*)ws_get(ctx, WS_RPREV, nd * sizeof(double), &st);
      if (!rp) return st;
      int8_t* sg = (int8_t*)ws_get(ctx, WS_SIGN, (size_t)N * n, &st);
      if (!sg) return st;
      int8_t* ks = (int8_t*)ws_get(ctx, WS_KEYSCRATCH, (size_t)N * pool.stride, &st);
      if (!ks) return st;
      HIP_TRY(hipMemsetAsync(rp, 0xFF, nd * sizeof(double), s), "rprev = NaN");
      EventTimer tm(s);
      if (T > 0) HIP_TRY(launch_descent_fp64(s, da, z, mm, vv, rp, sg, ks, pool, counters), "descent fp64");
      stt.ms_descent = tm.stop_ms();
    } else {
      const bool small = descent_f32_supported(n, d);
      if (!small && !descent_big_supported(n, d))
        return set_error(GRAVER_E_INVALID, "the MFMA descent supports n <= 1024 and d <= 1024");
      // |B_ij| <= 256 makes every bf16 operand exact; row l1 norms bound the
      // exact range of the candidate map.
      int* rowl1 = (int*)ws_get(ctx, WS_MISC, 64, &st);
      if (!rowl1) return st;
      float* Bp = nullptr;
      float* BTp = nullptr;
      unsigned char* img = nullptr;
      if (small) {
        Bp = (float*)ws_get(ctx, WS_MF_B, f32_pack_floats(n, d) * sizeof(float), &st);
        if (!Bp) return st;
        BTp = (float*)ws_get(ctx, WS_MF_BT, f32_pack_floats(n, d) * sizeof(float), &st);
        if (!BTp) return st;
        HIP_TRY(launch_f32_pack(s, n, d, prob->B, Bp, BTp, rowl1), "pack basis");
      } else {
        img = (unsigned char*)ws_get(ctx, WS_MF_B, big_image_bytes(n, d), &st);
        if (!img) return st;
        HIP_TRY(launch_big_pack(s, n, d, prob->B, img), "pack basis");
        HIP_TRY(launch_rowl1(s, n, d, prob->B, rowl1), "row norms");
      }
      int hrow[2] = {0, 0};
      HIP_TRY(hipMemcpyAsync(hrow, rowl1, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "row l1");
      HIP_TRY(hipStreamSynchronize(s), "sync");
      if (hrow[1] > 256)
        return set_error(GRAVER_E_INVALID, "the MFMA descent needs |B_ij| <= 256 (exact bf16 operands)");
      // large bases: candidates B r with |r_j| <= 256 must stay exact in fp32
      if (!small && (int64_t)hrow[0] * 256 >= (int64_t)1 << 24)
        return set_error(GRAVER_E_INVALID, "the MFMA descent needs every row l1 norm of B below 65536");
      const float zrange = (float)std::min(1073741824.0, std::floor(16777216.0 / std::max(hrow[0], 1)));
      const int DBlay = small ? (d + 15) / 16 : descent_big_dbp(d);
      const size_t sfloats = small ? f32_state_floats(n, d, N) : big_state_floats(d, N);
      float* fstate = (float*)ws_get(ctx, WS_MF_STATE, sfloats * sizeof(float), &st);
      if (!fstate) return st;
      int8_t* kscr = nullptr;
      if (!small) {
        kscr = (int8_t*)ws_get(ctx, WS_KEYSCRATCH, ((size_t)N + 64) * pool.stride, &st);
        if (!kscr) return st;
      }
      HIP_TRY(launch_state_io_db(s, d, DBlay, N, fstate, z, mm, vv, 1), "state in");
      LogDev lg{};
      lg.stride = pool.stride;
      lg.cap = prm->collect ? pool.cap : 0u;
      lg.rows = (int8_t*)ws_get(ctx, WS_LOG, (size_t)std::max<uint32_t>(lg.cap, 1) * pool.stride, &st);
      if (!lg.rows) return st;
      lg.count = (uint32_t*)ws_get(ctx, WS_LOG_COUNT, 64, &st);
      if (!lg.count) return st;
      const size_t sbytes = sfloats * sizeof(float);
      float* fbak = (float*)ws_get(ctx, WS_MF_BAK, sbytes, &st);
      if (!fbak) return st;
      unsigned long long* cbak = (unsigned long long*)ws_get(ctx, WS_MISC2, 64, &st);
      if (!cbak) return st;
      da.log = lg;
      const int bf16_total = da.bf16_iters;
      // The candidate log holds pool_capacity rows per launch.  A launch whose
      // log overflows is rolled back (state and counters) and replayed in two
      // halves, so every candidate reaches the pool.
      int done = 0, chunk = T;
      while (done < T) {
        int c = std::min(chunk, T - done);
        // a launch of the large-basis kernel uses a single forward form
        if (!small && done < bf16_total) c = std::min(c, bf16_total - done);
        DescentArgs dc = da;
        dc.T = c;
        dc.bc = dbc + 2 * (size_t)done;
        dc.bf16_iters = std::max(0, std::min(c, bf16_total - done));
        HIP_TRY(hipMemcpyAsync(fbak, fstate, sbytes, hipMemcpyDeviceToDevice, s), "state backup");
        HIP_TRY(hipMemcpyAsync(cbak, counters, 64, hipMemcpyDeviceToDevice, s), "counter backup");
        HIP_TRY(hipMemsetAsync(lg.count, 0, 64, s), "clear log count");
        EventTimer tm(s);
        if (small)
          HIP_TRY(launch_descent_f32(s, dc, Bp, BTp, fstate, pool, counters, zrange), "descent mfma");
        else
          HIP_TRY(launch_descent_big(s, dc, img, fstate, kscr, counters), "descent mfma (large)");
        stt.ms_descent += tm.stop_ms();
        uint32_t lflag[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(lflag, lg.count, sizeof(lflag), hipMemcpyDeviceToHost, s), "log flag");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        if (lflag[1]) {
          if (c == 1) return set_error(GRAVER_E_POOL_FULL, "one iteration yields more candidates than pool_capacity");
          HIP_TRY(hipMemcpyAsync(fstate, fbak, sbytes, hipMemcpyDeviceToDevice, s), "state rollback");
          HIP_TRY(hipMemcpyAsync(counters, cbak, 64, hipMemcpyDeviceToDevice, s), "counter rollback");
          chunk = std::max(1, c / 2);
          continue;
        }
        if (prm->collect) {
          HIP_TRY(launch_log_insert(s, lg, pool), "log insert");
          // stop as soon as the pool cannot hold the distinct candidates
          uint32_t pf[3] = {0, 0, 0};
          HIP_TRY(hipMemcpyAsync(pf, pool.count, sizeof(pf), hipMemcpyDeviceToHost, s), "pool flags");
          HIP_TRY(hipStreamSynchronize(s), "sync");
          if (pf[1]) return set_error(GRAVER_E_POOL_FULL, "more distinct candidates than pool_capacity");
          if (pf[2]) return set_error(GRAVER_E_POOL_FULL, "hash probe limit reached");
        }
        done += c;
      }
      HIP_TRY(launch_state_io_db(s, d, DBlay, N, fstate, z, mm, vv, 0), "state out");

    }
  }
  HIP_TRY(hipGetLastError(), "descent launch");

  // Counters and pool status.
  unsigned long long hc[C_NCOUNTERS] = {};
  uint32_t hp[3] = {};
  HIP_TRY(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, s), "counters");
  HIP_TRY(hipMemcpyAsync(hp, pool.count, sizeof(hp), hipMemcpyDeviceToHost, s), "pool count");
  HIP_TRY(hipStreamSynchronize(s), "descent");
  stt.emit_events = (int64_t)hc[C_EMIT];
  stt.inbox_events = (int64_t)hc[C_INBOX];
  stt.out_of_range = (int64_t)hc[C_RANGE];

  if (state) {
    if (state->z && state->z != z)
      HIP_TRY(hipMemcpyAsync(state->z, z, nd * sizeof(double), hipMemcpyDeviceToDevice, s), "z out");
    if (state->m) HIP_TRY(hipMemcpyAsync(state->m, mm, nd * sizeof(double), hipMemcpyDeviceToDevice, s), "m out");
    if (state->v) HIP_TRY(hipMemcpyAsync(state->v, vv, nd * sizeof(double), hipMemcpyDeviceToDevice, s), "v out");
  }

  *count_out = 0;
  if (!prm->collect) {
    if (stats) *stats = stt;
    HIP_TRY(hipStreamSynchronize(s), "sync");
    return GRAVER_OK;
  }
  if (hp[1]) return set_error(GRAVER_E_POOL_FULL, "more distinct candidates than pool_capacity");
  if (hp[2]) return set_error(GRAVER_E_POOL_FULL, "hash probe limit reached");
  uint32_t count = std::min<uint32_t>(hp[0], pool.cap);
  stt.unique = count;

  {
    EventTimer tm(s);
    unsigned int* bad = (unsigned int*)ws_get(ctx, WS_FLAGS, 64, &st);
    if (!bad) return st;
    const size_t nnz = csr_col.size();
    const size_t ints = ((size_t)m + 1 + nnz + 1) / 2 * 2;  // int32 part, padded to 8 bytes
    auto* csr = (int32_t*)ws_get(ctx, WS_V_CSR, ints * 4 + std::max<size_t>(nnz, 1) * 8, &st);
    if (!csr) return st;
    HIP_TRY(hipMemcpyAsync(csr, csr_rp.data(), csr_rp.size() * 4, hipMemcpyHostToDevice, s), "csr");
    if (nnz) {
      HIP_TRY(hipMemcpyAsync(csr + m + 1, csr_col.data(), nnz * 4, hipMemcpyHostToDevice, s), "csr");
      HIP_TRY(hipMemcpyAsync(csr + ints, csr_val.data(), nnz * 8, hipMemcpyHostToDevice, s), "csr");
    }
    HIP_TRY(launch_verify(s, pool, count, m, csr, csr + m + 1, reinterpret_cast<const int64_t*>(csr + ints), bad),
            "verify");
    unsigned int hbad = 0;
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s), "verify flag");
    stt.ms_verify = tm.stop_ms();
    if (hbad) return set_error(GRAVER_E_NOT_KERNEL, "a collected candidate fails A g = 0");
    stt.verified = count;
  }
  if ((int64_t)count > keys_cap) {
    if (stats) *stats = stt;
    *count_out = count;
    return set_error(GRAVER_E_CAPACITY, "keys_cap too small for the collected set");
  }
  {
    EventTimer tm(s);
    uint32_t p2 = 1024;
    while (p2 < count) p2 <<= 1;
    uint32_t* idx = (uint32_t*)ws_get(ctx, WS_SORT_IDX, (size_t)p2 * sizeof(uint32_t), &st);
    if (!idx) return st;
    HIP_TRY(launch_sort_keys(s, pool.keys, pool.stride, n, count, idx, nullptr, 0, nullptr), "sort");
    HIP_TRY(launch_gather_keys(s, pool.keys, pool.stride, n, idx, count, keys_out, n), "gather");
    stt.ms_sort = tm.stop_ms();
  }
  *count_out = count;
  if (stats) *stats = stt;
  return GRAVER_OK;
}

graver_status graver_filter(graver_ctx* ctx, int32_t n, const int8_t* keys_in, int64_t count_in,
                            int8_t* keys_out, int64_t keys_cap, int64_t* count_out) {
  if (!ctx || !count_out) return set_error(GRAVER_E_INVALID, "NULL argument");
  if (n < 1 || n > 4096 || count_in < 0 || count_in > ((int64_t)1 << 31) - 1024)
    return set_error(GRAVER_E_INVALID, "bad n or count");
  if (count_in > 0 && !keys_in) return set_error(GRAVER_E_INVALID, "keys_in is NULL");
  if (keys_cap < 0 || (keys_cap > 0 && !keys_out)) return set_error(GRAVER_E_INVALID, "bad output buffer");
  hipSetDevice(ctx->device);
  graver_status st = GRAVER_OK;
  hipError_t e = launch_filter(ctx->stream, ctx, n, keys_in, count_in, keys_out, keys_cap, count_out, &st);
  if (st != GRAVER_OK) return st;
  if (e != hipSuccess) return hip_error(e, "filter");
  return GRAVER_OK;
}

graver_status graver_augment(graver_ctx* ctx, const graver_problem* prob, const graver_objective* f,
                             const int8_t* dirs, int64_t K, int32_t S, const int64_t* x_starts,
                             const graver_augment_params* params, int64_t* x_out, double* f_out,
                             int64_t* steps_out, int32_t* best_out) {
  if (!ctx || !f || !params) return set_error(GRAVER_E_INVALID, "NULL argument");
  hipSetDevice(ctx->device);
  std::vector<int64_t> hl, hu;
  graver_status st = validate_problem(ctx, prob, true, hl, hu);
  if (st != GRAVER_OK) return st;
  if (K < 0 || K > ((int64_t)1 << 30) || (K > 0 && !dirs)) return set_error(GRAVER_E_INVALID, "bad dirs");
  if (S < 1 || !x_starts || !x_out || !f_out || !steps_out)
    return set_error(GRAVER_E_INVALID, "need S >= 1 and device start/output buffers");
  if (params->max_steps < 0) return set_error(GRAVER_E_INVALID, "max_steps < 0");
  AugArgs a{};
  a.n = prob->n;
  a.m = prob->m;
  a.S = S;
  a.K = (int32_t)K;
  a.A = prob->A;
  a.b = prob->b;
  a.l = prob->l;
  a.u = prob->u;
  a.kind = f->kind;
  a.degree = f->degree;
  a.Q = f->Q;
  a.c = f->c;
  a.coef = f->coef;
  a.dirs = dirs;
  a.max_steps = params->max_steps;
  if (f->kind == GRAVER_F_QUADRATIC) {
    if (!f->Q || !f->c) return set_error(GRAVER_E_INVALID, "quadratic objective needs Q and c");
    std::vector<double> hQ;
    if ((st = copy_to_host(ctx, hQ, f->Q, (size_t)a.n * a.n)) != GRAVER_OK) return st;
    for (int i = 0; i < a.n; ++i)
      for (int j = 0; j < i; ++j)
        if (hQ[(size_t)i * a.n + j] != hQ[(size_t)j * a.n + i])
          return set_error(GRAVER_E_INVALID, "Q must be symmetric");
  } else if (f->kind == GRAVER_F_SEPARABLE_POLY) {
    if (!f->coef || f->degree < 0 || f->degree > 8)
      return set_error(GRAVER_E_INVALID, "separable polynomial needs coef and 0 <= degree <= 8");
  } else {
    return set_error(GRAVER_E_INVALID, "unknown objective kind");
  }
  return run_augment(ctx, a, x_starts, x_out, f_out, steps_out, best_out);
}

graver_status graver_init_solutions(graver_ctx* ctx, const graver_problem* prob,
                                    const graver_init_params* prm, const double* x0,
                                    double* x_out, int64_t* sol_out, int32_t* feasible_out,
                                    int64_t* n_feasible) {
  if (!ctx || !prm || !sol_out || !feasible_out) return set_error(GRAVER_E_INVALID, "NULL argument");
  hipSetDevice(ctx->device);
  if (!prob) return set_error(GRAVER_E_INVALID, "problem is NULL");
  if (prob->m < 1 || prob->n < 1 || prob->n > 4096)
    return set_error(GRAVER_E_INVALID, "need m >= 1 and 1 <= n <= 4096");
  if (!prob->A || !prob->b || !prob->l || !prob->u)
    return set_error(GRAVER_E_INVALID, "A, b, l, u must be device pointers");
  const int m = prob->m, n = prob->n;
  const int64_t S = prm->n_starts;
  if (S < 1 || S > (int64_t)1 << 26 || prm->iters < 0)
    return set_error(GRAVER_E_INVALID, "bad n_starts / iters");
  if (prm->init_mode != 0 && prm->init_mode != 1) return set_error(GRAVER_E_INVALID, "bad init_mode");
  if (prm->init_mode == 1 && !x0) return set_error(GRAVER_E_INVALID, "init_mode 1 needs x0");
  if (!(prm->beta1 >= 0 && prm->beta1 < 1) || !(prm->beta2 >= 0 && prm->beta2 < 1))
    return set_error(GRAVER_E_INVALID, "bad Adam parameters");
  graver_status st = GRAVER_OK;
  std::vector<int64_t> hA, hb, hl, hu;
  if ((st = copy_to_host(ctx, hA, prob->A, (size_t)m * n)) != GRAVER_OK) return st;
  if ((st = copy_to_host(ctx, hb, prob->b, (size_t)m)) != GRAVER_OK) return st;
  if ((st = copy_to_host(ctx, hl, prob->l, (size_t)n)) != GRAVER_OK) return st;
  if ((st = copy_to_host(ctx, hu, prob->u, (size_t)n)) != GRAVER_OK) return st;
  const double lim = 9007199254740992.0;  // 2^53
  for (int j = 0; j < n; ++j) {
    if (hl[j] > hu[j]) return set_error(GRAVER_E_INVALID, "l <= u violated");
    if (std::fabs((double)hl[j]) >= lim || std::fabs((double)hu[j]) >= lim)
      return set_error(GRAVER_E_OVERFLOW, "bounds reach 2^53");
  }
  for (int i = 0; i < m; ++i) {
    double row = 0.0;
    for (int j = 0; j < n; ++j)
      row += std::fabs((double)hA[(size_t)i * n + j]) *
             std::max(std::fabs((double)hl[j]), std::fabs((double)hu[j]));
    if (row >= lim || std::fabs((double)hb[i]) >= lim)
      return set_error(GRAVER_E_OVERFLOW, "sum_j |A_ij| max(|l_j|, |u_j|) or |b_i| reaches 2^53");
  }

  hipStream_t s = ctx->stream;
  const int T = prm->iters;
  std::vector<double> hbc(2 * (size_t)std::max(T, 1));
  for (int k = 0; k < T; ++k) {
    double t = (double)k + 1;
    hbc[2 * k] = 1.0 - std::pow(prm->beta1, t);
    hbc[2 * k + 1] = 1.0 - std::pow(prm->beta2, t);
  }
  double* dbc = (double*)ws_get(ctx, WS_BC, hbc.size() * sizeof(double), &st);
  if (!dbc) return st;
  HIP_TRY(hipMemcpyAsync(dbc, hbc.data(), hbc.size() * sizeof(double), hipMemcpyHostToDevice, s),
          "copy bias corrections");
  const size_t sn = (size_t)S * n;
  double* X = (double*)ws_get(ctx, WS_I_X, sn * sizeof(double), &st);
  if (!X) return st;
  double* M = (double*)ws_get(ctx, WS_I_M, sn * sizeof(double), &st);
  if (!M) return st;
  double* V = (double*)ws_get(ctx, WS_I_V, sn * sizeof(double), &st);
  if (!V) return st;
  double* G = prm->init_mode == 0 ? (double*)ws_get(ctx, WS_I_G, sn * sizeof(double), &st) : nullptr;
  if (prm->init_mode == 0 && !G) return st;
  auto* cnt = (unsigned int*)ws_get(ctx, WS_FLAGS, 64, &st);
  if (!cnt) return st;

  InitArgs a{};
  a.m = m;
  a.n = n;
  a.T = T;
  a.S = S;
  a.A = prob->A;
  a.b = prob->b;
  a.l = prob->l;
  a.u = prob->u;
  a.lr = prm->lr;
  a.beta1 = prm->beta1;
  a.beta2 = prm->beta2;
  a.eps = prm->eps;
  a.lambda3 = prm->lambda3;
  a.one_minus_b1 = 1.0 - prm->beta1;
  a.one_minus_b2 = 1.0 - prm->beta2;
  a.bc = dbc;
  HIP_TRY(launch_init_sol(s, a, prm->init_mode == 1 ? x0 : nullptr, prm->seed, prm->first_start, X, M, V, nullptr, G,
                          sol_out, feasible_out, cnt),
          "init_sol kernels");
  if (x_out) HIP_TRY(hipMemcpyAsync(x_out, X, sn * sizeof(double), hipMemcpyDeviceToDevice, s), "copy x_out");
  unsigned int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s), "copy feasible count");
  HIP_TRY(hipStreamSynchronize(s), "stream synchronize");
  if (n_feasible) *n_feasible = (int64_t)h;
  return GRAVER_OK;
}

}  // extern "C"
