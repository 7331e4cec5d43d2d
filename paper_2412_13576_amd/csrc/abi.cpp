// C ABI entry points of the gfx950 library: argument validation, device
// workspace, and the orchestration of the kernels of each hot-path stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "graver_internal.h"

namespace graver {

static thread_local std::string g_last_error = "no error";

// Device scratch of graver_augment_noalloc: one array per GPU, held until
// the process ends.  Host code never passes `scratch` itself to a kernel (in
// host code the name is a host-side stand-in); it uses the device address
// that hipGetSymbolAddress returns for the current device, looked up once
// per device when the first context on that device is created.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Device address of this device's scratch array (device must be current).
static graver_status scratch_lookup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return GRAVER_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
  g_scratch_dev[device] = ptr;
  return GRAVER_OK;
}

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

void* ws_get(graver_ctx* ctx, Ws& w, int slot, size_t bytes, graver_status* st) {
  if (bytes == 0) bytes = 256;
  if (w.cap[slot] >= bytes) return w.buf[slot];
  if (w.buf[slot]) {
    (void)hipStreamSynchronize(ctx->stream);  // errors surface on the next checked call
    (void)hipFree(w.buf[slot]);
    w.buf[slot] = nullptr;
    w.cap[slot] = 0;
  }
  size_t want = bytes + bytes / 4;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *st = set_error(GRAVER_E_NOMEM, "device workspace allocation failed");
    return nullptr;
  }
  w.buf[slot] = p;
  w.cap[slot] = want;
  return p;
}

void* ws_get(graver_ctx* ctx, int slot, size_t bytes, graver_status* st) {
  return ws_get(ctx, ctx->ws, slot, bytes, st);
}

void ws_free(Ws& w) {
  for (int i = 0; i < Ws::kSlots; ++i)
    if (w.buf[i]) {
      (void)hipFree(w.buf[i]);
      w.buf[i] = nullptr;
      w.cap[i] = 0;
    }
}

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
    case GRAVER_E_CANCELLED: return "cancelled";
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
  if (device >= kMaxDevices) return set_error(GRAVER_E_INVALID, "device ordinal beyond the library's limit");
  graver_status sst = scratch_lookup(device);
  if (sst != GRAVER_OK) return sst;
  graver_ctx* c = new graver_ctx();
  c->device = device;
  *out = c;
  return GRAVER_OK;
}

void graver_ctx_destroy(graver_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);  // teardown: nothing to report to
  (void)hipStreamSynchronize(ctx->stream);
  ws_free(ctx->ws);
  for (Ws* w : ctx->batch_ws) {
    ws_free(*w);
    delete w;
  }
  solve_cache_free(ctx);
  tile_cache_free(ctx);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  delete ctx;
}

graver_status graver_ctx_trim(graver_ctx* ctx) {
  if (!ctx) return set_error(GRAVER_E_INVALID, "ctx is NULL");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "stream synchronize");
  ws_free(ctx->ws);
  for (Ws* w : ctx->batch_ws) ws_free(*w);
  return GRAVER_OK;
}

graver_status graver_ctx_set_stream(graver_ctx* ctx, void* hip_stream) {
  if (!ctx) return set_error(GRAVER_E_INVALID, "ctx is NULL");
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return GRAVER_OK;
}

graver_status graver_kernel_basis(int32_t m, int32_t n, const int64_t* A, int32_t lll,
                                  int64_t* B_out, int32_t* d_out, double* P_out) {
  Phase ph("graver_kernel_basis (host)");
  if (m < 1 || n < 1 || n > 4096 || !A || !B_out || !d_out)
    return set_error(GRAVER_E_INVALID, "graver_kernel_basis: bad arguments");
  return kernel_basis_host(m, n, A, lll, B_out, d_out, P_out);
}

graver_status graver_filter(graver_ctx* ctx, int32_t n, const int8_t* keys_in, int64_t count_in,
                            int8_t* keys_out, int64_t keys_cap, int64_t* count_out) {
  if (!ctx || !count_out) return set_error(GRAVER_E_INVALID, "NULL argument");
  if (n < 1 || n > 4096 || count_in < 0 || count_in > ((int64_t)1 << 31) - 1024)
    return set_error(GRAVER_E_INVALID, "bad n or count");
  if (count_in > 0 && !keys_in) return set_error(GRAVER_E_INVALID, "keys_in is NULL");
  if (keys_cap < 0 || (keys_cap > 0 && !keys_out)) return set_error(GRAVER_E_INVALID, "bad output buffer");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  Phase ph("graver_filter (dedup, minimality)");
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
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  Phase ph("graver_augment (Algorithm 1)");
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
  int w = 1;
  for (int i = 0; i < a.n; ++i) w = (int)std::max<int64_t>(w, hu[i] - hl[i] + 1);
  return run_augment(ctx, a, w, x_starts, x_out, f_out, steps_out, best_out);
}

graver_status graver_augment_noalloc(graver_ctx* ctx, const graver_problem* prob, const graver_objective* f,
                                     const int8_t* dirs, int64_t K, int32_t S, const int64_t* x_starts,
                                     const graver_augment_params* params, int64_t* x_out, double* f_out,
                                     int64_t* steps_out, int32_t* best_out) {
  if (!ctx || !f || !params || !prob) return set_error(GRAVER_E_INVALID, "NULL argument");
  if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_scratch_dev[ctx->device])
    return set_error(GRAVER_E_INVALID, "no scratch address for this context's device");
  if (prob->m < 1 || prob->n < 1 || prob->n > 4096)
    return set_error(GRAVER_E_INVALID, "need m >= 1 and 1 <= n <= 4096");
  if (!prob->A || !prob->b || !prob->l || !prob->u)
    return set_error(GRAVER_E_INVALID, "A, b, l, u must be device pointers");
  if (K < 0 || K > ((int64_t)1 << 30) || (K > 0 && !dirs)) return set_error(GRAVER_E_INVALID, "bad dirs");
  if (S < 1 || !x_starts || !x_out || !f_out || !steps_out)
    return set_error(GRAVER_E_INVALID, "need S >= 1 and device start/output buffers");
  if (params->max_steps < 0) return set_error(GRAVER_E_INVALID, "max_steps < 0");
  if (f->kind == GRAVER_F_QUADRATIC) {
    if (!f->Q || !f->c) return set_error(GRAVER_E_INVALID, "quadratic objective needs Q and c");
  } else if (f->kind == GRAVER_F_SEPARABLE_POLY) {
    if (!f->coef || f->degree < 0 || f->degree > 8)
      return set_error(GRAVER_E_INVALID, "separable polynomial needs coef and 0 <= degree <= 8");
  } else {
    return set_error(GRAVER_E_INVALID, "unknown objective kind");
  }
  // every width u - l is at most 127 (checked below), so a value table of
  // width 128 serves any box
  const int w = 128;
  const size_t need = aug_work_bytes(prob->n, S, K, w);
  if (need > kNoallocScratchBytes)
    return set_error(GRAVER_E_CAPACITY, "graver_augment_noalloc: the call needs " + std::to_string(need) +
                                            " bytes of scratch, the limit is " +
                                            std::to_string(kNoallocScratchBytes));
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  hipStream_t s = ctx->stream;
  AugWork wk = aug_work_carve(g_scratch_dev[ctx->device], prob->n, S, K, w);
  // bounds and symmetry of Q checked on the device (no host copy of the instance)
  unsigned int* vflag = wk.flags + 8;
  HIP_TRY(launch_aug_validate(s, prob->n, prob->l, prob->u, f->kind == GRAVER_F_QUADRATIC ? f->Q : nullptr, vflag),
          "validate");
  unsigned int hv = 0;
  HIP_TRY(hipMemcpyAsync(&hv, vflag, sizeof(hv), hipMemcpyDeviceToHost, s), "validate");
  HIP_TRY(hipStreamSynchronize(s), "validate");
  if (hv & 1u) return set_error(GRAVER_E_INVALID, "l <= u violated");
  if (hv & 2u) return set_error(GRAVER_E_INVALID, "u - l must be <= 127 (int8 keys)");
  if (hv & 4u) return set_error(GRAVER_E_INVALID, "Q must be symmetric");
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
  return run_augment_ws(s, a, w, wk, x_starts, x_out, f_out, steps_out, best_out);
}

graver_status graver_init_solutions(graver_ctx* ctx, const graver_problem* prob,
                                    const graver_init_params* prm, const double* x0,
                                    double* x_out, int64_t* sol_out, int32_t* feasible_out,
                                    int64_t* n_feasible) {
  if (!ctx || !prm || !sol_out || !feasible_out) return set_error(GRAVER_E_INVALID, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  Phase ph("graver_init_solutions (eq. init_sol)");
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
