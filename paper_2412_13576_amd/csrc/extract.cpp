// Parallel Extraction (Algorithm 2) on the device: one instance per call
// (graver_extract) or many instances per call (graver_extract_batch).
//
// An instance is a job with its own device workspace: setup (validation,
// bias corrections, pool, starts, packed basis, wave-native state), the
// descent (one or more launches), and finish (state out, A g = 0, sort,
// output).  In a batch every large-basis job of the same tile shape and
// forward form runs in one grid; the descent phase of the batch (state
// backups, grids, log inserts) can be captured in a HIP graph.  A job whose
// candidate log overflowed in the batched grid is rolled back and replayed
// alone (in halves, as in a single call); the rows its log did hold are
// already in its pool, and the replay emits them again, so the set is the
// same.  The tile shape of a basis size is either the fixed table or, with
// autotuning, the fastest of the candidate shapes in a short timed trial,
// kept in the context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "descent_sparse.h"
#include "graver_internal.h"

namespace graver {

namespace {

enum JobKind { JOB_FP64, JOB_SMALL, JOB_BIG, JOB_SPARSE };

struct Job {
  // call arguments
  const graver_problem* prob = nullptr;
  const graver_extract_params* prm = nullptr;
  graver_state* state = nullptr;
  int8_t* keys_out = nullptr;
  int64_t keys_cap = 0;
  Ws* ws = nullptr;
  // sizes and host copies
  int n = 0, d = 0, m = 0, T = 0;
  int64_t N = 0;
  std::vector<int64_t> hl, hu;
  std::vector<int32_t> csr_rp, csr_col;
  std::vector<int64_t> csr_val;
  graver_extract_stats stt{};
  // device buffers
  double* dbc = nullptr;
  float* dstepf = nullptr;
  double *z = nullptr, *mm = nullptr, *vv = nullptr;
  size_t nd = 0;
  PoolDev pool{};
  unsigned long long* counters = nullptr;
  DescentArgs da{};
  JobKind kind = JOB_FP64;
  BigShape sh{};
  float *Bp = nullptr, *BTp = nullptr;
  unsigned char* img = nullptr;
  float* fstate = nullptr;
  int8_t* kscr = nullptr;
  LogDev lg{};
  float* fbak = nullptr;
  unsigned long long* cbak = nullptr;
  float zrange = 0.f;
  int DBlay = 0;
  size_t sbytes = 0;
  int bf16_total = 0;
  int done = 0;
  SparseImage sp;  // row lists of B (sparse form)
  uint32_t *sp_ent = nullptr, *sp_row = nullptr;
};

struct TileCache {
  std::map<std::pair<int, int>, BigShape> best;  // (row blocks, column blocks) -> shape
};

void* W(graver_ctx* ctx, Job& j, int slot, size_t bytes, graver_status* st) {
  return ws_get(ctx, *j.ws, slot, bytes, st);
}

// A's nonzeros as CSR (host), for the exact check A g = 0 (condition C1).
graver_status build_csr(const std::vector<int64_t>& hA, int m, int n, std::vector<int32_t>& rp,
                        std::vector<int32_t>& col, std::vector<int64_t>& val) {
  rp.assign((size_t)m + 1, 0);
  col.clear();
  val.clear();
  for (int i = 0; i < m; ++i) {
    for (int c = 0; c < n; ++c) {
      const int64_t av = hA[(size_t)i * n + c];
      if (av <= -((int64_t)1 << 31) || av >= ((int64_t)1 << 31))
        return set_error(GRAVER_E_OVERFLOW, "|A_ij| must be below 2^31");
      if (av != 0) {
        col.push_back(c);
        val.push_back(av);
      }
    }
    rp[i + 1] = (int32_t)col.size();
  }
  return GRAVER_OK;
}

// Condition C1 on the device for `count` key rows of `stride` bytes: the
// number of rows with A g != 0 goes to *nbad (host).
graver_status verify_rows(graver_ctx* ctx, Ws& w, int m, const std::vector<int32_t>& rp,
                          const std::vector<int32_t>& col, const std::vector<int64_t>& val, const int8_t* keys,
                          int n, int stride, uint32_t count, unsigned int* nbad) {
  hipStream_t s = ctx->stream;
  graver_status st = GRAVER_OK;
  unsigned int* bad = (unsigned int*)ws_get(ctx, w, WS_FLAGS, 64, &st);
  if (!bad) return st;
  const size_t nnz = col.size();
  const size_t ints = ((size_t)m + 1 + nnz + 1) / 2 * 2;  // int32 part, padded to 8 bytes
  auto* csr = (int32_t*)ws_get(ctx, w, WS_V_CSR, ints * 4 + std::max<size_t>(nnz, 1) * 8, &st);
  if (!csr) return st;
  HIP_TRY(hipMemcpyAsync(csr, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, s), "csr");
  if (nnz) {
    HIP_TRY(hipMemcpyAsync(csr + m + 1, col.data(), nnz * 4, hipMemcpyHostToDevice, s), "csr");
    HIP_TRY(hipMemcpyAsync(csr + ints, val.data(), nnz * 8, hipMemcpyHostToDevice, s), "csr");
  }
  PoolDev view{};
  view.keys = const_cast<int8_t*>(keys);
  view.n = n;
  view.stride = stride;
  HIP_TRY(launch_verify(s, view, count, m, (int64_t)nnz, csr, csr + m + 1, reinterpret_cast<const int64_t*>(csr + ints),
                        bad),
          "verify");
  unsigned int hbad = 0;
  HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s), "verify flag");
  HIP_TRY(hipStreamSynchronize(s), "verify");  // rp, col, val are the caller's host vectors
  *nbad = hbad;
  return GRAVER_OK;
}

// Validation, host checks and the device setup of one job (everything
// before its first descent launch).  force_big routes an MFMA job through
// the large-basis kernel even when the small one would fit; autotune picks
// the large kernel's tile shape by a timed trial.
graver_status job_setup(graver_ctx* ctx, Job& j, bool force_big, bool autotune) {
  const graver_problem* prob = j.prob;
  const graver_extract_params* prm = j.prm;
  graver_status st = validate_problem(ctx, prob, false, j.hl, j.hu);
  if (st != GRAVER_OK) return st;
  const int n = prob->n, d = prob->d, m = prob->m;
  const int64_t N = prm->n_starts;
  const int T = prm->iters;
  j.n = n;
  j.d = d;
  j.m = m;
  j.N = N;
  j.T = T;
  if (d < 1 || d > n || !prob->B) return set_error(GRAVER_E_INVALID, "need a basis B with 1 <= d <= n");
  if (N < 1 || N > (int64_t)1 << 30 || T < 0) return set_error(GRAVER_E_INVALID, "bad n_starts / iters");
  if (prm->precision != GRAVER_FP64 && prm->precision != GRAVER_FP32 && prm->precision != GRAVER_BF16)
    return set_error(GRAVER_E_INVALID, "unknown precision");
  if (prm->polish_iters < 0) return set_error(GRAVER_E_INVALID, "polish_iters < 0");
  if (prm->init_mode == 0 && !prob->P) return set_error(GRAVER_E_INVALID, "init_mode 0 needs P");
  if (prm->init_mode == 1 && (!j.state || !j.state->z))
    return set_error(GRAVER_E_INVALID, "init_mode 1 needs state->z");
  if (prm->init_mode != 0 && prm->init_mode != 1) return set_error(GRAVER_E_INVALID, "bad init_mode");
  if (prm->collect && (prm->pool_capacity < 1 || prm->pool_capacity > ((int64_t)1 << 31)))
    return set_error(GRAVER_E_INVALID, "pool_capacity must be in [1, 2^31]");
  if (prm->t0 < 0 || !(prm->beta1 >= 0 && prm->beta1 < 1) || !(prm->beta2 >= 0 && prm->beta2 < 1))
    return set_error(GRAVER_E_INVALID, "bad Adam parameters");
  if (prm->collect && (j.keys_cap < 0 || (j.keys_cap > 0 && !j.keys_out)))
    return set_error(GRAVER_E_INVALID, "bad output buffer");

  // B must be a kernel basis: A B = 0 exactly.  A's nonzeros (CSR) serve
  // the exact check of the collected candidates.
  {
    std::vector<int64_t> hA, hB;
    if ((st = copy_to_host(ctx, hA, prob->A, (size_t)m * n)) != GRAVER_OK) return st;
    if ((st = build_csr(hA, m, n, j.csr_rp, j.csr_col, j.csr_val)) != GRAVER_OK) return st;
    if ((st = copy_to_host(ctx, hB, prob->B, (size_t)n * d)) != GRAVER_OK) return st;
    for (int i = 0; i < m; ++i)
      for (int c = 0; c < d; ++c) {
        __int128 s = 0;
        for (int k = 0; k < n; ++k) s += (__int128)hA[(size_t)i * n + k] * hB[(size_t)k * d + c];
        if (s != 0) return set_error(GRAVER_E_NOT_KERNEL, "A B != 0: B is not a kernel basis");
      }
    if (prm->form < GRAVER_FORM_AUTO || prm->form > GRAVER_FORM_SPARSE) return set_error(GRAVER_E_INVALID, "unknown form");
    if (prm->form == GRAVER_FORM_SPARSE && prm->precision != GRAVER_FP32)
      return set_error(GRAVER_E_INVALID, "the sparse form runs binary32 descents only");
    if (prm->precision == GRAVER_FP32 && prm->form != GRAVER_FORM_DENSE &&
        !sparse_image_build(n, d, hB.data(), j.hl.data(), j.hu.data(), j.sp) && prm->form == GRAVER_FORM_SPARSE)
      return set_error(GRAVER_E_INVALID, "B does not fit the sparse form (n, d <= 1024, at most 128 row-list entries per lane)");
  }

  hipStream_t s = ctx->stream;
  j.stt = graver_extract_stats{};
  j.stt.start_iterations = N * (int64_t)T;

  // Bias corrections 1 - beta^t for t = t0+1 .. t0+T (host libm pow).
  std::vector<double> hbc(2 * (size_t)std::max(T, 1));
  for (int k = 0; k < T; ++k) {
    double t = (double)prm->t0 + k + 1;
    hbc[2 * k] = 1.0 - std::pow(prm->beta1, t);
    hbc[2 * k + 1] = 1.0 - std::pow(prm->beta2, t);
  }
  j.dbc = (double*)W(ctx, j, WS_BC, hbc.size() * sizeof(double), &st);
  if (!j.dbc) return st;
  HIP_TRY(hipMemcpyAsync(j.dbc, hbc.data(), hbc.size() * sizeof(double), hipMemcpyHostToDevice, s),
          "copy bias corrections");
  // the binary32 kernels' per-iteration factors, from the same divisions
  // they would otherwise do in binary64 every iteration
  std::vector<float> hsf(hbc.size());
  for (size_t k = 0; k + 1 < hbc.size(); k += 2) {
    hsf[k] = (float)(prm->lr / hbc[k]);
    hsf[k + 1] = (float)(1.0 / hbc[k + 1]);
  }
  j.dstepf = (float*)W(ctx, j, WS_STEPF, hsf.size() * sizeof(float), &st);
  if (!j.dstepf) return st;
  HIP_TRY(hipMemcpyAsync(j.dstepf, hsf.data(), hsf.size() * sizeof(float), hipMemcpyHostToDevice, s),
          "copy step factors");
  HIP_TRY(hipStreamSynchronize(s), "sync");  // hbc and hsf are locals

  j.nd = (size_t)N * d;
  j.z = (double*)W(ctx, j, WS_Z, j.nd * sizeof(double), &st);
  if (!j.z) return st;
  j.mm = (double*)W(ctx, j, WS_M, j.nd * sizeof(double), &st);
  if (!j.mm) return st;
  j.vv = (double*)W(ctx, j, WS_V, j.nd * sizeof(double), &st);
  if (!j.vv) return st;

  // Pool.
  PoolDev& pool = j.pool;
  pool.n = n;
  pool.stride = key_stride(n);
  uint64_t cap = prm->collect ? (uint64_t)prm->pool_capacity : 1;
  uint64_t tsize = 1024;
  while (tsize < 2 * cap) tsize <<= 1;
  pool.cap = (uint32_t)std::min<uint64_t>(cap, 0xFFFFFFF0u);
  pool.tmask = tsize - 1;
  pool.keys = (int8_t*)W(ctx, j, WS_POOL_KEYS, (size_t)pool.cap * pool.stride, &st);
  if (!pool.keys) return st;
  pool.table = (uint64_t*)W(ctx, j, WS_POOL_TABLE, tsize * sizeof(uint64_t), &st);
  if (!pool.table) return st;
  pool.count = (uint32_t*)W(ctx, j, WS_POOL_COUNT, 64, &st);
  if (!pool.count) return st;
  j.counters = (unsigned long long*)W(ctx, j, WS_COUNTERS, 64, &st);
  if (!j.counters) return st;

  {
    EventTimer tm(s);
    if (prm->init_mode == 0) {
      double* g0 = (double*)W(ctx, j, WS_G0, (size_t)N * n * sizeof(double), &st);
      if (!g0) return st;
      HIP_TRY(launch_init_box(s, n, d, N, prob->P, prob->l, prob->u, prm->seed, prm->first_start, g0, j.z),
              "init kernels");
      HIP_TRY(hipMemsetAsync(j.mm, 0, j.nd * sizeof(double), s), "clear m");
      HIP_TRY(hipMemsetAsync(j.vv, 0, j.nd * sizeof(double), s), "clear v");
    } else {
      HIP_TRY(hipMemcpyAsync(j.z, j.state->z, j.nd * sizeof(double), hipMemcpyDeviceToDevice, s), "copy z");
      if (j.state->m)
        HIP_TRY(hipMemcpyAsync(j.mm, j.state->m, j.nd * sizeof(double), hipMemcpyDeviceToDevice, s), "copy m");
      else
        HIP_TRY(hipMemsetAsync(j.mm, 0, j.nd * sizeof(double), s), "clear m");
      if (j.state->v)
        HIP_TRY(hipMemcpyAsync(j.vv, j.state->v, j.nd * sizeof(double), hipMemcpyDeviceToDevice, s), "copy v");
      else
        HIP_TRY(hipMemsetAsync(j.vv, 0, j.nd * sizeof(double), s), "clear v");
    }
    HIP_TRY(launch_pool_clear(s, pool), "pool clear");
    HIP_TRY(hipMemsetAsync(j.counters, 0, 64, s), "clear counters");
    j.stt.ms_init = tm.stop_ms();
  }

  DescentArgs& da = j.da;
  da = DescentArgs{};
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
  da.bc = j.dbc;
  da.stepf = j.dstepf;
  da.collect = prm->collect;
  da.bf16_iters = prm->precision == GRAVER_BF16 ? std::max(0, T - prm->polish_iters) : 0;
  da.lim_uniform = (int32_t)(j.hu[0] - j.hl[0]);
  for (int i = 1; i < n; ++i)
    if (j.hu[i] - j.hl[i] != j.hu[0] - j.hl[0]) da.lim_uniform = -1;
  j.bf16_total = da.bf16_iters;
  j.done = 0;

  if (prm->precision == GRAVER_FP64) {
    j.kind = JOB_FP64;
    return GRAVER_OK;
  }

  const bool small0 = !force_big && descent_f32_supported(n, d);
  // the sparse form: asked for, or automatic where the large kernel would run
  const bool sparse = j.sp.nc > 0 && (prm->form == GRAVER_FORM_SPARSE || (!small0 && sparse_form_pays(j.sp, n, d)));
  const bool small = small0 && !sparse;
  if (!small && !sparse && !descent_big_supported(n, d))
    return set_error(GRAVER_E_INVALID, "the MFMA descent supports n <= 1024 and d <= 1024");
  j.kind = sparse ? JOB_SPARSE : (small ? JOB_SMALL : JOB_BIG);
  // |B_ij| <= 256 makes every bf16 operand exact; row l1 norms bound the
  // exact range of the candidate map.
  int* rowl1 = (int*)W(ctx, j, WS_MISC, 64, &st);
  if (!rowl1) return st;
  if (small) {
    j.Bp = (float*)W(ctx, j, WS_MF_B, f32_pack_floats(n, d) * sizeof(float), &st);
    if (!j.Bp) return st;
    j.BTp = (float*)W(ctx, j, WS_MF_BT, f32_pack_floats(n, d) * sizeof(float), &st);
    if (!j.BTp) return st;
    HIP_TRY(launch_f32_pack(s, n, d, prob->B, j.Bp, j.BTp, rowl1), "pack basis");
  } else {
    HIP_TRY(launch_rowl1(s, n, d, prob->B, rowl1), "row norms");
  }
  int hrow[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(hrow, rowl1, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "row l1");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  if (hrow[1] > 256)
    return set_error(GRAVER_E_INVALID, "the MFMA descent needs |B_ij| <= 256 (exact bf16 operands)");
  // large bases: candidates B r with |r_j| <= 256 must stay exact in fp32
  if (j.kind == JOB_BIG && (int64_t)hrow[0] * 256 >= (int64_t)1 << 24)
    return set_error(GRAVER_E_INVALID, "the MFMA descent needs every row l1 norm of B below 65536");
  j.zrange = (float)std::min(1073741824.0, std::floor(16777216.0 / std::max(hrow[0], 1)));
  if (sparse) {
    j.sp_ent = (uint32_t*)W(ctx, j, WS_MF_B, j.sp.ent.size() * sizeof(uint32_t), &st);
    if (!j.sp_ent) return st;
    j.sp_row = (uint32_t*)W(ctx, j, WS_MF_BT, j.sp.row.size() * sizeof(uint32_t), &st);
    if (!j.sp_row) return st;
    HIP_TRY(hipMemcpyAsync(j.sp_ent, j.sp.ent.data(), j.sp.ent.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s),
            "row lists");
    HIP_TRY(hipMemcpyAsync(j.sp_row, j.sp.row.data(), j.sp.row.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s),
            "row slots");
    j.stt.row_entries = j.sp.ew;
    j.stt.row_slots = j.sp.nc;
  } else if (!small) {
    j.kscr = (int8_t*)W(ctx, j, WS_KEYSCRATCH, ((size_t)N + 64) * pool.stride, &st);
    if (!j.kscr) return st;
    j.sh = big_shape_default(d);
    if (autotune) {
      auto* tc = static_cast<TileCache*>(ctx->tile_cache);
      if (!tc) ctx->tile_cache = tc = new TileCache();
      const std::pair<int, int> key((n + 15) / 16, (d + 15) / 16);
      auto it = tc->best.find(key);
      if (it != tc->best.end()) {
        j.sh = it->second;
      } else {
        BigShape cand[8];
        const int nc = big_shape_candidates(d, cand, 8);
        size_t img_max = 0, st_max = 0;
        for (int c = 0; c < nc; ++c) {
          img_max = std::max(img_max, big_image_bytes(n, cand[c]));
          st_max = std::max(st_max, big_state_floats(cand[c], N));
        }
        auto* timg = (unsigned char*)W(ctx, j, WS_MF_B, img_max, &st);
        if (!timg) return st;
        auto* tstate = (float*)W(ctx, j, WS_MF_BAK, st_max * sizeof(float), &st);
        if (!tstate) return st;
        auto* tdesc = W(ctx, j, WS_BIG_DESC, 4096, &st);
        if (!tdesc) return st;
        double best_ms = 0.0;
        for (int c = 0; c < nc; ++c) {
          HIP_TRY(launch_big_pack(s, n, d, cand[c], prob->B, timg), "pack basis");
          HIP_TRY(launch_fill_u64(s, reinterpret_cast<uint64_t*>(tstate), big_state_floats(cand[c], N) / 2, 0),
                  "trial state");
          BigJob bj{};
          bj.a = da;
          bj.a.T = std::min(T, 8);
          bj.a.collect = 0;
          bj.a.bf16_iters = j.bf16_total > 0 ? bj.a.T : 0;
          bj.img = timg;
          bj.state = tstate;
          bj.scratch = j.kscr;
          bj.counters = j.counters;
          std::vector<unsigned char> hd;
          int64_t blocks = 0;
          int nbmax = 1;
          big_desc_prepare(cand[c], &bj, 1, hd, &blocks, &nbmax);
          HIP_TRY(hipMemcpyAsync(tdesc, hd.data(), hd.size(), hipMemcpyHostToDevice, s), "trial table");
          double ms = 0.0;
          for (int rep = 0; rep < 2; ++rep) {  // the first launch loads the code object
            EventTimer tm(s);
            HIP_TRY(launch_descent_big(s, cand[c], bj.a.bf16_iters > 0, tdesc, 1, blocks, nbmax), "trial");
            ms = tm.stop_ms();
          }
          if (c == 0 || ms < best_ms) {
            best_ms = ms;
            j.sh = cand[c];
          }
        }
        HIP_TRY(hipMemsetAsync(j.counters, 0, 64, s), "clear counters");
        tc->best[key] = j.sh;
      }
    }
    j.img = (unsigned char*)W(ctx, j, WS_MF_B, big_image_bytes(n, j.sh), &st);
    if (!j.img) return st;
    HIP_TRY(launch_big_pack(s, n, d, j.sh, prob->B, j.img), "pack basis");
  }
  j.DBlay = small || sparse ? (d + 15) / 16 : j.sh.cs * j.sh.dbpw;
  if (j.kind == JOB_BIG) {
    j.stt.tile_slices = j.sh.cs;
    j.stt.tile_blocks = j.sh.dbpw;
  }
  const size_t sfloats = small || sparse ? f32_state_floats(n, d, N) : big_state_floats(j.sh, N);
  j.fstate = (float*)W(ctx, j, WS_MF_STATE, sfloats * sizeof(float), &st);
  if (!j.fstate) return st;
  HIP_TRY(launch_state_io_db(s, d, j.DBlay, N, j.fstate, j.z, j.mm, j.vv, 1), "state in");
  LogDev& lg = j.lg;
  lg.stride = pool.stride;
  lg.cap = prm->collect ? pool.cap : 0u;
  lg.rows = (int8_t*)W(ctx, j, WS_LOG, (size_t)std::max<uint32_t>(lg.cap, 1) * pool.stride, &st);
  if (!lg.rows) return st;
  lg.count = (uint32_t*)W(ctx, j, WS_LOG_COUNT, 64, &st);
  if (!lg.count) return st;
  j.sbytes = sfloats * sizeof(float);
  j.fbak = (float*)W(ctx, j, WS_MF_BAK, j.sbytes, &st);
  if (!j.fbak) return st;
  j.cbak = (unsigned long long*)W(ctx, j, WS_MISC2, 64, &st);
  if (!j.cbak) return st;
  da.log = lg;
  return GRAVER_OK;
}

// Descent of one job from j.done up to iteration `until`, alone on the
// stream.  The candidate log holds pool_capacity rows per launch; a launch
// whose log overflows is rolled back (state and counters) and replayed in
// two halves, so every candidate reaches the pool.
graver_status job_descend(graver_ctx* ctx, Job& j, int until) {
  hipStream_t s = ctx->stream;
  graver_status st = GRAVER_OK;
  if (j.kind == JOB_FP64) {
    if (j.done >= until) return GRAVER_OK;
    double* rp = (double*)W(ctx, j, WS_RPREV, j.nd * sizeof(double), &st);
    if (!rp) return st;
    int8_t* sg = (int8_t*)W(ctx, j, WS_SIGN, (size_t)j.N * j.n, &st);
    if (!sg) return st;
    int8_t* ks = (int8_t*)W(ctx, j, WS_KEYSCRATCH, (size_t)j.N * j.pool.stride, &st);
    if (!ks) return st;
    HIP_TRY(hipMemsetAsync(rp, 0xFF, j.nd * sizeof(double), s), "rprev = NaN");
    EventTimer tm(s);
    if (j.T > 0)
      HIP_TRY(launch_descent_fp64(s, j.da, j.z, j.mm, j.vv, rp, sg, ks, j.pool, j.counters), "descent fp64");
    j.stt.ms_descent += tm.stop_ms();
    j.done = j.T;
    return GRAVER_OK;
  }
  const bool small = j.kind == JOB_SMALL;
  int chunk = until - j.done;
  void* ddesc = nullptr;
  if (j.kind == JOB_BIG) {
    ddesc = W(ctx, j, WS_BIG_DESC, 4096, &st);
    if (!ddesc) return st;
  }
  while (j.done < until) {
    int c = std::min(chunk, until - j.done);
    // a launch of the large-basis kernel uses a single forward form
    if (!small && j.done < j.bf16_total) c = std::min(c, j.bf16_total - j.done);
    DescentArgs dc = j.da;
    dc.T = c;
    dc.bc = j.dbc + 2 * (size_t)j.done;
    dc.stepf = j.dstepf + 2 * (size_t)j.done;
    dc.bf16_iters = std::max(0, std::min(c, j.bf16_total - j.done));
    HIP_TRY(hipMemcpyAsync(j.fbak, j.fstate, j.sbytes, hipMemcpyDeviceToDevice, s), "state backup");
    HIP_TRY(hipMemcpyAsync(j.cbak, j.counters, 64, hipMemcpyDeviceToDevice, s), "counter backup");
    HIP_TRY(launch_fill_u64(s, reinterpret_cast<uint64_t*>(j.lg.count), 8, 0), "clear log count");
    std::vector<unsigned char> hd;
    EventTimer tm(s);
    if (small) {
      HIP_TRY(launch_descent_f32(s, dc, j.Bp, j.BTp, j.fstate, j.pool, j.counters, j.zrange), "descent mfma");
    } else if (j.kind == JOB_SPARSE) {
      HIP_TRY(launch_descent_sparse(s, dc, j.sp, j.sp_ent, j.sp_row, j.fstate, (int64_t)(j.sbytes / sizeof(float) / 3),
                                    j.counters, j.zrange),
              "descent (sparse form)");
    } else {
      BigJob bj{dc, j.img, j.fstate, j.kscr, j.counters};
      int64_t blocks = 0;
      int nbmax = 1;
      big_desc_prepare(j.sh, &bj, 1, hd, &blocks, &nbmax);
      HIP_TRY(hipMemcpyAsync(ddesc, hd.data(), hd.size(), hipMemcpyHostToDevice, s), "descriptor");
      HIP_TRY(launch_descent_big(s, j.sh, dc.bf16_iters > 0, ddesc, 1, blocks, nbmax), "descent mfma (large)");
    }
    j.stt.ms_descent += tm.stop_ms();
    uint32_t lflag[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(lflag, j.lg.count, sizeof(lflag), hipMemcpyDeviceToHost, s), "log flag");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (lflag[1]) {
      if (c == 1) return set_error(GRAVER_E_POOL_FULL, "one iteration yields more candidates than pool_capacity");
      HIP_TRY(hipMemcpyAsync(j.fstate, j.fbak, j.sbytes, hipMemcpyDeviceToDevice, s), "state rollback");
      HIP_TRY(hipMemcpyAsync(j.counters, j.cbak, 64, hipMemcpyDeviceToDevice, s), "counter rollback");
      chunk = std::max(1, c / 2);
      continue;
    }
    if (j.prm->collect) {
      HIP_TRY(launch_log_insert(s, j.lg, j.pool), "log insert");
      // stop as soon as the pool cannot hold the distinct candidates
      uint32_t pf[3] = {0, 0, 0};
      HIP_TRY(hipMemcpyAsync(pf, j.pool.count, sizeof(pf), hipMemcpyDeviceToHost, s), "pool flags");
      HIP_TRY(hipStreamSynchronize(s), "sync");
      if (pf[1]) return set_error(GRAVER_E_POOL_FULL, "more distinct candidates than pool_capacity");
      if (pf[2]) return set_error(GRAVER_E_POOL_FULL, "hash probe limit reached");
    }
    j.done += c;
  }
  return GRAVER_OK;
}

// Everything after the descent: state out, counters, A g = 0, sort, output.
graver_status job_finish(graver_ctx* ctx, Job& j, int64_t* count_out) {
  hipStream_t s = ctx->stream;
  graver_status st = GRAVER_OK;
  if (j.kind != JOB_FP64) HIP_TRY(launch_state_io_db(s, j.d, j.DBlay, j.N, j.fstate, j.z, j.mm, j.vv, 0), "state out");
  HIP_TRY(hipGetLastError(), "descent launch");
  unsigned long long hc[C_NCOUNTERS] = {};
  uint32_t hp[3] = {};
  HIP_TRY(hipMemcpyAsync(hc, j.counters, sizeof(hc), hipMemcpyDeviceToHost, s), "counters");
  HIP_TRY(hipMemcpyAsync(hp, j.pool.count, sizeof(hp), hipMemcpyDeviceToHost, s), "pool count");
  HIP_TRY(hipStreamSynchronize(s), "descent");
  j.stt.emit_events = (int64_t)hc[C_EMIT];
  j.stt.inbox_events = (int64_t)hc[C_INBOX];
  j.stt.out_of_range = (int64_t)hc[C_RANGE];

  graver_state* state = j.state;
  if (state) {
    if (state->z && state->z != j.z)
      HIP_TRY(hipMemcpyAsync(state->z, j.z, j.nd * sizeof(double), hipMemcpyDeviceToDevice, s), "z out");
    if (state->m) HIP_TRY(hipMemcpyAsync(state->m, j.mm, j.nd * sizeof(double), hipMemcpyDeviceToDevice, s), "m out");
    if (state->v) HIP_TRY(hipMemcpyAsync(state->v, j.vv, j.nd * sizeof(double), hipMemcpyDeviceToDevice, s), "v out");
  }

  *count_out = 0;
  if (!j.prm->collect) {
    HIP_TRY(hipStreamSynchronize(s), "sync");
    return GRAVER_OK;
  }
  if (hp[1]) return set_error(GRAVER_E_POOL_FULL, "more distinct candidates than pool_capacity");
  if (hp[2]) return set_error(GRAVER_E_POOL_FULL, "hash probe limit reached");
  uint32_t count = std::min<uint32_t>(hp[0], j.pool.cap);
  j.stt.unique = count;
  {
    EventTimer tm(s);
    unsigned int hbad = 0;
    if ((st = verify_rows(ctx, *j.ws, j.m, j.csr_rp, j.csr_col, j.csr_val, j.pool.keys, j.n, j.pool.stride, count,
                          &hbad)) != GRAVER_OK)
      return st;
    j.stt.ms_verify = tm.stop_ms();
    if (hbad) return set_error(GRAVER_E_NOT_KERNEL, "a collected candidate fails A g = 0");
    j.stt.verified = count;
  }
  if ((int64_t)count > j.keys_cap) {
    *count_out = count;
    return set_error(GRAVER_E_CAPACITY, "keys_cap too small for the collected set");
  }
  {
    EventTimer tm(s);
    if (j.prm->any_order) {
      if (count)
        HIP_TRY(hipMemcpy2DAsync(j.keys_out, j.n, j.pool.keys, j.pool.stride, j.n, count, hipMemcpyDeviceToDevice, s),
                "copy keys");
    } else {
      uint32_t p2 = 1024;
      while (p2 < count) p2 <<= 1;
      uint32_t* idx = (uint32_t*)W(ctx, j, WS_SORT_IDX, (size_t)p2 * sizeof(uint32_t), &st);
      uint64_t* pk = (uint64_t*)W(ctx, j, WS_SORT_TMP, (size_t)p2 * sizeof(uint64_t), &st);
      if (!idx || !pk) return st;
      HIP_TRY(launch_sort_keys(s, j.pool.keys, j.pool.stride, count, idx, pk), "sort");
      HIP_TRY(launch_gather_keys(s, j.pool.keys, j.pool.stride, j.n, idx, count, j.keys_out, j.n), "gather");
    }
    j.stt.ms_sort = tm.stop_ms();
  }
  *count_out = count;
  return GRAVER_OK;
}

}  // namespace

void tile_cache_free(graver_ctx* ctx) {
  delete static_cast<TileCache*>(ctx->tile_cache);
  ctx->tile_cache = nullptr;
}

}  // namespace graver

using namespace graver;

extern "C" graver_status graver_extract(graver_ctx* ctx, const graver_problem* prob,
                                        const graver_extract_params* prm, graver_state* state,
                                        int8_t* keys_out, int64_t keys_cap, int64_t* count_out,
                                        graver_extract_stats* stats) {
  if (!ctx || !prm || !count_out) return set_error(GRAVER_E_INVALID, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  Phase ph("graver_extract");
  Job j;
  j.prob = prob;
  j.prm = prm;
  j.state = state;
  j.keys_out = keys_out;
  j.keys_cap = keys_cap;
  j.ws = &ctx->ws;
  graver_status st;
  {
    Phase p1("extract: setup (validation, starts, pool)");
    st = job_setup(ctx, j, false, false);
  }
  if (st != GRAVER_OK) return st;
  {
    Phase p2("extract: descent and collection (Algorithm 2)");
    st = job_descend(ctx, j, j.T);
  }
  if (st != GRAVER_OK) return st;
  {
    Phase p3("extract: A g = 0, output");
    st = job_finish(ctx, j, count_out);
  }
  if (stats && (st == GRAVER_OK || st == GRAVER_E_CAPACITY)) *stats = j.stt;
  return st;
}

extern "C" graver_status graver_verify(graver_ctx* ctx, int32_t m, int32_t n, const int64_t* A, const int8_t* keys,
                                       int64_t count, int64_t* n_bad) {
  if (!ctx || !A) return set_error(GRAVER_E_INVALID, "NULL argument");
  if (m < 1 || n < 1 || n > 4096 || count < 0 || count > ((int64_t)1 << 31) - 1024)
    return set_error(GRAVER_E_INVALID, "bad m, n or count");
  if (count > 0 && !keys) return set_error(GRAVER_E_INVALID, "keys is NULL");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  graver_status st = GRAVER_OK;
  std::vector<int64_t> hA;
  std::vector<int32_t> rp, col;
  std::vector<int64_t> val;
  if ((st = copy_to_host(ctx, hA, A, (size_t)m * n)) != GRAVER_OK) return st;
  if ((st = build_csr(hA, m, n, rp, col, val)) != GRAVER_OK) return st;
  // rows restrided to the verification kernels' layout (multiple of 16 bytes)
  const int stride = key_stride(n);
  int8_t* rows = (int8_t*)ws_get(ctx, WS_KEYSCRATCH, (size_t)std::max<int64_t>(count, 1) * stride, &st);
  if (!rows) return st;
  if (count)
    HIP_TRY(hipMemcpy2DAsync(rows, stride, keys, n, n, (size_t)count, hipMemcpyDeviceToDevice, ctx->stream),
            "restride keys");
  unsigned int hbad = 0;
  if ((st = verify_rows(ctx, ctx->ws, m, rp, col, val, rows, n, stride, (uint32_t)count, &hbad)) != GRAVER_OK)
    return st;
  if (n_bad) *n_bad = hbad;
  if (hbad)
    return set_error(GRAVER_E_NOT_KERNEL, std::to_string(hbad) + " of " + std::to_string(count) +
                                              " rows fail A g = 0");
  return GRAVER_OK;
}

extern "C" graver_status graver_extract_batch(graver_ctx* ctx, int32_t count, const graver_problem* probs,
                                              const graver_extract_params* params, graver_state* const* states,
                                              int8_t* const* keys_out, const int64_t* keys_cap,
                                              int64_t* count_out, graver_extract_stats* stats,
                                              const graver_batch_params* bp, graver_batch_stats* bstats) {
  if (!ctx || !probs || !params || !count_out || !bp) return set_error(GRAVER_E_INVALID, "NULL argument");
  if (count < 1 || count > 4096) return set_error(GRAVER_E_INVALID, "need 1 <= count <= 4096");
  Phase ph("graver_extract_batch");
  for (int i = 0; i < count; ++i)
    if (params[i].collect && (!keys_out || !keys_cap)) return set_error(GRAVER_E_INVALID, "keys_out / keys_cap");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  hipStream_t s = ctx->stream;
  while ((int)ctx->batch_ws.size() < count) ctx->batch_ws.push_back(new Ws());
  std::vector<Job> jobs(count);
  graver_batch_stats bs{};
  graver_status st = GRAVER_OK;
  for (int i = 0; i < count; ++i) {
    Job& j = jobs[i];
    j.prob = &probs[i];
    j.prm = &params[i];
    j.state = states ? states[i] : nullptr;
    j.keys_out = keys_out ? keys_out[i] : nullptr;
    j.keys_cap = keys_cap ? keys_cap[i] : 0;
    j.ws = ctx->batch_ws[i];
    if ((st = job_setup(ctx, j, false, bp->autotune != 0)) != GRAVER_OK) return st;
  }

  // Large-basis jobs: at most two rounds (the bf16 phase of BF16 jobs and
  // every FP32 job, then the FP32 polish of BF16 jobs); each round launches
  // one grid per (tile shape, forward form).
  for (int round = 0; round < 2; ++round) {
    struct Part {
      int job;
      int begin, end;
      bool bf16;
    };
    std::vector<Part> parts;
    for (int i = 0; i < count; ++i) {
      Job& j = jobs[i];
      if (j.kind != JOB_BIG || j.T == 0) continue;
      if (round == 0) {
        if (j.bf16_total > 0) parts.push_back({i, 0, j.bf16_total, true});
        else parts.push_back({i, 0, j.T, false});
      } else if (j.bf16_total > 0 && j.bf16_total < j.T) {
        parts.push_back({i, j.bf16_total, j.T, false});
      }
    }
    if (parts.empty()) continue;
    // groups by (shape, form)
    std::map<std::pair<int, int>, std::vector<int>> groups;  // (cs*100+dbpw, bf16) -> part indices
    for (int p = 0; p < (int)parts.size(); ++p) {
      const Job& j = jobs[parts[p].job];
      groups[{j.sh.cs * 100 + j.sh.dbpw, parts[p].bf16 ? 1 : 0}].push_back(p);
    }
    struct Launch {
      BigShape sh;
      bool bf16;
      std::vector<unsigned char> host;
      void* dev;
      int count;
      int64_t blocks;
      int nbmax;
    };
    std::vector<Launch> launches;
    launches.reserve(groups.size());
    for (auto& kv : groups) {
      Launch L;
      L.sh = jobs[parts[kv.second[0]].job].sh;
      L.bf16 = kv.first.second != 0;
      std::vector<BigJob> bjs;
      for (int p : kv.second) {
        const Part& pt = parts[p];
        Job& j = jobs[pt.job];
        DescentArgs dc = j.da;
        dc.T = pt.end - pt.begin;
        dc.bc = j.dbc + 2 * (size_t)pt.begin;
        dc.stepf = j.dstepf + 2 * (size_t)pt.begin;
        dc.bf16_iters = pt.bf16 ? dc.T : 0;
        bjs.push_back(BigJob{dc, j.img, j.fstate, j.kscr, j.counters});
      }
      big_desc_prepare(L.sh, bjs.data(), (int)bjs.size(), L.host, &L.blocks, &L.nbmax);
      // the table lives in the workspace of the group's first job (its
      // own single-job table slot is not used while the batch runs)
      Job& owner = jobs[parts[kv.second[0]].job];
      L.dev = W(ctx, owner, WS_BIG_DESC, std::max<size_t>(L.host.size(), 4096), &st);
      if (!L.dev) return st;
      L.count = (int)bjs.size();
      launches.push_back(std::move(L));
    }
    // Descriptor tables first (host memory; not part of a graph).
    for (Launch& L : launches)
      HIP_TRY(hipMemcpyAsync(L.dev, L.host.data(), L.host.size(), hipMemcpyHostToDevice, s), "table");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    // The device work of the round: backups, log counts, grids, log
    // inserts.  With use_graph it is captured and launched as a graph (no
    // memset nodes: the counts are cleared by a fill kernel).
    auto enqueue = [&](hipStream_t q) -> graver_status {
      for (const Part& pt : parts) {
        Job& j = jobs[pt.job];
        HIP_TRY(hipMemcpyAsync(j.fbak, j.fstate, j.sbytes, hipMemcpyDeviceToDevice, q), "state backup");
        HIP_TRY(hipMemcpyAsync(j.cbak, j.counters, 64, hipMemcpyDeviceToDevice, q), "counter backup");
        HIP_TRY(launch_fill_u64(q, reinterpret_cast<uint64_t*>(j.lg.count), 8, 0), "clear log count");
      }
      for (Launch& L : launches)
        HIP_TRY(launch_descent_big(q, L.sh, L.bf16, L.dev, L.count, L.blocks, L.nbmax), "batched descent");
      for (const Part& pt : parts) {
        Job& j = jobs[pt.job];
        if (j.prm->collect) HIP_TRY(launch_log_insert(q, j.lg, j.pool), "log insert");
      }
      return GRAVER_OK;
    };
    EventTimer tm(s);
    if (bp->use_graph) {
      // captured on the context's private stream (the caller's stream may be
      // the legacy default stream, which cannot be captured), run on `s`
      if (!ctx->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking),
                                        "capture stream");
      const hipStream_t cs = ctx->capture_stream;
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
      graver_status est = enqueue(cs);
      hipError_t ce = hipStreamEndCapture(cs, &graph);
      if (est != GRAVER_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return est;
      }
      if (ce != hipSuccess) return hip_error(ce, "end capture");
      hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_error(ie, "graph instantiate");
      }
      hipError_t le = hipGraphLaunch(exec, s);
      hipError_t se = hipStreamSynchronize(s);
      (void)hipGraphExecDestroy(exec);
      (void)hipGraphDestroy(graph);
      if (le != hipSuccess) return hip_error(le, "graph launch");
      if (se != hipSuccess) return hip_error(se, "graph sync");
      ++bs.graphs;
    } else {
      if ((st = enqueue(s)) != GRAVER_OK) return st;
    }
    const double ms = tm.stop_ms();
    bs.ms_descent += ms;
    bs.launches += (int)launches.size();
    // per job: log overflow -> roll back and replay alone; pool overflow -> error
    for (const Part& pt : parts) {
      Job& j = jobs[pt.job];
      uint32_t lflag[2] = {0, 0}, pf[3] = {0, 0, 0};
      HIP_TRY(hipMemcpyAsync(lflag, j.lg.count, sizeof(lflag), hipMemcpyDeviceToHost, s), "log flag");
      HIP_TRY(hipMemcpyAsync(pf, j.pool.count, sizeof(pf), hipMemcpyDeviceToHost, s), "pool flags");
      HIP_TRY(hipStreamSynchronize(s), "sync");
      if (pf[1]) return set_error(GRAVER_E_POOL_FULL, "more distinct candidates than pool_capacity");
      if (pf[2]) return set_error(GRAVER_E_POOL_FULL, "hash probe limit reached");
      j.stt.ms_descent += ms;  // the shared grid's time (the batch total is in bstats)
      if (lflag[1]) {
        HIP_TRY(hipMemcpyAsync(j.fstate, j.fbak, j.sbytes, hipMemcpyDeviceToDevice, s), "state rollback");
        HIP_TRY(hipMemcpyAsync(j.counters, j.cbak, 64, hipMemcpyDeviceToDevice, s), "counter rollback");
        j.done = pt.begin;
        if ((st = job_descend(ctx, j, pt.end)) != GRAVER_OK) return st;
        ++bs.replays;
      } else {
        j.done = pt.end;
      }
    }
  }
  // small-basis and binary64 jobs run alone
  for (int i = 0; i < count; ++i) {
    Job& j = jobs[i];
    if (j.kind == JOB_BIG) continue;
    if ((st = job_descend(ctx, j, j.T)) != GRAVER_OK) return st;
    bs.launches += 1;
  }
  for (int i = 0; i < count; ++i) {
    st = job_finish(ctx, jobs[i], &count_out[i]);
    if (stats) stats[i] = jobs[i].stt;
    if (st != GRAVER_OK) return st;
  }
  if (bstats) *bstats = bs;
  return GRAVER_OK;
}
