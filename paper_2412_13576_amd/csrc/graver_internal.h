// Internal declarations shared by the host entry points and the kernel
// launchers of the gfx950 library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "graver.h"

namespace graver {
// A set of device workspace buffers, one per slot, each grown on demand.
struct Ws {
  static constexpr int kSlots = 72;
  void* buf[kSlots] = {};
  size_t cap[kSlots] = {};
};
}  // namespace graver

struct graver_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  graver::Ws ws;                       // workspace of single-instance calls
  std::vector<graver::Ws*> batch_ws;   // one per instance of a batched call
  void* solve_cache = nullptr;         // graver::SolveCache (bases and filtered sets by (A, u - l))
  void* tile_cache = nullptr;          // graver::TileCache (autotuned large-kernel shapes)
  hipStream_t capture_stream = nullptr;  // private stream for graph capture (default priority)
};

namespace graver {

graver_status set_error(graver_status s, const std::string& msg);
graver_status hip_error(hipError_t e, const char* what);

#define HIP_TRY(expr, what)                               \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_error(e_, what);     \
  } while (0)
// the same inside functions that return a hipError_t
#define HIP_RET(expr)                                     \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return e_;                      \
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

// A named phase on rocprofv3's marker trace (--marker-trace) for the
// lifetime of the object (a roctx range; free when no tool is attached).
struct Phase {
  explicit Phase(const char* name) { roctxRangePushA(name); }
  ~Phase() { roctxRangePop(); }
  Phase(const Phase&) = delete;
  Phase& operator=(const Phase&) = delete;
};

// Device time between construction and stop_ms() on one stream.
struct EventTimer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  // timing only: a failed event call leaves the time at 0 and is not an error
  explicit EventTimer(hipStream_t st) : s(st) {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, s);
  }
  double stop_ms() {
    float ms = 0.f;
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
  }
  ~EventTimer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

graver_status validate_problem(graver_ctx* ctx, const graver_problem* p, bool need_b,
                               std::vector<int64_t>& hl, std::vector<int64_t>& hu);
void ws_free(Ws& w);

// Workspace slots (each grows on demand and is reused across calls).
enum Slot : int {
  WS_Z = 0, WS_M, WS_V, WS_RPREV, WS_SIGN, WS_KEYSCRATCH, WS_G0,
  WS_POOL_KEYS, WS_POOL_TABLE, WS_POOL_COUNT, WS_COUNTERS,
  WS_BF, WS_BC, WS_SORT_IDX, WS_SORT_TMP, WS_FLAGS, WS_SCAN, WS_SCAN2,
  WS_F_CANON, WS_F_UNIQ, WS_F_L1, WS_F_MASK, WS_F_LO, WS_F_ALIVE, WS_F_CHUNK,
  WS_A_R, WS_A_PART, WS_A_DONE, WS_A_QG, WS_A_TAB,
  WS_MF_B, WS_MF_BT, WS_MF_STATE, WS_MISC,
  WS_F_CODE, WS_F_HIST, WS_F_OFF, WS_F_BITS, WS_F_BL, WS_LOG, WS_LOG_COUNT, WS_MF_BAK, WS_MISC2,
  WS_I_X, WS_I_M, WS_I_V, WS_I_R, WS_I_G,
  WS_S_KEYS, WS_S_F, WS_S_SOL, WS_S_FEAS, WS_S_IDX, WS_S_STARTS, WS_S_X, WS_S_FV, WS_S_STEPS, WS_S_B, WS_S_P,
  WS_V_CSR, WS_BIG_DESC, WS_R_KEYS, WS_R_HIST, WS_STEPF, WS_F_FIRST,
  WS_END
};
static_assert(WS_END <= Ws::kSlots, "too many workspace slots");
void* ws_get(graver_ctx* ctx, int slot, size_t bytes, graver_status* st);
void* ws_get(graver_ctx* ctx, Ws& w, int slot, size_t bytes, graver_status* st);

graver_status kernel_basis_host(int32_t m, int32_t n, const int64_t* A, int32_t do_lll,
                                int64_t* B_out, int32_t* d_out, double* P_out);

// ---- device pool (hash set of int8 keys) --------------------------------
struct PoolDev {
  int8_t* keys;        // cap x stride bytes
  uint64_t* table;     // tsize entries, 0 = empty
  uint32_t* count;     // [0] allocated keys, [1] full flag, [2] probe-limit flag
  uint64_t tmask;      // tsize - 1
  uint32_t cap;
  int32_t n, stride;   // key length, row stride (multiple of 16)
};
inline int key_stride(int n) { return (n + 15) / 16 * 16; }

// Append-only candidate log written by the MFMA descent (rows of `stride`
// bytes; all-zero rows are unused slots) and later inserted into the pool.
struct LogDev {
  int8_t* rows;
  uint32_t* count;  // rows reserved so far (may exceed cap)
  uint32_t cap;
  int32_t stride;
};

// Counters written by the descent kernels (atomic adds, int64).
enum Counter : int { C_EMIT = 0, C_INBOX, C_RANGE, C_NCOUNTERS };

// Blocks of 256 threads for a grid-stride loop over `threads` items: a
// dispatch counts at most 2^32 - 1 work-items, so the grid is capped at
// 2^22 blocks (2^30 threads) and each thread loops.
inline unsigned stride_grid(uint64_t threads) {
  const uint64_t b = (threads + 255) / 256;
  return (unsigned)(b < ((uint64_t)1 << 22) ? (b > 0 ? b : 1) : ((uint64_t)1 << 22));
}

// ---- launchers (implemented in the .hip files) --------------------------
struct DescentArgs {
  int32_t n, d, N, T;
  const int64_t* B;     // n x d (device)
  const int64_t* l;
  const int64_t* u;
  double lr, beta1, beta2, eps, lambda1, lambda2;
  double one_minus_b1, one_minus_b2;
  const double* bc;     // 2*T bias corrections (device): [2k] = 1-b1^t, [2k+1] = 1-b2^t
  const float* stepf;   // 2*T (device): [2k] = (float)(lr / bc[2k]), [2k+1] = (float)(1 / bc[2k+1])
  int32_t collect;
  int32_t bf16_iters;   // MFMA path: iterations k < bf16_iters use the bf16 hi/lo forward
  int32_t lim_uniform;  // u_i - l_i when equal for every i, else -1
  LogDev log;           // MFMA path: candidate log
};

struct InitArgs {
  int32_t m, n, T;
  int64_t S;
  const int64_t* A;
  const int64_t* b;
  const int64_t* l;
  const int64_t* u;
  double lr, beta1, beta2, eps, lambda3, one_minus_b1, one_minus_b2;
  const double* bc;
};
hipError_t launch_gather_rows_i64(hipStream_t s, const int64_t* src, int n, const int32_t* idx, int64_t cnt,
                                  int64_t* dst);
void solve_cache_free(graver_ctx* ctx);
void tile_cache_free(graver_ctx* ctx);

hipError_t launch_init_sol(hipStream_t s, const InitArgs& a, const double* x0, uint64_t seed, int64_t first,
                           double* X, double* M, double* V, double* R, double* gscratch, int64_t* xr,
                           int32_t* feas, unsigned int* nfeas);

hipError_t launch_init_box(hipStream_t s, int n, int d, int64_t N, const double* P,
                           const int64_t* l, const int64_t* u, uint64_t seed,
                           int64_t first_start, double* g_scratch, double* z_out);
hipError_t launch_descent_fp64(hipStream_t s, const DescentArgs& a, double* z, double* m,
                               double* v, double* rprev, int8_t* sign_scratch,
                               int8_t* key_scratch, PoolDev pool, unsigned long long* counters);
bool descent_f32_supported(int n, int d);
hipError_t launch_descent_f32(hipStream_t s, const DescentArgs& a, const float* Bf_packed,
                              const float* BTf_packed, float* state, PoolDev pool,
                              unsigned long long* counters, float zrange);
hipError_t launch_f32_pack(hipStream_t s, int n, int d, const int64_t* B, float* Bp, float* BTp,
                           int* rowl1max_dev);
size_t f32_pack_floats(int n, int d);
size_t f32_state_floats(int n, int d, int64_t N);
hipError_t launch_f32_state_io(hipStream_t s, int n, int d, int64_t N, float* state,
                               double* z, double* m, double* v, int to_device);

hipError_t launch_state_io_db(hipStream_t s, int d, int DB, int64_t N, float* state, double* z, double* m,
                              double* v, int to_device);
// Large-basis kernel: a start group's coordinates split over cs waves of
// dbpw 16-column blocks each (image and state layouts use cs * dbpw blocks).
struct BigShape {
  int cs = 0, dbpw = 0;
};
BigShape big_shape_default(int d);
bool big_shape_fits(BigShape sh, int d);  // an instantiated shape with cs * dbpw * 16 >= d
int big_shape_candidates(int d, BigShape* out, int cap);
bool descent_big_supported(int n, int d);
hipError_t launch_rowl1(hipStream_t s, int n, int d, const int64_t* B, int* rowl1);
size_t big_image_bytes(int n, BigShape sh);
size_t big_state_floats(BigShape sh, int64_t N);
hipError_t launch_big_pack(hipStream_t s, int n, int d, BigShape sh, const int64_t* B, unsigned char* img);
// One instance of a (possibly batched) large-kernel launch.
struct BigJob {
  DescentArgs a;
  const unsigned char* img;
  float* state;
  int8_t* scratch;
  unsigned long long* counters;
};
// Descriptor table of a launch over `count` jobs of one shape: host image
// (kept alive by the caller until the stream has consumed it) and its size.
size_t big_desc_prepare(BigShape sh, const BigJob* jobs, int count, std::vector<unsigned char>& host,
                        int64_t* total_blocks, int* max_nb);
// One grid over every job's start groups; the table must already be on the device.
hipError_t launch_descent_big(hipStream_t s, BigShape sh, bool bf16_forward, const void* dev_desc, int count,
                              int64_t total_blocks, int max_nb);

hipError_t launch_pool_clear(hipStream_t s, PoolDev p);
// p[0 .. n) = value (a kernel, so it may be captured in a graph)
hipError_t launch_fill_u64(hipStream_t s, uint64_t* p, uint64_t n, uint64_t value);
hipError_t launch_log_insert(hipStream_t s, LogDev log, PoolDev pool);
hipError_t launch_verify(hipStream_t s, PoolDev p, uint32_t count, int m, int64_t nnz, const int32_t* rp,
                         const int32_t* col, const int64_t* val, unsigned int* bad);
hipError_t launch_sort_keys(hipStream_t s, const int8_t* keys, int stride, uint32_t count, uint32_t* idx,
                            uint64_t* pk);
hipError_t launch_gather_keys(hipStream_t s, const int8_t* keys, int stride, int n,
                              const uint32_t* idx, uint32_t count, int8_t* out, int out_stride);

// filter
hipError_t launch_filter(hipStream_t s, graver_ctx* ctx, int n, const int8_t* in, int64_t count_in,
                         int8_t* out, int64_t cap, int64_t* count_out, graver_status* st);

// augment
struct AugArgs {
  int32_t n, m, S, K;
  const int64_t* A;
  const int64_t* b;
  const int64_t* l;
  const int64_t* u;
  int32_t kind, degree;
  const double* Q;
  const double* c;
  const double* coef;
  const int8_t* dirs;
  int64_t max_steps;
};
// Device scratch of one augmentation call, carved from one block of
// aug_work_bytes(n, S, K, w) bytes (w > max(u - l): width of the value table
// of a separable objective).
struct AugWork {
  unsigned int* flags;  // 64 bytes: start check, step activity
  uint32_t* done;       // S
  double* R;            // S x n
  void* partial;        // S x (direction blocks) best moves
  uint64_t* qg;         // K cached q_g
  double* tab;          // n x w
  int32_t* best;        // best start
};
size_t aug_work_bytes(int n, int S, int64_t K, int w);
AugWork aug_work_carve(void* base, int n, int S, int64_t K, int w);
hipError_t launch_aug_validate(hipStream_t s, int n, const int64_t* l, const int64_t* u, const double* Q,
                               unsigned int* flag);
graver_status run_augment(graver_ctx* ctx, const AugArgs& a, int w, const int64_t* x_starts,
                          int64_t* x_out, double* f_out, int64_t* steps_out, int32_t* best_out);
graver_status run_augment_ws(hipStream_t s, const AugArgs& a, int w, const AugWork& wk, const int64_t* x_starts,
                             int64_t* x_out, double* f_out, int64_t* steps_out, int32_t* best_out);

}  // namespace graver
