/*
 * graver.h -- C ABI of the MI355X (gfx950) library for parallel Graver-basis
 * extraction and multi-start augmentation.
 *
 * Method: Liu, Wang, Yang, "Parallel Graver Basis Extraction for Nonlinear
 * Integer Optimization".  The problem (Section 1, eq. INLP) is
 *     min f(x)  s.t.  A x = b,  l <= x <= u,  x in Z^n,
 * with A in Z^{m x n}, b in Z^m, l, u in Z^n.
 *
 * Conventions for every entry point:
 *   - Matrices are row-major.  Integer data is int64 unless stated.
 *   - "device" pointers are HIP device addresses (for example the data
 *     pointer of a torch tensor on the GPU); "host" pointers are ordinary
 *     process memory.  Inputs are borrowed for the duration of the call;
 *     outputs are written by the library into caller-owned buffers.
 *   - GPU work is issued on the context's stream (graver_ctx_set_stream);
 *     calls that return a host value synchronise that stream before
 *     returning.  Each context must be used by one host thread at a time.
 *   - Every call returns a graver_status.  On an error nothing is written to
 *     the outputs named as such, and graver_last_error() returns a message.
 */
#ifndef GRAVER_H
#define GRAVER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GRAVER_OK = 0,
  GRAVER_E_INVALID = -1,          /* bad shape, pointer or parameter        */
  GRAVER_E_INFEASIBLE_START = -2, /* augmentation start violates Ax=b or l<=x<=u */
  GRAVER_E_NOT_KERNEL = -3,       /* a basis column or a candidate has A g != 0 */
  GRAVER_E_OVERFLOW = -4,         /* exact integer arithmetic would overflow */
  GRAVER_E_POOL_FULL = -5,        /* more distinct candidates than pool_capacity */
  GRAVER_E_NOMEM = -6,            /* device allocation failed               */
  GRAVER_E_DEVICE = -7,           /* HIP runtime error                      */
  GRAVER_E_CAPACITY = -8,         /* caller's output buffer is too small    */
  GRAVER_E_CANCELLED = -9         /* a served request was cancelled         */
} graver_status;

typedef enum {
  GRAVER_FP64 = 0, /* descent in binary64, bit-reproducible (parity mode)   */
  GRAVER_FP32 = 1, /* descent in binary32 on MFMA                           */
  GRAVER_BF16 = 2  /* contractions on bf16 MFMA, fp32 accumulate, fp32 polish */
} graver_precision;

/* How a binary32 descent forms the products with B (graver_extract_params.form). */
typedef enum {
  GRAVER_FORM_AUTO = 0,   /* sparse row lists when B's pay off (see below), else matrix cores */
  GRAVER_FORM_DENSE = 1,  /* matrix cores (MFMA) for every product                 */
  GRAVER_FORM_SPARSE = 2  /* row lists of B's nonzeros: gathers and exact scatter-adds,
                             one start per wavefront; GRAVER_FP32 only, n <= 1024,
                             d <= 1024, at most 128 row-list entries per lane       */
} graver_form;

typedef enum {
  GRAVER_F_QUADRATIC = 1,     /* f(x) = x^T Q x + c^T x, Q symmetric n x n  */
  GRAVER_F_SEPARABLE_POLY = 2 /* f(x) = sum_i sum_{k=0..deg} coef[i*(deg+1)+k] x_i^k */
} graver_f_kind;

typedef struct graver_ctx graver_ctx;

/* Instance data, all device pointers.  B is an n x d integer kernel basis
 * (columns span Ker_Z(A), Theorem 3.2), P = (B^T B)^{-1} B^T is d x n
 * (Section 3.1) and may be NULL when starts are supplied by the caller. */
typedef struct {
  int32_t m, n, d;
  const int64_t* A; /* m x n */
  const int64_t* b; /* m, used by graver_augment only */
  const int64_t* l; /* n */
  const int64_t* u; /* n */
  const int64_t* B; /* n x d */
  const double* P;  /* d x n or NULL */
} graver_problem;

/* Objective (device pointers).  Q must be symmetric (checked). */
typedef struct {
  int32_t kind;       /* graver_f_kind */
  int32_t degree;     /* separable polynomial degree, 0..8 */
  const double* Q;    /* n x n (quadratic) */
  const double* c;    /* n (quadratic) */
  const double* coef; /* n x (degree+1) (separable polynomial) */
} graver_objective;

/* Parameters of Parallel Extraction (Algorithm 2, Section 3.2). */
typedef struct {
  int64_t n_starts;  /* N, number of parallel starts                        */
  int32_t iters;     /* T, Adam steps taken by this call                     */
  int32_t precision; /* graver_precision                                     */
  double lr, beta1, beta2, eps; /* Adam (paper: lr 0.003; 0.9, 0.999, 1e-8)  */
  double lambda1, lambda2;      /* eq. loss weights (paper: 0.85, 1)         */
  int32_t init_mode; /* 0: g ~ Uniform(l-u, u-l) by Philox4x32-10 from seed,
                        z = P g;  1: z, m, v taken from the state buffers    */
  int32_t t0;        /* Adam steps already taken (resume); step t0+k uses
                        bias corrections 1 - beta^(t0+k)                     */
  int32_t polish_iters; /* GRAVER_BF16: last iterations run in FP32          */
  int32_t collect;   /* 1: collect candidates (Algorithm 2); 0: descent only */
  uint64_t seed;     /* Philox key for init_mode 0                           */
  int64_t first_start; /* Philox counter offset of start 0 (init_mode 0)     */
  int64_t pool_capacity; /* maximum number of distinct candidates (>= 1)     */
  int32_t any_order; /* 0: keys sorted lexicographically (deterministic order);
                        1: keys in the pool's order (the same set; for callers
                        that filter next, which sorts anyway)               */
  int32_t form;      /* graver_form.  AUTO takes the sparse form for a
                        GRAVER_FP32 call that the large matrix-core kernel
                        would run when B's padded row lists hold at most an
                        eighth of the n x d products.  The sparse form's exact
                        range is |round(z_j)| <= floor(2^24 / max row l1 of B)
                        (the small matrix-core kernel's); the large kernel's
                        is |round(z_j)| <= 256                               */
} graver_extract_params;

/* Optional descent state, device pointers to N x d binary64 arrays.  With
 * init_mode 1, z (required), m and v (NULL = zeros) are the starting state;
 * when non-NULL they receive the final state of the call. */
typedef struct {
  double* z;
  double* m;
  double* v;
} graver_state;

typedef struct {
  int64_t start_iterations; /* N * T                                         */
  int64_t emit_events;      /* iterates whose rounded coordinates changed    */
  int64_t inbox_events;     /* of those, nonzero and inside [l-u, u-l]       */
  int64_t unique;           /* distinct candidates collected                 */
  int64_t verified;         /* distinct candidates with A g = 0              */
  int64_t out_of_range;     /* iterates with a coordinate beyond the exact range */
  double ms_init, ms_descent, ms_verify, ms_sort; /* device time per phase  */
  int32_t tile_slices;      /* large-basis kernel: waves per start group     */
  int32_t tile_blocks;      /* and 16-column blocks per wave (0 otherwise)    */
  int32_t row_entries;      /* sparse form: row-list entries per lane (0 otherwise) */
  int32_t row_slots;        /* and its slots of 64 rows (0 otherwise)           */
} graver_extract_stats;

typedef struct {
  int64_t max_steps; /* cap on moves per start (>= 0)                        */
} graver_augment_params;

/* Parameters of the initial-solution search (Section 3.3, eq. init_sol). */
typedef struct {
  int64_t n_starts; /* S, number of parallel starting points                 */
  int32_t iters;    /* Adam steps per start                                  */
  int32_t init_mode; /* 0: x ~ Uniform(l, u) by Philox4x32-10 from seed;
                        1: starting points supplied in x0                    */
  double lr, beta1, beta2, eps; /* Adam                                      */
  double lambda3;   /* weight of the integrality term (paper: 0.1)           */
  uint64_t seed;    /* Philox key for init_mode 0                            */
  int64_t first_start; /* Philox counter offset of start 0 (init_mode 0)     */
} graver_init_params;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  The context owns device
 * workspace (grown on demand, freed by graver_ctx_destroy).  Stream: the
 * null stream until graver_ctx_set_stream. */
graver_status graver_ctx_create(graver_ctx** out, int32_t device);
void graver_ctx_destroy(graver_ctx* ctx);
/* Releases the device workspace the context grew for earlier calls (descent
 * state, candidate pool and log, filter and augmentation buffers; the solve
 * cache and tuned tile shapes stay).  For pipelines whose stages each need
 * most of the device memory, e.g. an extraction of about 1e8 candidates
 * followed by their filter: trimming between the two frees the pool before
 * the filter allocates.  Synchronises the context's stream first. */
graver_status graver_ctx_trim(graver_ctx* ctx);
/* Issue all GPU work of this context on `hip_stream` (a hipStream_t, e.g.
 * torch.cuda.current_stream().cuda_stream); NULL selects the null stream. */
graver_status graver_ctx_set_stream(graver_ctx* ctx, void* hip_stream);
/* Message of the last error on the calling thread (never NULL). */
const char* graver_last_error(void);
const char* graver_status_string(graver_status s);

/* ---- kernel basis (host) ---------------------------------------------- */

/* Lemma 3.1 / Theorem 3.2 and Appendix A.  From A (host, m x n) computes a
 * unimodular K with A K = (H | 0) in Hermite normal form by integer column
 * operations, takes B = the last d = n - rank(A) columns, and LLL-reduces
 * them when `lll` is nonzero (Algorithm 3: size reduction with
 * nearest-integer coefficients, ties to even, and exchange when
 * ||b*_{i-1}||^2 > 2 ||b*_i||^2), all in exact integer arithmetic.
 * Outputs (host): B_out n x d row-major (capacity n*n entries), *d_out,
 * and when P_out is non-NULL the d x n matrix (B^T B)^{-1} B^T in binary64
 * (capacity n*n entries).  GRAVER_E_OVERFLOW if an entry of K or B leaves
 * int64.  Needs no GPU. */
graver_status graver_kernel_basis(int32_t m, int32_t n, const int64_t* A, int32_t lll,
                                  int64_t* B_out, int32_t* d_out, double* P_out);

/* ---- the hot path (device) --------------------------------------------- */

/* Parallel Extraction, Algorithm 2 (Section 3.2).  For each of N starts,
 * T Adam steps on eq. loss
 *   Phi(z) = ||B z||_1 + lambda1 sum_i (z_i - floor z_i)(ceil z_i - z_i)
 *            + lambda2 max{1/||z||_inf - 1, 0};
 * after every step the iterate is rounded to r (nearest integer, ties to
 * even), g = B r is formed exactly and kept when g != 0 and
 * l - u <= g <= u - l (condition C4).  Distinct candidates are checked for
 * A g = 0 (condition C1) and returned sorted lexicographically (signed,
 * component 0 first) as int8 rows in keys_out (device, capacity keys_cap
 * rows of n bytes); *count_out (host) receives the count.  Requires
 * max(u - l) <= 127.  Errors: GRAVER_E_POOL_FULL when more than
 * pool_capacity distinct candidates appear, GRAVER_E_CAPACITY when
 * keys_cap is too small, GRAVER_E_NOT_KERNEL when a candidate fails A g = 0.
 * state and stats may be NULL. */
graver_status graver_extract(graver_ctx* ctx, const graver_problem* prob,
                             const graver_extract_params* params, graver_state* state,
                             int8_t* keys_out, int64_t keys_cap, int64_t* count_out,
                             graver_extract_stats* stats);

/* ---- batched extraction ----------------------------------------------- */

typedef struct {
  int32_t autotune;  /* 1: the large-basis tile shape of each basis size is the
                        fastest candidate in a short timed trial (kept in the
                        context); 0: the fixed shape table                     */
  int32_t use_graph; /* 1: each round of the batched descent (state backups,
                        grids, log inserts) is captured and run as a HIP graph */
} graver_batch_params;

typedef struct {
  double ms_descent; /* device time of the batched descent rounds             */
  int32_t launches;  /* descent grids launched                                */
  int32_t replays;   /* instances replayed alone after a log overflow         */
  int32_t graphs;    /* rounds run as a graph                                 */
} graver_batch_stats;

/* Parallel Extraction for `count` independent instances in one call.
 * Instance i is described by probs[i], params[i], states[i] (states may be
 * NULL, entries may be NULL) and writes keys_out[i] (device, keys_cap[i]
 * rows), count_out[i] and stats[i] (may be NULL), exactly as graver_extract
 * does for one instance.  Every instance with n > 128 or d > 128 in FP32 or
 * BF16 runs in a shared grid with the other instances of the same tile
 * shape and forward form (one launch for all of them; the bf16 phase and the
 * FP32 polish of BF16 instances are two rounds); the other instances run
 * alone.  With the fixed shape table an instance's results equal a single
 * graver_extract call's bit for bit.  Each instance keeps its own device
 * workspace in the context.  The first error ends the call. */
graver_status graver_extract_batch(graver_ctx* ctx, int32_t count, const graver_problem* probs,
                                   const graver_extract_params* params, graver_state* const* states,
                                   int8_t* const* keys_out, const int64_t* keys_cap, int64_t* count_out,
                                   graver_extract_stats* stats, const graver_batch_params* batch,
                                   graver_batch_stats* batch_stats);

/* Minimality filter with deduplication (condition C3, Section 3; the
 * conformal order of Section 1).  Input: count_in int8 rows of n bytes
 * (device), entries in [-127, 127] (the negation of every entry must be an
 * int8; candidates of a box of widths at most 127 always are).  The set
 * C = X u (-X) without 0 is formed; g in C is dropped
 * when some h in C, h != g, satisfies h_i g_i >= 0 and |h_i| <= |g_i| for
 * all i.  Output (device, capacity keys_cap rows): one representative per
 * pair {g, -g} (first nonzero entry positive), sorted lexicographically;
 * *count_out (host) receives the count. */
graver_status graver_filter(graver_ctx* ctx, int32_t n, const int8_t* keys_in, int64_t count_in,
                            int8_t* keys_out, int64_t keys_cap, int64_t* count_out);

/* Condition C1 (Section 3) on its own: A g = 0 exactly for each of the
 * `count` int8 rows of n bytes in keys (device), with A (device, m x n,
 * |A_ij| < 2^31) -- the check graver_extract applies to every distinct
 * candidate, here for a direction set the caller brings (for example one
 * read from a file before graver_augment).  *n_bad (host, may be NULL)
 * receives the number of rows with A g != 0; the call returns
 * GRAVER_E_NOT_KERNEL when it is nonzero, GRAVER_E_OVERFLOW when some
 * |A_ij| >= 2^31. */
graver_status graver_verify(graver_ctx* ctx, int32_t m, int32_t n, const int64_t* A, const int8_t* keys,
                            int64_t count, int64_t* n_bad);

/* Multi-start augmentation (Algorithm 1 from every start; MAPE, Section
 * 3.3).  Directions: the K int8 rows `dirs` (device) and their negations,
 * ordered as given with each row followed by its negation.  From each of
 * the S starts x_starts (device, S x n; each must satisfy A x = b and
 * l <= x <= u, else GRAVER_E_INFEASIBLE_START) the best move
 * (g, lambda), lambda = 1..lambda_max(g) keeping x + lambda g in the box,
 * is the one with the smallest Delta = f(x + lambda g) - f(x) (ties: earlier
 * direction, then smaller lambda), evaluated in binary64 with a fixed
 * formula (quadratic: Delta = lambda a_g + lambda^2 q_g with
 * r = c + 2 Q x, a_g = sum g_i r_i, q_g = sum g_i (sum Q_ij g_j) over the
 * support of g in ascending order; separable polynomial: the ascending sum
 * over the support of p_i(x_i + lambda g_i) - p_i(x_i), Horner from the top
 * coefficient); it is taken when Delta < 0, until no move improves or
 * max_steps moves were made.  Outputs (device): x_out S x n, f_out S
 * (f at the end point, ascending sums, no fused multiply-add), steps_out S;
 * *best_out (host, may be NULL) = index of the smallest f_out (ties: lowest). */
graver_status graver_augment(graver_ctx* ctx, const graver_problem* prob,
                             const graver_objective* f, const int8_t* dirs, int64_t K,
                             int32_t S, const int64_t* x_starts,
                             const graver_augment_params* params, int64_t* x_out,
                             double* f_out, int64_t* steps_out, int32_t* best_out);

/* graver_augment for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as graver_augment; the context supplies
 * the device and the stream.  It calls no hipMalloc / hipFree: its scratch
 * (start flags, per-start r rows, per-block best moves, the q_g cache, the
 * value table) is one fixed 64 MiB array per GPU in the library, allocated
 * with the library's code object and held until the process ends.  Calls
 * needing more (about 8 S n + 16 S ceil(K / 256) + 8 K + 1024 n bytes) return
 * GRAVER_E_CAPACITY and do nothing.  l <= u, u - l <= 127 and the symmetry
 * of Q are checked on the device (GRAVER_E_INVALID).  Every call on one GPU
 * shares that array: calls that overlap on one GPU (several host threads or
 * streams) race and must be serialised by the caller; each call
 * re-initialises what it reads. */
graver_status graver_augment_noalloc(graver_ctx* ctx, const graver_problem* prob,
                                     const graver_objective* f, const int8_t* dirs, int64_t K,
                                     int32_t S, const int64_t* x_starts,
                                     const graver_augment_params* params, int64_t* x_out,
                                     double* f_out, int64_t* steps_out, int32_t* best_out);

/* Initial feasible solutions (Section 3.3, eq. init_sol).  From each of S
 * starting points, `iters` Adam steps minimise
 *     ||A x - b||^2 + lambda3 * sum_i (x_i - floor x_i)(ceil x_i - x_i)
 * with x projected onto [l, u] after every step; then r = round-half-even(x)
 * is feasible when A r = b exactly and l <= r <= u.  Arithmetic is binary64
 * with a fixed order (residual res_i = (sum_j A_ij x_j) - b_i, gradient
 * 2 sum_i A_ij res_i + lambda3 ((ceil x_j + floor x_j) - 2 x_j), ascending
 * sums from 0, no fused multiply-add), so results are bit-reproducible.
 * prob->B and prob->P are not used.  Inputs: x0 (device, S x n binary64,
 * read when init_mode is 1, else may be NULL).  Outputs (device): x_out
 * (S x n binary64, the final iterates, may be NULL), sol_out (S x n int64,
 * the rounded points), feasible_out (S int32, 1 when feasible);
 * *n_feasible (host, may be NULL) = number of feasible rows.  Errors:
 * GRAVER_E_OVERFLOW when sum_j |A_ij| max(|l_j|, |u_j|) or |b_i| reaches
 * 2^53 (the exact test then could not be done in int64 / the residual would
 * not be exact). */
graver_status graver_init_solutions(graver_ctx* ctx, const graver_problem* prob,
                                    const graver_init_params* params, const double* x0,
                                    double* x_out, int64_t* sol_out, int32_t* feasible_out,
                                    int64_t* n_feasible);

/* ---- linear inequalities (Section 3.4) --------------------------------- */

/* Slack form of  A x = b, G x >= h, l <= x <= u  (eq. NLIP_ineq_slack):
 *     [A 0; G -I] (x, s) = (b, h),  l <= x <= u,  0 <= s <= s_max,
 * s_max_i = sum_j max(G_ij l_j, G_ij u_j) - h_i (the largest slack any x in
 * the box has, so no feasible point is lost), and, when B (an n x d kernel
 * basis of A) is given, the kernel basis [B; G B] of the lifted matrix (the
 * corollary of Section 3.4): its surrogate is eq. surrogate_ineq.  The
 * lifted program (n + m' variables, m + m' rows) then goes through the
 * ordinary entry points; the first n coordinates of its points are x.
 * All host pointers, row-major.  m may be 0 (no equalities; then B = I).
 * Outputs: A_out (m+m') x (n+m'), b_out m+m', l_out and u_out n+m',
 * Bt_out (n+m') x d.  Errors: GRAVER_E_INVALID when some row of G x >= h
 * holds nowhere in the box; GRAVER_E_OVERFLOW on int64 overflow.  (The
 * int8 keys of the extraction need every u - l, slack rows included, at
 * most 127.) */
graver_status graver_lift_inequalities(int32_t m, int32_t n, const int64_t* A, const int64_t* b,
                                       const int64_t* l, const int64_t* u, int32_t mi,
                                       const int64_t* G, const int64_t* h, int32_t d,
                                       const int64_t* B, int64_t* A_out, int64_t* b_out,
                                       int64_t* l_out, int64_t* u_out, int64_t* Bt_out);

/* ---- end-to-end solve (MAPE, Section 3.3) ----------------------------- */

typedef struct {
  graver_extract_params extract; /* Algorithm 2; collect must be 1; init_mode
                                    0 draws starts with P (computed by the
                                    library when prob->B is NULL)            */
  graver_init_params init;       /* eq. init_sol starting points             */
  int64_t max_steps;             /* augmentation cap per start (>= 0)        */
  int32_t lll;                   /* library-computed basis: LLL-reduce it    */
  const int64_t* x_starts;       /* device, n_x_starts x n: feasible points
                                    the caller already has, augmented after
                                    the initial solutions (may be NULL)     */
  int32_t n_x_starts;
  int32_t reuse;                 /* 1: look up / keep the basis and the
                                    filtered set of this (A, u - l) in the
                                    context (Section 3.3: the Graver basis
                                    depends on A only, so instances sharing A
                                    reuse one extraction)                    */
} graver_solve_params;

typedef struct {
  int32_t d;                 /* kernel dimension n - rank(A)                 */
  int32_t reused;            /* 1 when the cached set was used               */
  int32_t best_start;        /* index of the best start among the feasible ones */
  int64_t unique;            /* distinct verified candidates (0 when reused) */
  int64_t filtered;          /* size of the filtered direction set F         */
  int64_t feasible_starts;   /* feasible rounded initial solutions           */
  int64_t augment_steps;     /* moves made over all starts                   */
  double ms_basis, ms_extract, ms_filter, ms_init, ms_augment; /* host wall time per phase */
} graver_solve_stats;

/* MAPE end to end: kernel basis (Lemma 3.1, Theorem 3.2; host, or the
 * caller's prob->B / prob->P), Parallel Extraction (Algorithm 2), the
 * minimality filter, initial feasible solutions (eq. init_sol), and
 * augmentation (Algorithm 1) from every feasible initial solution, in the
 * order found, then from the caller's x_starts, with directions F u (-F);
 * the best end point is the answer (ties: the lowest start index).
 * prob: device pointers A, b, l, u; B (n x d) and P (d x n) may be NULL.
 * Outputs: x_best (device, n int64), *f_best (host), stats (host, may be
 * NULL).  GRAVER_E_INFEASIBLE_START when there is no start at all (no
 * feasible initial solution and no x_starts) or an x_starts row violates
 * A x = b or l <= x <= u.
 * With reuse, the context keeps the basis and F of each distinct (A, u - l)
 * until it is destroyed; a later call with the same (A, u - l) skips the
 * basis, the extraction and the filter (its extraction parameters are then
 * not used). */
graver_status graver_solve(graver_ctx* ctx, const graver_problem* prob, const graver_objective* f,
                           const graver_solve_params* params, int64_t* x_best, double* f_best,
                           graver_solve_stats* stats);

/* ---- serving ----------------------------------------------------------- */

typedef struct graver_server graver_server;

typedef struct {
  int32_t device;
  int64_t hbm_budget;    /* bytes of device memory admitted requests may hold  */
  int32_t max_batch;     /* requests per batched extraction                     */
  int32_t gpu_workers;   /* concurrent batches (each on its own stream)         */
  int32_t host_threads;  /* kernel-basis threads                                */
  int32_t autotune;      /* graver_batch_params.autotune                        */
  int32_t use_graph;     /* graver_batch_params.use_graph                       */
  int32_t batch_window_us; /* a worker that admitted fewer than max_batch requests
                            waits up to this long for more ready ones          */
} graver_server_params;

/* One INLP request; every pointer is host memory, read during submit only. */
typedef struct {
  int32_t m, n;
  const int64_t* A;      /* m x n */
  const int64_t* b;      /* m */
  const int64_t* l;      /* n */
  const int64_t* u;      /* n */
  int32_t f_kind;        /* graver_f_kind */
  int32_t f_degree;
  const double* Q;       /* n x n (quadratic) */
  const double* c;       /* n (quadratic) */
  const double* coef;    /* n x (degree+1) (separable polynomial) */
  graver_extract_params extract; /* init_mode 0 (starts z = P g) */
  graver_init_params init;       /* initial-solution search */
  int64_t max_steps;             /* augmentation cap per start */
  int32_t lll;                   /* LLL-reduce the basis */
  const int64_t* x_starts;       /* n_x_starts x n feasible points, may be NULL */
  int32_t n_x_starts;
} graver_request;

typedef struct {
  graver_status status;    /* of the request's solve                          */
  double f_best;
  int32_t d;
  int64_t unique, filtered, feasible_starts, augment_steps;
  int32_t batch_size;      /* requests in its batched extraction              */
  int32_t reused_basis;    /* 1 when the basis came from the A-keyed cache     */
  double t_submit, t_ready, t_admit, t_done; /* seconds on the server's clock  */
} graver_result;

/* A request server (Section 3.3's MAPE per request) with continuous
 * batching: host threads compute kernel bases (Lemma 3.1, Theorem 3.2;
 * cached by A, whose basis every request with that A reuses); requests whose
 * basis is ready are admitted while their estimated device footprint
 * (basis, starts and descent state, candidate pool and log, filter and
 * augmentation buffers) fits in hbm_budget, in arrival order, and join the
 * next batched extraction of a free GPU worker (graver_extract_batch);
 * each request then runs the filter, the initial-solution search and the
 * augmentation on that worker's stream, and its device memory is released.
 * Several workers keep several batches on the device at once.
 * Errors of one request are reported in its result. */
graver_status graver_server_create(graver_server** out, const graver_server_params* params);
/* Copies the request; *ticket identifies it.  Never blocks on the GPU. */
graver_status graver_server_submit(graver_server* srv, const graver_request* req, int64_t* ticket);
/* Blocks until the request is done; x_best (host, n values, may be NULL). */
graver_status graver_server_wait(graver_server* srv, int64_t ticket, graver_result* result, int64_t* x_best);
/* Non-blocking form of graver_server_wait: *done (host) = 1 when the
 * request has finished, and then result and x_best are written and the
 * ticket is released exactly as graver_server_wait does; *done = 0 leaves
 * everything untouched.  GRAVER_E_INVALID for an unknown or released ticket. */
graver_status graver_server_poll(graver_server* srv, int64_t ticket, int32_t* done, graver_result* result,
                                 int64_t* x_best);
/* Cancels a request.  One still waiting for its basis or for admission
 * leaves its queue at once (it holds no device memory); one already on the
 * GPU stops at its next stage boundary (after the batched extraction it
 * shares with others) and its device memory is released with its batch.
 * Its result then has status GRAVER_E_CANCELLED; the ticket stays valid
 * until graver_server_wait / _poll collects it.  *cancelled (host) = 1 when
 * the request will end cancelled, 0 when it had already finished (its result
 * stands).  GRAVER_E_INVALID for an unknown or released ticket. */
graver_status graver_server_cancel(graver_server* srv, int64_t ticket, int32_t* cancelled);
/* Finishes every submitted request, then stops the threads. */
void graver_server_destroy(graver_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* GRAVER_H */
