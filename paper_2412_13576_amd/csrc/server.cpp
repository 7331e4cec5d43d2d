// Request server with continuous batching (MAPE per request, Section 3.3).
//
// Threads: `host_threads` basis workers (kernel basis and P on the host,
// shared by every request with the same A and LLL flag) and `gpu_workers`
// GPU workers, each with its own context and stream.  A GPU worker admits
// ready requests in arrival order while their estimated device footprint
// fits in the budget (and at most max_batch of them), runs their extraction
// as one batched call, then the filter, the initial-solution search and the
// augmentation of each request on its stream, and releases the memory.
// Requests that become ready while a batch runs are picked up by the next
// free worker, so batches overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "graver_internal.h"

namespace graver {
namespace {

struct BasisEntry {
  std::vector<int64_t> A;
  int m = 0, n = 0, d = 0, lll = 1;
  std::vector<int64_t> B;
  std::vector<double> P;
  graver_status st = GRAVER_OK;
  std::string err;
  bool ready = false;
};

struct Req {
  int64_t id = 0;
  int m = 0, n = 0;
  std::vector<int64_t> A, b, l, u, xs;
  int f_kind = 0, f_degree = 0;
  std::vector<double> Q, c, coef;
  graver_extract_params ex{};
  graver_init_params ini{};
  int64_t max_steps = 0;
  int lll = 1, nxs = 0;
  std::shared_ptr<BasisEntry> basis;
  size_t footprint = 0;
  bool done = false;
  std::atomic<bool> cancel{false};  // graver_server_cancel was called before it finished
  graver_result res{};
  std::vector<int64_t> x_best;
};

}  // namespace
}  // namespace graver

struct graver_server {
  graver_server_params prm{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_prep, cv_ready, cv_done;
  std::deque<std::shared_ptr<graver::Req>> queued, ready;
  std::map<int64_t, std::shared_ptr<graver::Req>> all;
  std::map<std::string, std::shared_ptr<graver::BasisEntry>> bases;
  int64_t next_id = 1;
  size_t used = 0;
  int in_flight = 0;  // requests admitted and not done
  int64_t unfinished = 0;
  bool stop = false;
  std::vector<std::thread> threads;
};

namespace graver {
namespace {

double now_s(graver_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

// Estimated device bytes of one request (inputs, extraction, filter,
// initial solutions, augmentation).
size_t footprint(const Req& r, int d) {
  const size_t n = r.n, m = r.m, N = r.ex.n_starts, cap = r.ex.pool_capacity;
  const size_t stride = (n + 15) / 16 * 16, dpad = (d + 15) / 16 * 16 + 16;
  size_t b = 8 * (m * n + m + 2 * n + 2 * n * d);
  b += r.f_kind == GRAVER_F_QUADRATIC ? 8 * (n * n + n) : 8 * n * (r.f_degree + 1);
  b += 24 * N * d + 8 * N * n + 24 * N * dpad + N * stride;   // state, starts, scratch
  b += cap * (3 * stride + n + 24);                            // pool, log, table, keys out
  b += 4 * cap * stride;                                       // filter
  const size_t S = r.ini.n_starts + r.nxs;
  b += S * n * 40;                                             // initial solutions, augmentation
  return b + (64 << 20);
}

void basis_worker(graver_server* s) {
  for (;;) {
    std::shared_ptr<Req> r;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_prep.wait(lk, [&] { return s->stop || !s->queued.empty(); });
      if (s->queued.empty()) return;
      r = s->queued.front();
      s->queued.pop_front();
    }
    std::string key(reinterpret_cast<const char*>(r->A.data()), r->A.size() * sizeof(int64_t));
    key += std::to_string(r->m) + "x" + std::to_string(r->n) + (r->lll ? "L" : "H");
    std::shared_ptr<BasisEntry> e;
    bool compute = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      auto it = s->bases.find(key);
      if (it == s->bases.end()) {
        e = std::make_shared<BasisEntry>();
        s->bases[key] = e;
        compute = true;
      } else {
        e = it->second;
        r->res.reused_basis = 1;
      }
    }
    if (compute) {
      std::vector<int64_t> B((size_t)r->n * r->n);
      std::vector<double> P((size_t)r->n * r->n);
      int32_t d = 0;
      graver_status st = kernel_basis_host(r->m, r->n, r->A.data(), r->lll, B.data(), &d, P.data());
      std::unique_lock<std::mutex> lk(s->mu);
      e->st = st;
      if (st != GRAVER_OK) e->err = graver_last_error();
      e->d = d;
      B.resize((size_t)r->n * d);
      P.resize((size_t)d * r->n);
      e->B = std::move(B);
      e->P = std::move(P);
      e->ready = true;
      s->cv_prep.notify_all();
    } else {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_prep.wait(lk, [&] { return e->ready; });
    }
    std::unique_lock<std::mutex> lk(s->mu);
    r->basis = e;
    r->res.t_ready = now_s(s);
    if (r->cancel || e->st != GRAVER_OK || e->d < 1) {
      r->res.status = r->cancel ? GRAVER_E_CANCELLED : e->st != GRAVER_OK ? e->st : GRAVER_E_INVALID;
      r->done = true;
      r->res.t_done = now_s(s);
      --s->unfinished;
      s->cv_done.notify_all();
      continue;
    }
    r->footprint = footprint(*r, e->d);
    s->ready.push_back(r);
    s->cv_ready.notify_all();
  }
}

struct DevBuf {
  std::vector<void*> ptrs;
  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  ~DevBuf() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

struct Live {
  std::shared_ptr<Req> r;
  graver_problem prob{};
  graver_objective obj{};
  int8_t* keys = nullptr;
  int64_t count = 0;
  graver_extract_stats est{};
};

template <class T>
T* upload(DevBuf& db, hipStream_t s, const std::vector<T>& v) {
  T* p = db.alloc<T>(v.size());
  // a failed copy is reported like a failed allocation (nullptr)
  if (p && !v.empty() && hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess)
    return nullptr;
  return p;
}

// Filter, initial solutions, augmentation and best-of for one request whose
// candidates are in L.keys (everything on ctx's stream).
graver_status finish_request(graver_ctx* ctx, Live& L, DevBuf& db) {
  Req& r = *L.r;
  hipStream_t s = ctx->stream;
  const int n = r.n;
  graver_status st;
  int8_t* F = db.alloc<int8_t>((size_t)std::max<int64_t>(L.count, 1) * n);
  if (!F) return set_error(GRAVER_E_NOMEM, "device allocation failed");
  int64_t K = 0;
  if ((st = graver_filter(ctx, n, L.count ? L.keys : nullptr, L.count, F, L.count, &K)) != GRAVER_OK) return st;
  r.res.filtered = K;
  const int64_t S = r.ini.n_starts;
  int64_t* sol = db.alloc<int64_t>((size_t)std::max<int64_t>(S, 1) * n);
  int32_t* feas = db.alloc<int32_t>((size_t)std::max<int64_t>(S, 1));
  if (!sol || !feas) return set_error(GRAVER_E_NOMEM, "device allocation failed");
  int64_t nfeas = 0;
  if (S > 0 && (st = graver_init_solutions(ctx, &L.prob, &r.ini, nullptr, nullptr, sol, feas, &nfeas)) != GRAVER_OK)
    return st;
  r.res.feasible_starts = nfeas;
  std::vector<int32_t> hf((size_t)std::max<int64_t>(S, 0));
  if (S > 0) {
    HIP_TRY(hipMemcpyAsync(hf.data(), feas, S * sizeof(int32_t), hipMemcpyDeviceToHost, s), "feasibility flags");
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "feasibility flags");
  }
  std::vector<int64_t> hsol;
  if (nfeas > 0) {
    hsol.resize((size_t)S * n);
    HIP_TRY(hipMemcpyAsync(hsol.data(), sol, hsol.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s),
            "initial solutions");
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "initial solutions");
  }
  std::vector<int64_t> starts;
  for (int64_t k = 0; k < S; ++k)
    if (hf[k]) starts.insert(starts.end(), hsol.begin() + k * n, hsol.begin() + (k + 1) * n);
  starts.insert(starts.end(), r.xs.begin(), r.xs.end());
  const int32_t S2 = (int32_t)(starts.size() / n);
  if (S2 == 0) return set_error(GRAVER_E_INFEASIBLE_START, "no initial solution is feasible and no x_starts");
  int64_t* dst = upload(db, s, starts);
  int64_t* xo = db.alloc<int64_t>((size_t)S2 * n);
  double* fo = db.alloc<double>(S2);
  int64_t* so = db.alloc<int64_t>(S2);
  if (!dst || !xo || !fo || !so) return set_error(GRAVER_E_NOMEM, "device allocation failed");
  graver_augment_params ap{r.max_steps};
  int32_t best = -1;
  if ((st = graver_augment(ctx, &L.prob, &L.obj, K ? F : nullptr, K, S2, dst, &ap, xo, fo, so, &best)) != GRAVER_OK)
    return st;
  std::vector<int64_t> hs(S2);
  r.x_best.assign(n, 0);
  double fb = 0.0;
  HIP_TRY(hipMemcpyAsync(hs.data(), so, S2 * sizeof(int64_t), hipMemcpyDeviceToHost, s), "best-of");
  HIP_TRY(hipMemcpyAsync(&fb, fo + best, sizeof(double), hipMemcpyDeviceToHost, s), "best-of");
  HIP_TRY(hipMemcpyAsync(r.x_best.data(), xo + (size_t)best * n, n * sizeof(int64_t), hipMemcpyDeviceToHost, s),
          "best-of");
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "best-of");
  r.res.f_best = fb;
  for (int64_t v : hs) r.res.augment_steps += v;
  return GRAVER_OK;
}

void gpu_worker(graver_server* s) {
  (void)hipSetDevice(s->prm.device);  // graver_ctx_create below checks the device
  graver_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  const bool ok = graver_ctx_create(&ctx, s->prm.device) == GRAVER_OK &&
                  hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
  if (ok) graver_ctx_set_stream(ctx, stream);
  for (;;) {
    std::vector<std::shared_ptr<Req>> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_ready.wait(lk, [&] {
        if (s->stop && s->ready.empty()) return true;
        if (s->ready.empty()) return false;
        const auto& f = s->ready.front();
        // admit when it fits, or when nothing else holds memory
        return s->used + f->footprint <= (size_t)s->prm.hbm_budget || s->in_flight == 0;
      });
      if (s->ready.empty()) break;
      while (!s->ready.empty() && (int)batch.size() < s->prm.max_batch) {
        auto& f = s->ready.front();
        if (!batch.empty() && s->used + f->footprint > (size_t)s->prm.hbm_budget) break;
        if (batch.empty() && s->in_flight > 0 && s->used + f->footprint > (size_t)s->prm.hbm_budget) break;
        s->used += f->footprint;
        ++s->in_flight;
        f->res.t_admit = now_s(s);
        batch.push_back(f);
        s->ready.pop_front();
      }
    }
    if (batch.empty()) continue;
    if ((int)batch.size() < s->prm.max_batch && s->prm.batch_window_us > 0) {
      // batching window: more requests may become ready shortly
      const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(s->prm.batch_window_us);
      std::unique_lock<std::mutex> lk(s->mu);
      while ((int)batch.size() < s->prm.max_batch) {
        if (s->ready.empty()) {
          if (s->cv_ready.wait_until(lk, until) == std::cv_status::timeout && s->ready.empty()) break;
          continue;
        }
        auto& f = s->ready.front();
        if (s->used + f->footprint > (size_t)s->prm.hbm_budget) break;
        s->used += f->footprint;
        ++s->in_flight;
        f->res.t_admit = now_s(s);
        batch.push_back(f);
        s->ready.pop_front();
      }
    }
    {
      DevBuf db;
      std::vector<Live> live(batch.size());
      graver_status bst = ok ? GRAVER_OK : GRAVER_E_DEVICE;
      for (size_t i = 0; i < batch.size() && bst == GRAVER_OK; ++i) {
        Req& r = *batch[i];
        Live& L = live[i];
        L.r = batch[i];
        r.res.batch_size = (int32_t)batch.size();
        r.res.d = r.basis->d;
        L.prob.m = r.m;
        L.prob.n = r.n;
        L.prob.d = r.basis->d;
        L.prob.A = upload(db, stream, r.A);
        L.prob.b = upload(db, stream, r.b);
        L.prob.l = upload(db, stream, r.l);
        L.prob.u = upload(db, stream, r.u);
        L.prob.B = upload(db, stream, r.basis->B);
        L.prob.P = upload(db, stream, r.basis->P);
        L.obj.kind = r.f_kind;
        L.obj.degree = r.f_degree;
        L.obj.Q = r.Q.empty() ? nullptr : upload(db, stream, r.Q);
        L.obj.c = r.c.empty() ? nullptr : upload(db, stream, r.c);
        L.obj.coef = r.coef.empty() ? nullptr : upload(db, stream, r.coef);
        L.keys = db.alloc<int8_t>((size_t)r.ex.pool_capacity * r.n);
        if (!L.prob.A || !L.prob.B || !L.keys) bst = set_error(GRAVER_E_NOMEM, "device allocation failed");
      }
      if (bst == GRAVER_OK && hipStreamSynchronize(stream) != hipSuccess)
        bst = set_error(GRAVER_E_DEVICE, "uploading the batch's instances failed");
      // one batched extraction; on failure every request is retried alone so
      // that one request's error does not fail the others
      if (bst == GRAVER_OK) {
        const int k = (int)batch.size();
        std::vector<graver_problem> probs(k);
        std::vector<graver_extract_params> prms(k);
        std::vector<int8_t*> kout(k);
        std::vector<int64_t> kcap(k), cnt(k, 0);
        std::vector<graver_extract_stats> est(k);
        for (int i = 0; i < k; ++i) {
          probs[i] = live[i].prob;
          prms[i] = batch[i]->ex;
          prms[i].any_order = 1;  // the filter sorts
          kout[i] = live[i].keys;
          kcap[i] = batch[i]->ex.pool_capacity;
        }
        graver_batch_params bp{s->prm.autotune, s->prm.use_graph};
        graver_batch_stats bs{};
        graver_status est_all = graver_extract_batch(ctx, k, probs.data(), prms.data(), nullptr, kout.data(),
                                                     kcap.data(), cnt.data(), est.data(), &bp, &bs);
        for (int i = 0; i < k; ++i) {
          Live& L = live[i];
          Req& r = *L.r;
          graver_status st = est_all;
          if (est_all == GRAVER_OK) {
            L.count = cnt[i];
            L.est = est[i];
          } else {
            graver_extract_params ex = r.ex;
            ex.any_order = 1;
            st = graver_extract(ctx, &L.prob, &ex, nullptr, L.keys, r.ex.pool_capacity, &L.count, &L.est);
          }
          if (st == GRAVER_OK) {
            r.res.unique = L.count;
            // a request cancelled while its extraction ran skips the rest
            st = r.cancel ? GRAVER_E_CANCELLED : finish_request(ctx, L, db);
          }
          r.res.status = r.cancel ? GRAVER_E_CANCELLED : st;
        }
      } else {
        for (auto& r : batch) r->res.status = bst;
      }
      // release the batch's device memory (request buffers and workspaces)
      (void)hipStreamSynchronize(stream);  // each request already holds its status
      ws_free(ctx->ws);
      for (Ws* w : ctx->batch_ws) ws_free(*w);
    }
    std::unique_lock<std::mutex> lk(s->mu);
    for (auto& r : batch) {
      s->used -= r->footprint;
      --s->in_flight;
      r->done = true;
      r->res.t_done = now_s(s);
      --s->unfinished;
    }
    s->cv_done.notify_all();
    s->cv_ready.notify_all();
  }
  if (ctx) graver_ctx_destroy(ctx);
  if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace
}  // namespace graver

using namespace graver;

extern "C" graver_status graver_server_create(graver_server** out, const graver_server_params* prm) {
  if (!out || !prm) return set_error(GRAVER_E_INVALID, "NULL argument");
  *out = nullptr;
  if (prm->hbm_budget < 1 || prm->max_batch < 1 || prm->gpu_workers < 1 || prm->host_threads < 1 ||
      prm->gpu_workers > 16 || prm->host_threads > 256)
    return set_error(GRAVER_E_INVALID, "bad server parameters");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || prm->device < 0 || prm->device >= count)
    return set_error(GRAVER_E_INVALID, "no such device");
  auto* s = new graver_server();
  s->prm = *prm;
  s->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < prm->host_threads; ++i) s->threads.emplace_back(basis_worker, s);
  for (int i = 0; i < prm->gpu_workers; ++i) s->threads.emplace_back(gpu_worker, s);
  *out = s;
  return GRAVER_OK;
}

extern "C" graver_status graver_server_submit(graver_server* s, const graver_request* q, int64_t* ticket) {
  if (!s || !q || !ticket) return set_error(GRAVER_E_INVALID, "NULL argument");
  if (q->m < 1 || q->n < 1 || q->n > 4096 || !q->A || !q->b || !q->l || !q->u)
    return set_error(GRAVER_E_INVALID, "bad request shape or pointers");
  if (q->f_kind == GRAVER_F_QUADRATIC ? (!q->Q || !q->c)
                                      : (q->f_kind != GRAVER_F_SEPARABLE_POLY || !q->coef || q->f_degree < 0 ||
                                         q->f_degree > 8))
    return set_error(GRAVER_E_INVALID, "bad objective");
  if (q->extract.init_mode != 0 || !q->extract.collect || q->extract.pool_capacity < 1 || q->n_x_starts < 0 ||
      (q->n_x_starts > 0 && !q->x_starts))
    return set_error(GRAVER_E_INVALID, "requests use init_mode 0, collect 1, pool_capacity >= 1");
  auto r = std::make_shared<Req>();
  const size_t m = q->m, n = q->n;
  r->m = q->m;
  r->n = q->n;
  r->A.assign(q->A, q->A + m * n);
  r->b.assign(q->b, q->b + m);
  r->l.assign(q->l, q->l + n);
  r->u.assign(q->u, q->u + n);
  r->f_kind = q->f_kind;
  r->f_degree = q->f_degree;
  if (q->f_kind == GRAVER_F_QUADRATIC) {
    r->Q.assign(q->Q, q->Q + n * n);
    r->c.assign(q->c, q->c + n);
  } else {
    r->coef.assign(q->coef, q->coef + n * (q->f_degree + 1));
  }
  r->ex = q->extract;
  r->ini = q->init;
  r->max_steps = q->max_steps;
  r->lll = q->lll;
  r->nxs = q->n_x_starts;
  if (q->n_x_starts > 0) r->xs.assign(q->x_starts, q->x_starts + (size_t)q->n_x_starts * n);
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stop) return set_error(GRAVER_E_INVALID, "server is stopping");
  r->id = s->next_id++;
  r->res.t_submit = now_s(s);
  s->all[r->id] = r;
  ++s->unfinished;
  s->queued.push_back(r);
  s->cv_prep.notify_one();
  *ticket = r->id;
  return GRAVER_OK;
}

extern "C" graver_status graver_server_wait(graver_server* s, int64_t ticket, graver_result* res, int64_t* x_best) {
  if (!s || !res) return set_error(GRAVER_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return set_error(GRAVER_E_INVALID, "unknown ticket");
  std::shared_ptr<Req> r = it->second;
  s->cv_done.wait(lk, [&] { return r->done; });
  *res = r->res;
  if (x_best && !r->x_best.empty()) std::memcpy(x_best, r->x_best.data(), r->x_best.size() * sizeof(int64_t));
  s->all.erase(it);
  return GRAVER_OK;
}

extern "C" graver_status graver_server_poll(graver_server* s, int64_t ticket, int32_t* done, graver_result* res,
                                            int64_t* x_best) {
  if (!s || !done || !res) return set_error(GRAVER_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return set_error(GRAVER_E_INVALID, "unknown ticket");
  std::shared_ptr<Req> r = it->second;
  *done = r->done ? 1 : 0;
  if (!r->done) return GRAVER_OK;
  *res = r->res;
  if (x_best && !r->x_best.empty()) std::memcpy(x_best, r->x_best.data(), r->x_best.size() * sizeof(int64_t));
  s->all.erase(it);
  return GRAVER_OK;
}

extern "C" graver_status graver_server_cancel(graver_server* s, int64_t ticket, int32_t* cancelled) {
  if (!s || !cancelled) return set_error(GRAVER_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return set_error(GRAVER_E_INVALID, "unknown ticket");
  std::shared_ptr<Req> r = it->second;
  if (r->done) {
    *cancelled = 0;
    return GRAVER_OK;
  }
  r->cancel = true;
  *cancelled = 1;
  // still waiting for a basis worker or for admission: it holds no device
  // memory, so it leaves its queue and finishes now; otherwise the worker
  // that holds it ends it at its next stage boundary
  for (auto* q : {&s->queued, &s->ready}) {
    auto qi = std::find(q->begin(), q->end(), r);
    if (qi == q->end()) continue;
    q->erase(qi);
    r->res.status = GRAVER_E_CANCELLED;
    r->res.t_done = now_s(s);
    r->done = true;
    --s->unfinished;
    s->cv_done.notify_all();
    s->cv_ready.notify_all();
    break;
  }
  return GRAVER_OK;
}

extern "C" void graver_server_destroy(graver_server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->unfinished == 0; });
    s->stop = true;
    s->cv_prep.notify_all();
    s->cv_ready.notify_all();
  }
  for (auto& t : s->threads) t.join();
  delete s;
}
