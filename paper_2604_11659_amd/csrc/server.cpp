// Request loop with continuous batching for encrypted sparse matmuls over several parameter sets.
//
// One worker thread owns a HIP stream and serves the requests of every context it was created with
// (for instance an N = 2^16 and an N = 2^17 parameter set, each with its keys resident). Requests (an
// encrypted CSR operand and an encrypted CSC operand already on the device, plus the context they
// belong to) wait in one FIFO queue and are admitted while fewer than max_inflight run and their
// memory fits the one HBM budget the server shares across its contexts. Every scheduling step takes,
// for each context, the next slice of products (with all their matched pairs) of every admitted
// request of that context and runs them as ONE merged launch stream, so requests that arrive while
// others run join the very next step and share its launches. A request completes when its last slice
// has been accumulated; its latency is submit -> completion.
//
// Memory accounting against the budget:
//   * fixed, charged at creation: every context's tables and evaluation keys (resident), the executor
//     scratch of each context (the server caps it; all requests of a context share it within a step)
//     and, for grouped plans, the tail's second ping-pong buffers;
//   * per request, charged at admission and released at completion: its result chunks and, for
//     grouped plans, its resident products and digit-tree partial sums.
// A request whose own charge exceeds what the budget leaves after the fixed part is refused at submit.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <thread>

#include "spmspm.h"

using namespace fhe;

namespace {
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

struct fhe_server {
  struct Req {
    uint64_t ticket = 0;
    int ctx_id = 0;
    std::unique_ptr<fhe_mat> C;
    Job job{};
    int32_t next_prod = 0;
    double t_submit = 0, t_done = 0;
    int state = 0;  // 0 queued, 1 in flight, 2 done, 3 failed, 4 cancelled
    bool cancel = false;    // cancelled while in flight: stops at the next step boundary
    bool planned = false;   // Algorithm 1's plan built (at submission for grouped plans, else at admission)
    size_t bytes = 0;       // charged while in flight
    size_t group_bytes = 0; // grouped plans: its resident products (part of `bytes`)
    int err = 0;
    std::string msg;
  };
  struct Ctx {
    fhe_ctx* ctx = nullptr;
    size_t ws_bytes = 0;    // executor scratch cap
    size_t tail_bytes = 0;  // grouped plans: the tail's second ping-pong buffers
  };
  std::vector<Ctx> ctxs;
  hipStream_t stream = nullptr;
  size_t budget = 0, fixed = 0, used = 0;
  int max_inflight = 1;
  int slice_products = 64;
  int plan_mode = FHE_PLAN_PER_PAIR;  // FHE_PLAN_* (grouped and tree plans run each request whole)
  bool hoist = false;
  size_t max_queue = 1024;
  std::mutex mu;
  std::condition_variable cv, done_cv, gone_cv;
  bool stop = false, closing = false;
  int waiters = 0;  // threads inside fhe_server_poll
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> active;
  uint64_t next_ticket = 1;
  std::vector<double> latencies;
  int64_t n_failed = 0, n_cancelled = 0, n_steps = 0, max_merged = 0, max_step_requests = 0;
  std::thread worker;

  bool grouped() const { return plan_mode != FHE_PLAN_PER_PAIR; }

  void finish(Req* r, int state, int err, const std::string& msg) {
    r->state = state;
    r->err = err;
    r->msg = msg;
    r->t_done = now_s();
    if (state == 2) latencies.push_back(r->t_done - r->t_submit);
    if (state == 3) ++n_failed;
    if (state == 4) ++n_cancelled;
    if (state != 2 && r->C) r->C->data.reset();  // no result to hand out: release it with the charge
    used -= r->bytes;
    active.erase(std::remove(active.begin(), active.end(), r->ticket), active.end());
  }

  void run() {
    (void)hipSetDevice(ctxs[0].ctx->device);
    for (;;) {
      std::vector<Req*> fresh;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
        if (stop) {  // closing: requests not yet admitted are cancelled, admitted ones run to the end
          for (uint64_t t : queue) {
            Req* r = reqs[t].get();
            r->state = 4;
            r->err = FHE_ECANCELED;
            r->msg = "server closed before the request was admitted";
            r->t_done = now_s();
            ++n_cancelled;
          }
          queue.clear();
          done_cv.notify_all();
          if (active.empty()) return;
        }
        // Admission in arrival order: by slot and by the shared HBM budget.
        while (!queue.empty() && (int)active.size() < max_inflight) {
          Req* r = reqs[queue.front()].get();
          if (fixed + used + r->bytes > budget) break;
          queue.pop_front();
          used += r->bytes;
          r->state = 1;
          active.push_back(r->ticket);
          fresh.push_back(r);
        }
      }
      for (Req* r : fresh) {
        try {
          if (!r->planned) {  // Algorithm 1's merge on the host, then the result chunks on the device
            r->job.plan = build_plan(ctxs[r->ctx_id].ctx->p, r->job.A, r->job.B, 0, INT64_MAX);
            index_plan(r->job.plan);
            r->planned = true;
          }
          prepare_result(ctxs[r->ctx_id].ctx, r->job, stream);
        } catch (const Error& e) {
          std::lock_guard<std::mutex> lk(mu);
          finish(r, 3, e.code, e.msg);
          done_cv.notify_all();
        }
      }
      // One merged launch stream per context with requests in flight.
      std::vector<std::vector<Slice>> slices(ctxs.size());
      std::vector<std::vector<Req*>> in_step(ctxs.size());
      {
        std::lock_guard<std::mutex> lk(mu);
        for (size_t ai = 0; ai < active.size();) {
          Req* r = reqs[active[ai]].get();
          if (r->cancel) {  // cancelled while in flight: its partial result is dropped
            finish(r, 4, FHE_ECANCELED, "request cancelled");
            done_cv.notify_all();
            continue;  // finish() removed it from `active`
          }
          ++ai;
          const int32_t np = (int32_t)r->job.plan.prods.size();
          // grouped plans sum over all the pairs of a request at once: one slice per request
          const int32_t hi = grouped() ? np : std::min(np, r->next_prod + slice_products);
          slices[r->ctx_id].push_back(Slice{&r->job, r->next_prod, hi});
          in_step[r->ctx_id].push_back(r);
        }
      }
      int64_t step_requests = 0;
      for (size_t c = 0; c < ctxs.size(); ++c) {
        if (in_step[c].empty()) continue;
        step_requests += (int64_t)in_step[c].size();
        ExecOpts o;
        o.grouped = plan_mode == FHE_PLAN_GROUPED;
        o.tree = plan_mode == FHE_PLAN_TREE;
        o.hoist = hoist;
        o.ws_bytes = ctxs[c].ws_bytes;
        if (grouped()) {  // every product of the step resident (charged per request)
          size_t g = 0;
          for (Req* r : in_step[c]) g += r->group_bytes;
          o.group_bytes = std::max<size_t>(g, 1);
        }
        int err = 0;
        std::string msg;
        try {
          execute_slices(ctxs[c].ctx, slices[c], stream, o);
        } catch (const Error& e) {
          err = e.code;
          msg = e.msg;
        }
        std::lock_guard<std::mutex> lk(mu);
        max_merged = std::max<int64_t>(max_merged, (int64_t)in_step[c].size());
        for (size_t i = 0; i < in_step[c].size(); ++i) {
          Req* r = in_step[c][i];
          if (err) {
            finish(r, 3, err, msg);
            continue;
          }
          r->next_prod = slices[c][i].hi;
          if (r->next_prod >= (int32_t)r->job.plan.prods.size()) finish(r, 2, 0, "");
        }
        done_cv.notify_all();
      }
      std::lock_guard<std::mutex> lk(mu);
      if (step_requests) {
        ++n_steps;
        max_step_requests = std::max(max_step_requests, step_requests);
      }
    }
  }
};

extern "C" {

int fhe_server_create(fhe_ctx* const* ctxs, size_t nctx, size_t hbm_budget, size_t workspace_bytes,
                      int32_t max_inflight, int32_t slice_products, int32_t max_queue, fhe_server** out) {
  if (!out) return set_error(FHE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctxs || nctx < 1 || max_inflight < 1 || slice_products < 1 || max_queue < 1)
    return set_error(FHE_EINVAL, "contexts, max_inflight, slice_products and max_queue must be given and >= 1");
  for (size_t c = 0; c < nctx; ++c) {
    if (!ctxs[c]) return set_error(FHE_EINVAL, "a context is NULL");
    if (ctxs[c]->device != ctxs[0]->device)  // one worker stream: one GPU
      return set_error(FHE_EINVAL, "the contexts of one server must be on one device");
  }
  std::unique_ptr<fhe_server> s(new fhe_server());
  s->budget = hbm_budget;
  s->max_inflight = max_inflight;
  s->slice_products = slice_products;
  s->max_queue = (size_t)max_queue;
  // Fixed part: tables and keys of every context, plus each context's executor scratch cap.
  size_t fixed = 0;
  for (size_t c = 0; c < nctx; ++c) fixed += ctx_resident_bytes(ctxs[c]);
  for (size_t c = 0; c < nctx; ++c) {
    fhe_ctx* ctx = ctxs[c];
    fhe_server::Ctx sc;
    sc.ctx = ctx;
    const WsPlan big = ws_plan(ctx, SIZE_MAX / 4, SIZE_MAX / 4, SIZE_MAX / 4);  // the 4096 / 8192 batch caps
    const WsPlan one = ws_plan(ctx, 0, 1, 1);                                     // one product, one pair
    size_t cap = workspace_bytes;
    if (!cap) {  // automatic: a quarter of what the budget leaves after the keys, shared by the contexts
      const size_t left = hbm_budget > fixed ? hbm_budget - fixed : 0;
      cap = left / (4 * nctx);
      const char* e = getenv("FHE_WORKSPACE_MB");
      cap = std::min(cap, (size_t)(e ? atoll(e) : 131072) << 20);
    }
    cap = std::max(cap, one.words * 8);
    cap = std::min(cap, big.words * 8);
    sc.ws_bytes = cap;
    const WsPlan w = ws_plan(ctx, cap, SIZE_MAX / 4, SIZE_MAX / 4);
    sc.tail_bytes = w.BB * 2 * (size_t)(ctx->p.nq - 1) * ctx->p.N * 8;
    {
      // the server owns the context's scratch from now on: drop a larger one left by earlier calls,
      // the grouped products kept by direct calls and the kept result blocks (the server charges
      // results and grouped products per request; blocks kept outside the budget would escape it)
      std::lock_guard<std::recursive_mutex> lk(ctx->exec_mu);
      ctx->results->clear(0);
      const bool drop_ws = ctx->ws_cache.bytes() > w.words * 8;
      if (drop_ws || ctx->group_cache.bytes()) {
        if (hipSetDevice(ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
          return set_error(FHE_EDEVICE, "device synchronisation failed");
        if (drop_ws) {
          ctx->graphs.clear();
          ctx->ws_cache.reset();
        }
        ctx->group_cache.reset();
      }
    }
    fixed += w.words * 8;
    s->ctxs.push_back(sc);
  }
  s->fixed = fixed;
  if (fixed > hbm_budget)
    return set_error(FHE_ENOMEM, "the budget is below the keys, tables and scratch the contexts hold");
  if (hipSetDevice(ctxs[0]->device) != hipSuccess) return set_error(FHE_EDEVICE, "hipSetDevice failed");
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
    return set_error(FHE_EDEVICE, "stream creation failed");
  fhe_server* raw = s.get();
  s->worker = std::thread([raw] { raw->run(); });
  *out = s.release();
  return FHE_OK;
}

int fhe_server_set_plan(fhe_server* s, int32_t mode) {
  if (!s) return set_error(FHE_EINVAL, "server is NULL");
  const int32_t plan = mode & ~FHE_PLAN_HOIST;
  if (plan != FHE_PLAN_PER_PAIR && plan != FHE_PLAN_GROUPED && plan != FHE_PLAN_TREE)
    return set_error(FHE_EINVAL, "unknown plan mode");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->next_ticket != 1)  // only before the first request
    return set_error(FHE_EAGAIN, "the plan mode can only be set before the first request");
  if (plan != FHE_PLAN_PER_PAIR) {  // the tail's second ping-pong buffers join the fixed part
    for (auto& c : s->ctxs) s->fixed += c.tail_bytes;
    if (s->fixed > s->budget) {
      for (auto& c : s->ctxs) s->fixed -= c.tail_bytes;
      return set_error(FHE_ENOMEM, "the grouped plan's extra buffers exceed the budget");
    }
  }
  s->plan_mode = plan;
  s->hoist = (mode & FHE_PLAN_HOIST) != 0;
  return FHE_OK;
}

int fhe_server_submit(fhe_server* s, int32_t ctx_id, const fhe_mat* A, const fhe_mat* B, uint64_t* ticket) {
  if (!s || !A || !B || !ticket) return set_error(FHE_EINVAL, "server, operands and ticket must be given");
  if (ctx_id < 0 || (size_t)ctx_id >= s->ctxs.size()) return set_error(FHE_EINVAL, "no such context id");
  if (A->kind != 0 || B->kind != 1) return set_error(FHE_EINVAL, "A must be a CSR operand and B a CSC operand");
  if (A->cols != B->rows) return set_error(FHE_ESHAPE, "A.cols != B.rows");
  const fhe_ctx* ctx = s->ctxs[ctx_id].ctx;
  std::unique_ptr<fhe_server::Req> r(new fhe_server::Req());
  r->ctx_id = ctx_id;
  r->C.reset(new fhe_mat());
  r->job = Job{A, B, Plan{}, r->C.get()};
  int mode;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    mode = s->plan_mode;
  }
  const int64_t S = ctx->p.S, nres = std::max<int64_t>(1, ((int64_t)A->rows * B->cols + S - 1) / S);
  r->bytes = (size_t)nres * 2 * (ctx->p.nq - 2) * ctx->p.N * 8;
  if (mode != FHE_PLAN_PER_PAIR) {  // the charge depends on the plan: build it now
    try {
      r->job.plan = build_plan(ctx->p, A, B, 0, INT64_MAX);
    } catch (const Error& e) {
      return set_error(e.code, e.msg.c_str());
    }
    index_plan(r->job.plan);
    r->planned = true;
    r->group_bytes = r->job.plan.prods.size() * 2 * (size_t)(ctx->p.nq - 1) * ctx->p.N * 8;
    r->bytes += grouped_resident_words(ctx->p, r->job.plan, mode == FHE_PLAN_TREE) * 8;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->plan_mode != mode) return set_error(FHE_EAGAIN, "the plan mode changed meanwhile");
  if (s->fixed + r->bytes > s->budget)  // would never fit, even alone
    return set_error(FHE_ENOMEM, "the request alone exceeds what the budget leaves after the fixed part");
  if (s->queue.size() >= s->max_queue) return set_error(FHE_EAGAIN, "the queue is full");
  r->ticket = s->next_ticket++;
  r->t_submit = now_s();
  *ticket = r->ticket;
  s->queue.push_back(r->ticket);
  s->reqs[r->ticket] = std::move(r);
  s->cv.notify_all();
  return FHE_OK;
}

int fhe_server_poll(fhe_server* s, uint64_t ticket, int32_t wait_ms, fhe_mat** C_out, double* latency_s) {
  if (!s || !C_out) return set_error(FHE_EINVAL, "server and C_out must be given");
  *C_out = nullptr;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(FHE_EINVAL, "unknown ticket");
  fhe_server::Req* r = it->second.get();
  if (r->state < 2 && wait_ms > 0 && !s->closing) {
    ++s->waiters;
    s->done_cv.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return r->state >= 2 || s->closing; });
    --s->waiters;
    s->gone_cv.notify_all();
  }
  if (r->state < 2) return set_error(FHE_EAGAIN, "the request has not finished");
  int rc = FHE_OK;
  if (r->state == 2) {
    *C_out = r->C.release();
    if (latency_s) *latency_s = r->t_done - r->t_submit;
  } else {
    rc = set_error(r->err ? r->err : FHE_EDEVICE, r->msg.c_str());
  }
  s->reqs.erase(it);
  return rc;
}

int fhe_server_cancel(fhe_server* s, uint64_t ticket) {
  if (!s) return set_error(FHE_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(FHE_EINVAL, "unknown ticket");
  fhe_server::Req* r = it->second.get();
  if (r->state >= 2) return FHE_OK;  // already finished: its outcome stands
  if (r->state == 0) {
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), ticket), s->queue.end());
    r->state = 4;
    r->err = FHE_ECANCELED;
    r->msg = "request cancelled";
    r->t_done = now_s();
    ++s->n_cancelled;
    s->done_cv.notify_all();
  } else {
    r->cancel = true;  // in flight: the worker drops it at the next step boundary
  }
  s->cv.notify_all();
  return FHE_OK;
}

int fhe_server_stats(fhe_server* s, fhe_server_info* out) {
  if (!s || !out) return set_error(FHE_EINVAL, "server and out must be given");
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> v = s->latencies;
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) -> double {
    if (v.empty()) return 0.0;
    size_t i = (size_t)std::ceil(q * (double)v.size()) - 1;
    return v[std::min(i, v.size() - 1)];
  };
  *out = fhe_server_info{};
  out->p50_s = pct(0.50);
  out->p99_s = pct(0.99);
  out->completed = (int64_t)v.size();
  out->failed = s->n_failed;
  out->cancelled = s->n_cancelled;
  out->inflight = (int64_t)s->active.size();
  out->queued = (int64_t)s->queue.size();
  out->steps = s->n_steps;
  out->max_merged = s->max_merged;
  out->max_step_requests = s->max_step_requests;
  out->budget_bytes = s->budget;
  out->fixed_bytes = s->fixed;
  out->inflight_bytes = s->used;
  return FHE_OK;
}

void fhe_server_free(fhe_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  {
    // every request is finished or cancelled now; wake the pollers still waiting and let them leave
    // before the server goes away
    std::unique_lock<std::mutex> lk(s->mu);
    s->closing = true;
    s->done_cv.notify_all();
    s->gone_cv.wait(lk, [&] { return s->waiters == 0; });
  }
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
