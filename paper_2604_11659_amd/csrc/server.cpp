// Request loop with continuous batching for encrypted sparse matmuls.
//
// A worker thread owns a HIP stream. Requests (an encrypted CSR operand and an encrypted CSC
// operand already resident on the device) are queued by fhe_server_submit and admitted while the
// number in flight is below max_inflight and their result buffers fit the HBM budget. Every
// scheduling step takes the next slice of products (with all their matched pairs) from every
// request in flight and runs them as ONE merged launch stream, so requests that arrive while others
// are running join the very next step and their work shares launches with the older ones. A request
// completes when its last slice has been accumulated; its latency is submit -> completion. With a
// grouped plan (fhe_server_set_plan) a request's slice is the whole request, since its groups span
// all of its products; requests still join the next step and share its launches.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
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
    std::unique_ptr<fhe_mat> C;
    Job job{};
    int32_t next_prod = 0;
    double t_submit = 0, t_done = 0;
    int state = 0;  // 0 queued, 1 in flight, 2 done, 3 failed
    size_t bytes = 0;
    int err = 0;
    std::string msg;
  };
  fhe_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  int max_inflight = 1;
  int slice_products = 64;
  int plan_mode = FHE_PLAN_PER_PAIR;  // FHE_PLAN_* (grouped and tree plans run each request whole)
  bool hoist = false;
  size_t max_queue = 1024;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  bool stop = false;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> active;
  size_t used = 0;
  uint64_t next_ticket = 1;
  std::vector<double> latencies;
  std::thread worker;

  void finish(Req* r, int state, int err, const std::string& msg) {
    r->state = state;
    r->err = err;
    r->msg = msg;
    r->t_done = now_s();
    if (state == 2) latencies.push_back(r->t_done - r->t_submit);
    used -= r->bytes;
    active.erase(std::remove(active.begin(), active.end(), r->ticket), active.end());
  }

  void run() {
    (void)hipSetDevice(ctx->device);
    for (;;) {
      std::vector<Req*> fresh;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
        if (stop) {  // closing: requests not yet admitted are cancelled, admitted ones run to the end
          for (uint64_t t : queue) {
            Req* r = reqs[t].get();
            r->state = 3;
            r->err = FHE_EAGAIN;
            r->msg = "server closed before the request was admitted";
            r->t_done = now_s();
          }
          queue.clear();
          done_cv.notify_all();
          if (active.empty()) return;
        }
        // Admission: by slot and by HBM budget for the result buffers.
        while (!queue.empty() && (int)active.size() < max_inflight) {
          Req* r = reqs[queue.front()].get();
          if (r->bytes > budget) {
            queue.pop_front();
            r->state = 3;
            r->err = FHE_ENOMEM;
            r->msg = "request result does not fit the server's HBM budget";
            r->t_done = now_s();
            done_cv.notify_all();
            continue;
          }
          if (used + r->bytes > budget) break;
          queue.pop_front();
          used += r->bytes;
          r->state = 1;
          active.push_back(r->ticket);
          fresh.push_back(r);
        }
      }
      for (Req* r : fresh) {
        try {
          prepare_result(ctx, r->job, stream);
        } catch (const Error& e) {
          std::lock_guard<std::mutex> lk(mu);
          finish(r, 3, e.code, e.msg);
          done_cv.notify_all();
        }
      }
      std::vector<Slice> slices;
      std::vector<Req*> in_step;
      {
        std::lock_guard<std::mutex> lk(mu);
        for (uint64_t t : active) {
          Req* r = reqs[t].get();
          const int32_t np = (int32_t)r->job.plan.prods.size();
          // grouped plans sum over all the pairs of a request at once: one slice per request
          const int32_t hi = plan_mode == FHE_PLAN_PER_PAIR ? std::min(np, r->next_prod + slice_products) : np;
          slices.push_back(Slice{&r->job, r->next_prod, hi});
          in_step.push_back(r);
        }
      }
      if (in_step.empty()) continue;
      int err = 0;
      std::string msg;
      try {
        execute_slices(ctx, slices, stream, plan_mode == FHE_PLAN_GROUPED, false, plan_mode == FHE_PLAN_TREE, hoist);
      } catch (const Error& e) {
        err = e.code;
        msg = e.msg;
      }
      std::lock_guard<std::mutex> lk(mu);
      for (size_t i = 0; i < in_step.size(); ++i) {
        Req* r = in_step[i];
        if (err) {
          finish(r, 3, err, msg);
          continue;
        }
        r->next_prod = slices[i].hi;
        if (r->next_prod >= (int32_t)r->job.plan.prods.size()) finish(r, 2, 0, "");
      }
      done_cv.notify_all();
    }
  }
};

extern "C" {

int fhe_server_create(fhe_ctx* ctx, size_t hbm_budget, int32_t max_inflight, int32_t slice_products,
                      int32_t max_queue, fhe_server** out) {
  if (!ctx || !out || max_inflight < 1 || slice_products < 1 || max_queue < 1) return FHE_EINVAL;
  *out = nullptr;
  std::unique_ptr<fhe_server> s(new fhe_server());
  s->ctx = ctx;
  s->budget = hbm_budget;
  s->max_inflight = max_inflight;
  s->slice_products = slice_products;
  s->max_queue = (size_t)max_queue;
  if (hipSetDevice(ctx->device) != hipSuccess) return FHE_EDEVICE;
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) return FHE_EDEVICE;
  fhe_server* raw = s.get();
  s->worker = std::thread([raw] { raw->run(); });
  *out = s.release();
  return FHE_OK;
}

int fhe_server_set_plan(fhe_server* s, int32_t mode) {
  if (!s) return FHE_EINVAL;
  const int32_t plan = mode & ~FHE_PLAN_HOIST;
  if (plan != FHE_PLAN_PER_PAIR && plan != FHE_PLAN_GROUPED && plan != FHE_PLAN_TREE) return FHE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->next_ticket != 1) return FHE_EAGAIN;  // only before the first request
  s->plan_mode = plan;
  s->hoist = (mode & FHE_PLAN_HOIST) != 0;
  return FHE_OK;
}

int fhe_server_submit(fhe_server* s, const fhe_mat* A, const fhe_mat* B, uint64_t* ticket) {
  if (!s || !A || !B || !ticket) return FHE_EINVAL;
  if (A->kind != 0 || B->kind != 1) return FHE_EINVAL;
  if (A->cols != B->rows) return FHE_ESHAPE;
  std::unique_ptr<fhe_server::Req> r(new fhe_server::Req());
  r->C.reset(new fhe_mat());
  try {
    r->job = Job{A, B, build_plan(s->ctx->p, A, B, 0, INT64_MAX), r->C.get()};
  } catch (const Error& e) {
    return e.code;
  }
  index_plan(r->job.plan);
  r->bytes = (size_t)r->job.plan.nres * 2 * (s->ctx->p.nq - 2) * s->ctx->p.N * 8;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->queue.size() >= s->max_queue) return FHE_EAGAIN;
  r->ticket = s->next_ticket++;
  r->t_submit = now_s();
  *ticket = r->ticket;
  s->queue.push_back(r->ticket);
  s->reqs[r->ticket] = std::move(r);
  s->cv.notify_all();
  return FHE_OK;
}

int fhe_server_poll(fhe_server* s, uint64_t ticket, int32_t wait_ms, fhe_mat** C_out, double* latency_s) {
  if (!s || !C_out) return FHE_EINVAL;
  *C_out = nullptr;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return FHE_EINVAL;
  fhe_server::Req* r = it->second.get();
  if (r->state < 2 && wait_ms > 0)
    s->done_cv.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return r->state >= 2; });
  if (r->state < 2) return FHE_EAGAIN;
  int rc = FHE_OK;
  if (r->state == 2) {
    *C_out = r->C.release();
    if (latency_s) *latency_s = r->t_done - r->t_submit;
  } else {
    rc = r->err ? r->err : FHE_EDEVICE;
  }
  s->reqs.erase(it);
  return rc;
}

int fhe_server_stats(fhe_server* s, double* p50_s, double* p99_s, int64_t* completed, int64_t* inflight,
                     int64_t* queued) {
  if (!s) return FHE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> v = s->latencies;
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) -> double {
    if (v.empty()) return 0.0;
    size_t i = (size_t)std::ceil(q * (double)v.size()) - 1;
    return v[std::min(i, v.size() - 1)];
  };
  if (p50_s) *p50_s = pct(0.50);
  if (p99_s) *p99_s = pct(0.99);
  if (completed) *completed = (int64_t)v.size();
  if (inflight) *inflight = (int64_t)s->active.size();
  if (queued) *queued = (int64_t)s->queue.size();
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
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
