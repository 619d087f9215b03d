// serve.hip -- continuous-batching update server (include/damf_serve.h).
//
// One server thread owns the context.  Clients admit requests under a memory
// cap; the thread takes every admitted request that fits into the next step
// (up to max_step_ops / max_step_requests), concatenates them as request
// segments and runs one update step:
//
//   prepare (segments) -> chain kernel (stream A, async)
//       || Step 4 of the previous step (stream B: push rounds)
//   -> wait A -> PPR fix-up + CSR edits -> [re-orth] -> defer this step's Step 4
//
// The fix-up and the graph edits wait until the previous push has finished
// (the fix-up reads the PPR invariant row by row, and the push walks the
// in-CSR); the chain kernel only adds to R with atomics, so it may run beside
// the push.  A request completes when its step's push ends; with nothing
// queued the deferred push runs at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/damf_serve.h"
#include "damf_internal.h"

using namespace damf;

namespace {

constexpr int64_t kReqOverheadBytes = 64;

struct Req {
  int64_t ticket = 0, k = 0, bytes = 0;
  std::vector<int32_t> src, dst;
  std::vector<int8_t> op;
  double submit_us = 0, start_us = 0, done_us = 0;
  int64_t step = -1, net = 0, chunks = 0;
  int32_t step_requests = 0;
  damf_status status = DAMF_OK;
  bool done = false;
};

}  // namespace

struct damf_server {
  damf_ctx *c = nullptr;
  damf_server_config cfg{};
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> queue;                   // admitted, not started (under mu)
  std::unordered_map<int64_t, Req *> reqs;   // until waited (under mu)
  int64_t next_ticket = 1;
  int64_t admitted_bytes = 0, peak_bytes = 0;
  bool stop = false, paused = false;
  damf_status dead = DAMF_OK;                // set after a device error
  hipStream_t push_stream = nullptr;
  // deferred Step 4 (worker thread only)
  std::vector<Req *> pending;
  int64_t pending_rows = 0;
  bool pending_push = false;
  // pinned staging of one step's ops
  int32_t *h_src = nullptr, *h_dst = nullptr;
  int8_t *h_op = nullptr;
  // statistics (under mu)
  std::vector<double> lat_ms;
  int64_t ops_done = 0, steps = 0, busy = 0, step_reqs_sum = 0, step_ops_sum = 0;
  double first_submit_us = -1.0, last_done_us = 0.0, push_overlap_ms = 0.0;
  std::chrono::steady_clock::time_point t0;
  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
        .count();
  }
};

namespace {

// Marks requests complete with status st (a request's own earlier failure wins).
void complete(damf_server *s, std::vector<Req *> &rs, damf_status st) {
  const double t = s->now_us();
  std::lock_guard<std::mutex> lk(s->mu);
  for (Req *r : rs) {
    if (r->status == DAMF_OK) r->status = st;
    r->done_us = t;
    r->done = true;
    s->admitted_bytes -= r->bytes;
    if (r->status == DAMF_OK) {
      s->lat_ms.push_back((t - r->submit_us) * 1e-3);
      s->ops_done += r->k;
    }
    s->last_done_us = t;
    std::vector<int32_t>().swap(r->src);
    std::vector<int32_t>().swap(r->dst);
    std::vector<int8_t>().swap(r->op);
  }
  rs.clear();
  s->cv_done.notify_all();
}

// After a device error the context is poisoned: fail everything admitted.
void fail_all(damf_server *s, damf_status st) {
  complete(s, s->pending, st);
  s->pending_push = false;
  std::vector<Req *> rest;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->dead = st;
    rest.assign(s->queue.begin(), s->queue.end());
    s->queue.clear();
  }
  complete(s, rest, st);
}

damf_status run_pending_push(damf_server *s, hipStream_t st, bool beside_chain) {
  int64_t r = 0, p = 0, e = 0;
  const double t = s->now_us();
  const bool all = s->c->enhance_pending;  // after a re-orthogonalisation
  hipError_t err = ppr_push(s->c, st, all ? nullptr : s->c->ws.pend_rows, all ? 0 : s->pending_rows,
                            &r, &p, &e);
  if (err != hipSuccess) return api_dev_fail(s->c, err, "PPR push");
  s->c->enhance_pending = false;
  if (beside_chain) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->push_overlap_ms += (s->now_us() - t) * 1e-3;
  }
  return DAMF_OK;
}

void finish_pending(damf_server *s, hipStream_t st, bool beside_chain) {
  if (!s->pending_push) return;
  damf_status rc = run_pending_push(s, st, beside_chain);
  s->pending_push = false;
  complete(s, s->pending, rc);
  if (rc != DAMF_OK) fail_all(s, rc);
}

void do_step(damf_server *s, std::vector<Req *> &step) {
  damf_ctx *c = s->c;
  const double t_start = s->now_us();
  const int nseg = (int)step.size();
  std::vector<int32_t> seg_end(nseg);
  int64_t k = 0;
  int64_t step_index;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    step_index = s->steps++;
    s->step_reqs_sum += nseg;
  }
  for (int i = 0; i < nseg; ++i) {
    Req *r = step[i];
    std::memcpy(s->h_src + k, r->src.data(), r->k * sizeof(int32_t));
    std::memcpy(s->h_dst + k, r->dst.data(), r->k * sizeof(int32_t));
    std::memcpy(s->h_op + k, r->op.data(), r->k * sizeof(int8_t));
    k += r->k;
    seg_end[i] = (int32_t)k;
    r->start_us = t_start;
    r->step = step_index;
    r->step_requests = nseg;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->step_ops_sum += k;
  }
  BatchHeader h{};
  damf_status st = step_prepare(c, k, s->h_src, s->h_dst, s->h_op, 0, nseg, seg_end.data(), &h);
  if (st != DAMF_OK) {
    // ops were validated at submit: this is a device failure
    finish_pending(s, c->stream, false);
    complete(s, step, st);
    if (c->poisoned) fail_all(s, st);
    return;
  }
  for (int i = 0; i < nseg; ++i) {
    step[i]->net = c->ws.seg_stats_host[2 * i];
    step[i]->chunks = c->ws.seg_stats_host[2 * i + 1];
  }
  st = step_chain(c, h);
  // the previous step's Step 4 runs beside this step's chunks
  if (st == DAMF_OK) finish_pending(s, s->push_stream, h.n_chunks > 0);
  if (st == DAMF_OK) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = api_dev_fail(c, e, "chain");
  }
  if (st == DAMF_OK) st = step_graph(c, h);
  if (st == DAMF_OK) st = step_finish(c, h);
  if (st == DAMF_OK && c->cfg.reorth_every > 0 && h.n_chunks > 0 &&
      ++c->batches_since_reorth >= c->cfg.reorth_every) {
    c->batches_since_reorth = 0;
    int bad = 0;  // a refused re-orthogonalisation leaves the (valid) state as it is
    hipError_t e = reorthogonalize(c, &bad);
    if (e != hipSuccess) st = api_dev_fail(c, e, "re-orthogonalisation");
    c->enhance_pending = c->enhance_pending || c->ppr_on;  // R rotated: push from every node
  }
  if (st != DAMF_OK) {
    finish_pending(s, c->stream, false);
    complete(s, step, st);
    if (c->poisoned) fail_all(s, st);
    return;
  }
  if (c->ppr_on && c->cfg.auto_enhance) {
    int64_t rows = 0;
    st = step_push_rows(c, h, nseg, &rows);
    if (st == DAMF_OK) {
      hipError_t e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) st = api_dev_fail(c, e, "push rows");
    }
    if (st != DAMF_OK) {
      complete(s, step, st);
      fail_all(s, st);
      return;
    }
    s->pending = step;
    s->pending_rows = rows;
    s->pending_push = true;
    if (!s->cfg.overlap_push) finish_pending(s, c->stream, false);
  } else {
    complete(s, step, DAMF_OK);
  }
}

void worker_main(damf_server *s) {
  (void)hipSetDevice(s->c->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_work.wait(lk, [&] {
      return s->stop || s->pending_push || (!s->paused && !s->queue.empty());
    });
    if (s->paused || s->queue.empty()) {
      if (s->pending_push) {
        lk.unlock();
        finish_pending(s, s->c->stream, false);
        lk.lock();
        continue;
      }
      if (s->stop && (s->queue.empty() || s->paused)) break;
      continue;
    }
    std::vector<Req *> step;
    int64_t tot = 0;
    while (!s->queue.empty() && (int)step.size() < s->cfg.max_step_requests &&
           tot + s->queue.front()->k <= s->cfg.max_step_ops) {
      tot += s->queue.front()->k;
      step.push_back(s->queue.front());
      s->queue.pop_front();
    }
    lk.unlock();
    do_step(s, step);
    lk.lock();
  }
  lk.unlock();
  finish_pending(s, s->c->stream, false);
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

}  // namespace

extern "C" {

void damf_server_config_default(damf_server_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->admit_bytes = 64ll << 20;
  cfg->max_step_ops = kMaxBatch;
  cfg->max_step_requests = kMaxRequests;
  cfg->overlap_push = 1;
  cfg->start_paused = 0;
}

damf_status damf_server_create(damf_ctx *ctx, const damf_server_config *cfg, damf_server **out) {
  if (!ctx || !out) return DAMF_E_INVALID_ARG;
  *out = nullptr;
  damf_server_config cf;
  if (cfg)
    cf = *cfg;
  else
    damf_server_config_default(&cf);
  if (cf.admit_bytes < 1 || cf.max_step_ops < 1 || cf.max_step_ops > kMaxBatch ||
      cf.max_step_requests < 1 || cf.max_step_requests > kMaxRequests)
    return DAMF_E_INVALID_ARG;
  if (ctx->poisoned) return DAMF_E_STATE;
  damf_server *s = new (std::nothrow) damf_server();
  if (!s) return DAMF_E_OOM;
  s->c = ctx;
  s->cfg = cf;
  s->paused = cf.start_paused != 0;
  s->t0 = std::chrono::steady_clock::now();
  if (hipSetDevice(ctx->device) != hipSuccess ||
      hipStreamCreateWithFlags(&s->push_stream, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc((void **)&s->h_src, kMaxBatch * sizeof(int32_t)) != hipSuccess ||
      hipHostMalloc((void **)&s->h_dst, kMaxBatch * sizeof(int32_t)) != hipSuccess ||
      hipHostMalloc((void **)&s->h_op, kMaxBatch * sizeof(int8_t)) != hipSuccess) {
    if (s->push_stream) (void)hipStreamDestroy(s->push_stream);
    if (s->h_src) (void)hipHostFree(s->h_src);
    if (s->h_dst) (void)hipHostFree(s->h_dst);
    if (s->h_op) (void)hipHostFree(s->h_op);
    delete s;
    return DAMF_E_DEVICE;
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return DAMF_OK;
}

damf_status damf_submit(damf_server *s, int64_t k, const int32_t *src, const int32_t *dst,
                        const int8_t *op, int64_t *ticket) {
  if (!s || !ticket) return DAMF_E_INVALID_ARG;
  if (k < 1 || k > s->cfg.max_step_ops || !src || !dst || !op) return DAMF_E_INVALID_ARG;
  const int64_t n = s->c->n;
  for (int64_t i = 0; i < k; ++i)
    if (src[i] < 0 || dst[i] < 0 || src[i] >= n || dst[i] >= n || (op[i] != 1 && op[i] != -1))
      return DAMF_E_OUT_OF_RANGE;
  const int64_t bytes = 9 * k + kReqOverheadBytes;
  Req *r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->dead != DAMF_OK) return DAMF_E_STATE;
    if (s->admitted_bytes + bytes > s->cfg.admit_bytes) {
      ++s->busy;
      return DAMF_E_BUSY;
    }
    s->admitted_bytes += bytes;
    s->peak_bytes = std::max(s->peak_bytes, s->admitted_bytes);
  }
  r = new (std::nothrow) Req();
  if (r) {
    r->k = k;
    r->bytes = bytes;
    r->src.assign(src, src + k);
    r->dst.assign(dst, dst + k);
    r->op.assign(op, op + k);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (!r) {
    s->admitted_bytes -= bytes;
    return DAMF_E_OOM;
  }
  r->ticket = s->next_ticket++;
  r->submit_us = s->now_us();
  if (s->first_submit_us < 0) s->first_submit_us = r->submit_us;
  s->reqs[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return DAMF_OK;
}

damf_status damf_wait(damf_server *s, int64_t ticket, int64_t timeout_us,
                      damf_request_info *info) {
  if (!s) return DAMF_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return DAMF_E_INVALID_ARG;
  Req *r = it->second;
  if (timeout_us < 0) {
    s->cv_done.wait(lk, [&] { return r->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                                  [&] { return r->done; })) {
    return DAMF_E_TIMEOUT;
  }
  if (info) {
    info->ticket = r->ticket;
    info->ops = r->k;
    info->step = r->step;
    info->step_requests = r->step_requests;
    info->status = r->status;
    info->net_entries = r->net;
    info->chunks = r->chunks;
    info->submit_us = r->submit_us;
    info->start_us = r->start_us;
    info->done_us = r->done_us;
    info->latency_ms = (r->done_us - r->submit_us) * 1e-3;
  }
  const damf_status st = r->status;
  s->reqs.erase(it);
  delete r;
  return st;
}

damf_status damf_server_resume(damf_server *s) {
  if (!s) return DAMF_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->paused = false;
  s->cv_work.notify_one();
  return DAMF_OK;
}

damf_status damf_server_get_stats(damf_server *s, damf_server_stats *out) {
  if (!s || !out) return DAMF_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->requests_done = (int64_t)s->lat_ms.size();
  out->ops_done = s->ops_done;
  out->steps = s->steps;
  out->busy_rejects = s->busy;
  out->admitted_bytes_peak = s->peak_bytes;
  out->elapsed_s = (s->first_submit_us >= 0) ? (s->last_done_us - s->first_submit_us) * 1e-6 : 0.0;
  out->ops_per_s = out->elapsed_s > 0 ? (double)s->ops_done / out->elapsed_s : 0.0;
  out->latency_p50_ms = percentile(s->lat_ms, 0.50);
  out->latency_p99_ms = percentile(s->lat_ms, 0.99);
  double sum = 0.0, mx = 0.0;
  for (double v : s->lat_ms) {
    sum += v;
    mx = std::max(mx, v);
  }
  out->latency_mean_ms = s->lat_ms.empty() ? 0.0 : sum / (double)s->lat_ms.size();
  out->latency_max_ms = mx;
  out->mean_requests_per_step = s->steps ? (double)s->step_reqs_sum / (double)s->steps : 0.0;
  out->mean_ops_per_step = s->steps ? (double)s->step_ops_sum / (double)s->steps : 0.0;
  out->push_overlapped_ms = s->push_overlap_ms;
  return DAMF_OK;
}

void damf_server_destroy(damf_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->paused = false;
    s->cv_work.notify_one();
  }
  if (s->worker.joinable()) s->worker.join();
  for (auto &kv : s->reqs) delete kv.second;
  (void)hipStreamSynchronize(s->push_stream);
  (void)hipStreamDestroy(s->push_stream);
  (void)hipHostFree(s->h_src);
  (void)hipHostFree(s->h_dst);
  (void)hipHostFree(s->h_op);
  delete s;
}

}  // extern "C"
