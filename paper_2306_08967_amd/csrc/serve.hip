// serve.hip -- continuous-batching update server (include/damf_serve.h).
//
// One server thread owns the context.  Clients admit requests under two
// memory caps (host staging and the device memory their graph edits may
// claim); the thread takes every admitted request that fits into the next
// step (up to max_step_ops / max_step_requests), concatenates them as request
// segments and runs one update step.  A request longer than max_step_ops runs
// alone as consecutive parts of max_step_ops ops (its ops in order, so the
// graph ends as with one batch).  Step:
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
#include <cmath>
#include <cstdio>
#include <string>
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
// device memory an op may claim: one entry (4 B) in each of the out- and
// in-CSR pools, times 3 for a moved row's reservation (len + len/2 + 8) and
// the old copy that compaction later frees
constexpr int64_t kDeviceBytesPerOp = 24;
constexpr int kMaxRequestOps = 1 << 20;
// chunk ranks the tuner tries, and steps per candidate
constexpr int kTuneRanks[] = {16, 32, 48, 64};
constexpr int kTuneSteps = 4;

struct Req {
  int64_t ticket = 0, k = 0, bytes = 0, dev_bytes = 0;
  int64_t sched = 0;  // ops handed to steps so far
  int32_t parts = 0, chunk_rank = 0;
  std::vector<int32_t> src, dst;
  std::vector<int8_t> op;
  double submit_us = 0, start_us = 0, done_us = 0;
  int64_t step = -1, net = 0, chunks = 0;
  int32_t step_requests = 0;
  damf_status status = DAMF_OK;
  bool done = false;
};

// ops [off, off + len) of a request, carried by one step; `last` marks the
// part that completes it
struct Part {
  Req *r;
  int64_t off, len;
  bool last;
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
  int64_t admitted_dev = 0, peak_dev = 0, dev_cap = 0;
  // chunk-rank tuner (worker thread only; tuned_rank read under mu)
  int tune_idx = -1, tune_left = 0, tuned_rank = 0;
  double tune_ms[4] = {}, tune_net[4] = {};
  int64_t tuner_steps = 0;
  std::string tune_key, tune_path;  // the cache path is copied at creation
  bool stop = false, paused = false;
  damf_status dead = DAMF_OK;                // set after a device error
  hipStream_t push_stream = nullptr;
  // deferred Step 4 (worker thread only)
  std::vector<Part> pending;
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

// Ends the step's parts with status st (a request's own earlier failure
// wins); a request completes with its last part, or with any part when
// `all` (the server stopped).
void complete(damf_server *s, std::vector<Part> &ps, damf_status st, bool all = false) {
  const double t = s->now_us();
  std::lock_guard<std::mutex> lk(s->mu);
  for (Part &pt : ps) {
    Req *r = pt.r;
    if (r->status == DAMF_OK) r->status = st;
    if ((!pt.last && !all) || r->done) continue;
    r->done_us = t;
    r->done = true;
    s->admitted_bytes -= r->bytes;
    s->admitted_dev -= r->dev_bytes;
    if (r->status == DAMF_OK) {
      s->lat_ms.push_back((t - r->submit_us) * 1e-3);
      s->ops_done += r->k;
    }
    s->last_done_us = t;
    std::vector<int32_t>().swap(r->src);
    std::vector<int32_t>().swap(r->dst);
    std::vector<int8_t>().swap(r->op);
  }
  ps.clear();
  s->cv_done.notify_all();
}

// After a device error the context is poisoned: fail everything admitted.
void fail_all(damf_server *s, damf_status st) {
  complete(s, s->pending, st, true);
  s->pending_push = false;
  std::vector<Part> rest;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->dead = st;
    for (Req *r : s->queue) rest.push_back(Part{r, 0, 0, true});
    s->queue.clear();
  }
  complete(s, rest, st, true);
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

// ---- chunk-rank tuner.  The chain's cost per net entry depends on the chunk
// rank r (core size d + r against the number of chunks); the tuner runs
// kTuneSteps steps at each candidate rank, keeps the one with the least chain
// time per net entry, and records it in the cache file under a key of the
// device architecture, n, d, precision and the graph size (log2 of m).

std::string tune_key(damf_ctx *c) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, c->device);
  char buf[256];
  const int64_t m = std::max<int64_t>(1, c->out.nnz_built);
  std::snprintf(buf, sizeof buf, "%s n=%lld d=%d precision=%d log2m=%d", prop.gcnArchName,
                (long long)c->n, c->d, c->split ? 1 : 0, (int)std::floor(std::log2((double)m)));
  return std::string(buf);
}

int tune_cache_lookup(const char *path, const std::string &key) {
  if (!path) return 0;
  FILE *f = std::fopen(path, "r");
  if (!f) return 0;
  char line[512];
  int r = 0;
  while (std::fgets(line, sizeof line, f)) {
    const std::string ln(line);
    const size_t at = ln.rfind(" r=");
    if (at != std::string::npos && ln.compare(0, at, key) == 0 && at == key.size())
      r = std::atoi(ln.c_str() + at + 3);  // the last entry for the key wins
  }
  std::fclose(f);
  return r;
}

void tune_cache_store(const char *path, const std::string &key, int r) {
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s r=%d\n", key.c_str(), r);
  std::fclose(f);
}

int tune_candidates(damf_ctx *c, int *out) {
  int cnt = 0;
  for (int r : kTuneRanks)
    if (r <= c->cfg.max_side && c->d + r <= kMaxCore) out[cnt++] = r;
  return cnt;
}

// before a step: the rank to use
void tune_before(damf_server *s) {
  if (s->tune_idx < 0) return;
  int cand[4];
  tune_candidates(s->c, cand);
  s->c->cfg.max_core_rank = cand[s->tune_idx];
}

// after a step: record its chain time per net entry; move on or decide
void tune_after(damf_server *s, double chain_ms, int64_t net) {
  if (s->tune_idx < 0 || net <= 0) return;
  s->tune_ms[s->tune_idx] += chain_ms;
  s->tune_net[s->tune_idx] += (double)net;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->tuner_steps;
  }
  if (--s->tune_left > 0) return;
  int cand[4];
  const int nc = tune_candidates(s->c, cand);
  if (s->tune_idx + 1 < nc) {
    ++s->tune_idx;
    s->tune_left = kTuneSteps;
    return;
  }
  int best = 0;
  for (int i = 1; i < nc; ++i)
    if (s->tune_ms[i] / s->tune_net[i] < s->tune_ms[best] / s->tune_net[best]) best = i;
  s->c->cfg.max_core_rank = cand[best];
  s->tune_idx = -1;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->tuned_rank = cand[best];
  }
  tune_cache_store(s->tune_path.empty() ? nullptr : s->tune_path.c_str(), s->tune_key, cand[best]);
}

void do_step(damf_server *s, std::vector<Part> &step) {
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
  tune_before(s);
  for (int i = 0; i < nseg; ++i) {
    Req *r = step[i].r;
    const int64_t off = step[i].off, len = step[i].len;
    std::memcpy(s->h_src + k, r->src.data() + off, len * sizeof(int32_t));
    std::memcpy(s->h_dst + k, r->dst.data() + off, len * sizeof(int32_t));
    std::memcpy(s->h_op + k, r->op.data() + off, len * sizeof(int8_t));
    k += len;
    seg_end[i] = (int32_t)k;
    if (r->parts++ == 0) r->start_us = t_start;
    r->step = step_index;
    r->step_requests = nseg;
    r->chunk_rank = c->cfg.max_core_rank;
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
    step[i].r->net += c->ws.seg_stats_host[2 * i];
    step[i].r->chunks += c->ws.seg_stats_host[2 * i + 1];
  }
  st = step_chain(c, h, nseg);
  // the previous step's Step 4 runs beside this step's chunks
  if (st == DAMF_OK) finish_pending(s, s->push_stream, h.n_chunks > 0);
  if (st == DAMF_OK) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = api_dev_fail(c, e, "chain");
  }
  if (st == DAMF_OK) st = step_check(c, h, false);
  if (st == DAMF_OK && h.n_chunks > 0) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[4], c->ev[5]) == hipSuccess) tune_after(s, ms, h.n_net);
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
    // whole requests while they fit; a request longer than a step runs
    // alone, one part of max_step_ops ops per step
    std::vector<Part> step;
    int64_t tot = 0;
    while (!s->queue.empty() && (int)step.size() < s->cfg.max_step_requests) {
      Req *f = s->queue.front();
      const int64_t rem = f->k - f->sched;
      if (rem <= s->cfg.max_step_ops - tot) {
        step.push_back(Part{f, f->sched, rem, true});
        f->sched = f->k;
        tot += rem;
        s->queue.pop_front();
        continue;
      }
      if (step.empty()) {
        step.push_back(Part{f, f->sched, (int64_t)s->cfg.max_step_ops, false});
        f->sched += s->cfg.max_step_ops;
      }
      break;
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
  cfg->admit_device_bytes = 0;
  cfg->max_request_ops = 1 << 16;
  cfg->autotune = 0;
  cfg->tune_cache = nullptr;
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
      cf.max_step_requests < 1 || cf.max_step_requests > kMaxRequests ||
      cf.max_request_ops < 1 || cf.max_request_ops > kMaxRequestOps || cf.admit_device_bytes < 0 ||
      (cf.autotune != 0 && cf.autotune != 1))
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
  if (cf.admit_device_bytes > 0) {
    s->dev_cap = cf.admit_device_bytes;
  } else {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    s->dev_cap = (int64_t)(free_b / 2);
  }
  s->tune_key = tune_key(ctx);
  if (cf.tune_cache) s->tune_path = cf.tune_cache;
  s->cfg.tune_cache = nullptr;  // the caller's string need not outlive the call
  if (cf.autotune) {
    const int cached = tune_cache_lookup(cf.tune_cache, s->tune_key);
    int cand[4];
    const int nc = tune_candidates(ctx, cand);
    bool ok = false;
    for (int i = 0; i < nc; ++i) ok = ok || cand[i] == cached;
    if (ok) {
      ctx->cfg.max_core_rank = cached;
      s->tuned_rank = cached;
    } else if (nc > 1) {
      s->tune_idx = 0;
      s->tune_left = kTuneSteps;
    }
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return DAMF_OK;
}

damf_status damf_submit(damf_server *s, int64_t k, const int32_t *src, const int32_t *dst,
                        const int8_t *op, int64_t *ticket) {
  if (!s || !ticket) return DAMF_E_INVALID_ARG;
  if (k < 1 || k > s->cfg.max_request_ops || !src || !dst || !op) return DAMF_E_INVALID_ARG;
  const int64_t n = s->c->n;
  for (int64_t i = 0; i < k; ++i)
    if (src[i] < 0 || dst[i] < 0 || src[i] >= n || dst[i] >= n || (op[i] != 1 && op[i] != -1))
      return DAMF_E_OUT_OF_RANGE;
  const int64_t bytes = 9 * k + kReqOverheadBytes;
  const int64_t dev = kDeviceBytesPerOp * k;
  Req *r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->dead != DAMF_OK) return DAMF_E_STATE;
    if (s->admitted_bytes + bytes > s->cfg.admit_bytes || s->admitted_dev + dev > s->dev_cap) {
      ++s->busy;
      return DAMF_E_BUSY;
    }
    s->admitted_bytes += bytes;
    s->admitted_dev += dev;
    s->peak_bytes = std::max(s->peak_bytes, s->admitted_bytes);
    s->peak_dev = std::max(s->peak_dev, s->admitted_dev);
  }
  r = new (std::nothrow) Req();
  if (r) {
    r->k = k;
    r->bytes = bytes;
    r->dev_bytes = dev;
    r->src.assign(src, src + k);
    r->dst.assign(dst, dst + k);
    r->op.assign(op, op + k);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (!r) {
    s->admitted_bytes -= bytes;
    s->admitted_dev -= dev;
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
    info->parts = r->parts;
    info->chunk_rank = r->chunk_rank;
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
  out->admitted_device_bytes_peak = s->peak_dev;
  out->device_cap_bytes = s->dev_cap;
  out->tuned_chunk_rank = s->tuned_rank;
  out->tuner_steps = s->tuner_steps;
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
