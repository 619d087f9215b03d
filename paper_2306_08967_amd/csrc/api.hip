// api.hip -- the C ABI (include/damf.h): context lifetime, argument checks,
// host <-> device marshalling, and the order of kernels per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "damf_internal.h"

namespace damf {
size_t chain_scratch_doubles();
}

using namespace damf;

namespace {

damf_status fail(damf_ctx *c, damf_status s, const char *msg) {
  if (c) c->err = msg;
  return s;
}

damf_status dev_fail(damf_ctx *c, hipError_t e, const char *where) {
  if (c) {
    c->poisoned = true;
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return (e == hipErrorOutOfMemory) ? DAMF_E_OOM : DAMF_E_DEVICE;
}

#define API_HIP(ctx, expr, where)                   \
  do {                                              \
    hipError_t _e = (expr);                         \
    if (_e != hipSuccess) return dev_fail(ctx, _e, where); \
  } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
  return hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
}

damf_status check_config(const damf_config *cfg) {
  if (!cfg) return DAMF_E_INVALID_ARG;
  // node ids are int32; row-parallel launches (TSQR, the rotation GEMMs) take
  // up to 4 work-items per node, and a dispatch holds fewer than 2^32
  if (cfg->n < 1 || cfg->n > kMaxNodes) return DAMF_E_INVALID_ARG;
  if (cfg->d < 1 || cfg->d > kMaxD) return DAMF_E_INVALID_ARG;
  if (cfg->max_core_rank < 1 || cfg->max_side < 1 || cfg->max_side > kMaxSide)
    return DAMF_E_INVALID_ARG;
  if (cfg->max_core_rank > cfg->max_side) return DAMF_E_INVALID_ARG;
  if (cfg->d + cfg->max_core_rank > kMaxCore) return DAMF_E_INVALID_ARG;
  if (!(cfg->alpha > 0.0 && cfg->alpha <= 1.0)) return DAMF_E_INVALID_ARG;
  if (!(cfg->eps > 0.0)) return DAMF_E_INVALID_ARG;
  if (!(cfg->tau >= 0.0)) return DAMF_E_INVALID_ARG;
  if (cfg->oversample < 0 || cfg->power_iters < 0) return DAMF_E_INVALID_ARG;
  if (cfg->d + cfg->oversample > kMaxCore) return DAMF_E_INVALID_ARG;
  if (!(cfg->graph_slack >= 1.0)) return DAMF_E_INVALID_ARG;
  if (cfg->reorth_every < 0) return DAMF_E_INVALID_ARG;
  if (cfg->precision != 0 && cfg->precision != 1) return DAMF_E_INVALID_ARG;
  if (cfg->kernel_timing != 0 && cfg->kernel_timing != 1) return DAMF_E_INVALID_ARG;
  if (!(cfg->jacobi_tol == 0.0 || (cfg->jacobi_tol >= 1e-14 && cfg->jacobi_tol <= 1e-6)))
    return DAMF_E_INVALID_ARG;
  if (!(cfg->flush_cond <= 0.0 || cfg->flush_cond >= 1.0)) return DAMF_E_INVALID_ARG;
  if (cfg->graph_chunks < 0 || cfg->graph_chunks > 64) return DAMF_E_INVALID_ARG;
  return DAMF_OK;
}

// Allocates everything except the graph.
damf_status alloc_state(damf_ctx *c) {
  const int64_t n = c->n;
  const int d = c->d;
  API_HIP(c, dalloc(&c->Ub, n * d), "alloc U_b");
  API_HIP(c, dalloc(&c->Vb, n * d), "alloc V_b");
  API_HIP(c, dalloc(&c->P, 2 * d * d), "alloc P");
  API_HIP(c, dalloc(&c->Pnext, 2 * d * d), "alloc P");
  API_HIP(c, dalloc(&c->sigma, kMaxCore), "alloc sigma");
  if (c->ppr_on) {
    API_HIP(c, dalloc(&c->Zb, n * d), "alloc Z_b");
    API_HIP(c, dalloc(&c->R, n * d), "alloc R");
  }
  Workspace &w = c->ws;
  API_HIP(c, dalloc(&w.ops_src, kMaxBatch), "alloc ws");
  API_HIP(c, dalloc(&w.ops_dst, kMaxBatch), "alloc ws");
  API_HIP(c, dalloc(&w.ops_op, kMaxBatch), "alloc ws");
  API_HIP(c, dalloc(&w.units, kMaxBatch), "alloc ws");
  API_HIP(c, dalloc(&w.unit_seg, kMaxBatch), "alloc ws");
  API_HIP(c, dalloc(&w.units_comb, kMaxBatch), "alloc ws");
  API_HIP(c, dalloc(&w.seg_end, kMaxRequests), "alloc ws");
  API_HIP(c, dalloc(&w.seg_stats, 2 * kMaxRequests), "alloc ws");
  API_HIP(c, hipHostMalloc((void **)&w.seg_stats_host, 3 * kMaxRequests * sizeof(int32_t)), "alloc pinned");
  API_HIP(c, dalloc(&w.pend_rows, 4 * kMaxBatch + 1), "alloc ws");
  API_HIP(c, dalloc(&w.edit_stage, (size_t)kEditStagePool), "alloc ws");
  API_HIP(c, dalloc(&w.edit_stage_top, 1), "alloc ws");
  API_HIP(c, dalloc(&w.chunk_ent, 2 * kMaxBatch), "alloc ws");
  API_HIP(c, dalloc(&w.net, 2 * kMaxBatch), "alloc ws");
  API_HIP(c, dalloc(&w.net_t, 2 * kMaxBatch), "alloc ws");
  API_HIP(c, dalloc(&w.rows_out, 2 * kMaxBatch + 1), "alloc ws");
  API_HIP(c, dalloc(&w.rowpos_out, 2 * kMaxBatch + 1), "alloc ws");
  API_HIP(c, dalloc(&w.rows_in, 2 * kMaxBatch + 1), "alloc ws");
  API_HIP(c, dalloc(&w.rowpos_in, 2 * kMaxBatch + 1), "alloc ws");
  API_HIP(c, dalloc(&w.chunks, 2 * kMaxBatch + 1), "alloc ws");
  API_HIP(c, dalloc(&w.chunk_s1, 2 * kMaxBatch + kMaxSide), "alloc ws");
  API_HIP(c, dalloc(&w.chunk_s2, 2 * kMaxBatch + kMaxSide), "alloc ws");
  API_HIP(c, dalloc(&w.hdr, 1), "alloc ws");
  API_HIP(c, hipHostMalloc((void **)&w.hdr_host, sizeof(BatchHeader)), "alloc pinned");
  API_HIP(c, dalloc(&w.cstats, 1), "alloc ws");
  API_HIP(c, hipHostMalloc((void **)&w.cstats_host, sizeof(ChainStats)), "alloc pinned");
  w.scratch_doubles = chain_scratch_doubles();
  API_HIP(c, dalloc(&w.scratch, w.scratch_doubles), "alloc scratch");
  API_HIP(c, dalloc(&w.undo_u, (size_t)(2 * kMaxBatch + kMaxSide) * d), "alloc undo log");
  API_HIP(c, dalloc(&w.undo_v, (size_t)(2 * kMaxBatch + kMaxSide) * d), "alloc undo log");
  if (c->ppr_on) API_HIP(c, dalloc(&w.undo_r, (size_t)(kRLogS1 + 2 * kMaxBatch + kMaxSide) * d), "alloc undo log");
  API_HIP(c, dalloc(&w.psave, 2 * (size_t)d * d + kMaxCore), "alloc undo log");
  API_HIP(c, dalloc(&w.counters, 16), "alloc ws");
  API_HIP(c, hipHostMalloc((void **)&w.counters_host, 16 * sizeof(int64_t)), "alloc pinned");
  API_HIP(c, hipHostMalloc((void **)&w.dscratch_host, 16 * sizeof(double)), "alloc pinned");
  if (c->ppr_on) {
    API_HIP(c, dalloc(&w.stamp, n), "alloc ppr");
    API_HIP(c, dalloc(&w.cand, n), "alloc ppr");
    API_HIP(c, dalloc(&w.cand2, n), "alloc ppr");
    API_HIP(c, dalloc(&w.frontier, n), "alloc ppr");
    API_HIP(c, hipMemsetAsync(w.stamp, 0xff, n * sizeof(int32_t), c->stream), "memset");
  }
  for (auto &e : c->ev) API_HIP(c, hipEventCreate(&e), "event");
  API_HIP(c, hipEventCreate(&c->ev_k[0]), "event");
  API_HIP(c, hipEventCreate(&c->ev_k[1]), "event");
  API_HIP(c, hipStreamCreateWithFlags(&c->scatter_stream, hipStreamNonBlocking), "stream");
  for (auto &e : c->ev_back) API_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  for (auto &e : c->ev_front) API_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  for (auto &e : c->ev_scatter) API_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  if (c->cfg.kernel_timing)
    for (auto &e : c->ev_core) API_HIP(c, hipEventCreate(&e), "event");
  return DAMF_OK;
}

void free_ctx(damf_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->scatter_stream) (void)hipStreamSynchronize(c->scatter_stream);
  csr_free(c->out);
  csr_free(c->in);
  void *ptrs[] = {c->Ub, c->Vb, c->Zb, c->R, c->P, c->Pnext, c->sigma,
                  c->ws.ops_src, c->ws.ops_dst, c->ws.ops_op, c->ws.units, c->ws.chunk_ent,
                  c->ws.net, c->ws.net_t, c->ws.rows_out, c->ws.rowpos_out, c->ws.rows_in,
                  c->ws.rowpos_in, c->ws.chunks, c->ws.chunk_s1, c->ws.chunk_s2, c->ws.hdr,
                  c->ws.cstats, c->ws.scratch, c->ws.counters, c->ws.stamp, c->ws.cand,
                  c->ws.cand2, c->ws.frontier, c->ws.unit_seg, c->ws.units_comb,
                  c->ws.seg_end, c->ws.seg_stats, c->ws.pend_rows, c->ws.edit_stage,
                  c->ws.edit_stage_top, c->ws.hbuf, c->ws.hnode, c->ws.hseg,
                  c->ws.push_ring, c->ws.push_log, c->ws.undo_u, c->ws.undo_v, c->ws.undo_r, c->ws.psave};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (c->ws.hdr_host) (void)hipHostFree(c->ws.hdr_host);
  if (c->ws.cstats_host) (void)hipHostFree(c->ws.cstats_host);
  if (c->ws.counters_host) (void)hipHostFree(c->ws.counters_host);
  if (c->ws.dscratch_host) (void)hipHostFree(c->ws.dscratch_host);
  if (c->ws.seg_stats_host) (void)hipHostFree(c->ws.seg_stats_host);
  if (c->ws.push_log_host) (void)hipHostFree(c->ws.push_log_host);
  for (auto &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : c->ev_k)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : c->ev_core)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : c->ev_back)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : c->ev_front)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : c->ev_scatter)
    if (e) (void)hipEventDestroy(e);
  for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  if (c->scatter_stream) {
    (void)hipStreamSynchronize(c->scatter_stream);
    (void)hipStreamDestroy(c->scatter_stream);
  }
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

// Builds out- and in-CSR from an edge list (host or device pointers).
damf_status build_graph(damf_ctx *c, int64_t m, const int32_t *src, const int32_t *dst,
                        int32_t flags) {
  if (m < 0 || (m > 0 && (!src || !dst))) return fail(c, DAMF_E_INVALID_ARG, "bad edge list");
  const int32_t *ds = src, *dd = dst;
  int32_t *own_s = nullptr, *own_d = nullptr;
  if (!(flags & DAMF_DEVICE_PTRS) && m > 0) {
    // host validation before anything is built
    for (int64_t e = 0; e < m; ++e)
      if (src[e] < 0 || dst[e] < 0 || src[e] >= c->n || dst[e] >= c->n)
        return fail(c, DAMF_E_OUT_OF_RANGE, "edge id out of range");
    API_HIP(c, dalloc(&own_s, m), "alloc edges");
    API_HIP(c, dalloc(&own_d, m), "alloc edges");
    API_HIP(c, hipMemcpyAsync(own_s, src, m * sizeof(int32_t), hipMemcpyHostToDevice, c->stream), "copy edges");
    API_HIP(c, hipMemcpyAsync(own_d, dst, m * sizeof(int32_t), hipMemcpyHostToDevice, c->stream), "copy edges");
    ds = own_s;
    dd = own_d;
  } else if (m > 0) {
    int32_t *bad = reinterpret_cast<int32_t *>(c->ws.counters);
    API_HIP(c, launch_validate_edges(ds, dd, m, c->n, bad, c->stream), "validate");
    int32_t hbad = 0;
    API_HIP(c, hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream), "validate");
    API_HIP(c, hipStreamSynchronize(c->stream), "validate");
    if (hbad) return fail(c, DAMF_E_OUT_OF_RANGE, "edge id out of range");
  }
  API_HIP(c, csr_build(c, c->out, ds, dd, m, c->cfg.graph_slack), "build CSR");
  API_HIP(c, csr_build(c, c->in, dd, ds, m, c->cfg.graph_slack), "build CSR^T");
  API_HIP(c, hipStreamSynchronize(c->stream), "build CSR");
  if (own_s) (void)hipFree(own_s);
  if (own_d) (void)hipFree(own_d);
  return DAMF_OK;
}

damf_status new_ctx(const damf_config *cfg, damf_ctx **out, damf_ctx **cptr) {
  if (!out) return DAMF_E_INVALID_ARG;
  *out = nullptr;
  damf_status st = check_config(cfg);
  if (st != DAMF_OK) return st;
  damf_ctx *c = new (std::nothrow) damf_ctx();
  if (!c) return DAMF_E_OOM;
  c->cfg = *cfg;
  c->n = cfg->n;
  c->d = cfg->d;
  c->ppr_on = cfg->alpha < 1.0;
  c->split = cfg->precision == 1;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return DAMF_E_DEVICE;
  }
  if (static_scratch_setup(c->device) != hipSuccess) {
    delete c;
    return DAMF_E_DEVICE;
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && khz > 0)
    c->wall_khz = (double)khz;
  if (cfg->hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(cfg->hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return DAMF_E_DEVICE;
    }
    c->own_stream = true;
  }
  *cptr = c;
  return DAMF_OK;
}

double ms_between(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return (double)ms;
}

}  // namespace

namespace damf {

damf_status api_fail(damf_ctx *c, damf_status s, const char *msg) { return fail(c, s, msg); }
damf_status api_dev_fail(damf_ctx *c, hipError_t e, const char *where) {
  return dev_fail(c, e, where);
}

damf_status step_prepare(damf_ctx *c, int64_t k, const int32_t *src, const int32_t *dst,
                         const int8_t *op, int32_t flags, int nseg, const int32_t *seg_end,
                         BatchHeader *h) {
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  if (k < 1 || k > kMaxBatch) return fail(c, DAMF_E_INVALID_ARG, "batch size out of range");
  if (!src || !dst || !op) return fail(c, DAMF_E_INVALID_ARG, "null op arrays");
  if (nseg < 1 || nseg > kMaxRequests || seg_end[nseg - 1] != k)
    return fail(c, DAMF_E_INVALID_ARG, "bad request segments");
  for (int i = 1; i < nseg; ++i)
    if (seg_end[i] < seg_end[i - 1]) return fail(c, DAMF_E_INVALID_ARG, "bad request segments");
  hipStream_t s = c->stream;
  Workspace &w = c->ws;
  if (flags & DAMF_DEVICE_PTRS) {
    API_HIP(c, hipMemcpyAsync(w.ops_src, src, k * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy ops");
    API_HIP(c, hipMemcpyAsync(w.ops_dst, dst, k * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy ops");
    API_HIP(c, hipMemcpyAsync(w.ops_op, op, k * sizeof(int8_t), hipMemcpyDeviceToDevice, s), "copy ops");
  } else {
    for (int64_t i = 0; i < k; ++i)
      if (src[i] < 0 || dst[i] < 0 || src[i] >= c->n || dst[i] >= c->n || (op[i] != 1 && op[i] != -1))
        return fail(c, DAMF_E_OUT_OF_RANGE, "op id or type out of range");
    API_HIP(c, hipMemcpyAsync(w.ops_src, src, k * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy ops");
    API_HIP(c, hipMemcpyAsync(w.ops_dst, dst, k * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy ops");
    API_HIP(c, hipMemcpyAsync(w.ops_op, op, k * sizeof(int8_t), hipMemcpyHostToDevice, s), "copy ops");
  }
  std::memcpy(w.seg_stats_host + 2 * kMaxRequests, seg_end, nseg * sizeof(int32_t));
  API_HIP(c, hipMemcpyAsync(w.seg_end, w.seg_stats_host + 2 * kMaxRequests, nseg * sizeof(int32_t),
                            hipMemcpyHostToDevice, s), "copy segments");
  API_HIP(c, hipEventRecord(c->ev[0], s), "event");
  API_HIP(c, launch_batch_prepare(c, (int)k, nseg), "batch prepare");
  API_HIP(c, hipMemcpyAsync(w.hdr_host, w.hdr, sizeof(BatchHeader), hipMemcpyDeviceToHost, s), "header");
  API_HIP(c, hipMemcpyAsync(w.seg_stats_host, w.seg_stats, 2 * nseg * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s), "request stats");
  API_HIP(c, hipStreamSynchronize(s), "batch prepare");
  *h = *w.hdr_host;
  if (h->bad_ops > 0) return fail(c, DAMF_E_OUT_OF_RANGE, "op id or type out of range");
  API_HIP(c, hipEventRecord(c->ev[1], s), "event");
  return DAMF_OK;
}

namespace {

// The batch's CSR edits (and, with fixup, Step 4's structural fix-up of the
// edited rows' residuals, after saving those rows of R for a rollback).
damf_status graph_edit(damf_ctx *c, const BatchHeader &h, bool fixup) {
  if (h.n_net <= 0) return DAMF_OK;
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  // make room first if the rows that outgrow their reservation could
  // overflow a pool
  API_HIP(c, launch_csr_need(c, c->out, w.net, w.rows_out, w.rowpos_out, h.n_rows_out, w.counters + 10), "pool need");
  API_HIP(c, launch_csr_need(c, c->in, w.net_t, w.rows_in, w.rowpos_in, h.n_rows_in, w.counters + 11), "pool need");
  API_HIP(c, hipMemcpyAsync(w.counters_host + 10, w.counters + 10, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s), "pool need");
  API_HIP(c, hipMemcpyAsync(w.counters_host + 8, c->out.top, sizeof(int64_t), hipMemcpyDeviceToHost, s), "pool");
  API_HIP(c, hipMemcpyAsync(w.counters_host + 9, c->in.top, sizeof(int64_t), hipMemcpyDeviceToHost, s), "pool");
  API_HIP(c, hipStreamSynchronize(s), "pool need");
  const int64_t need_out = w.counters_host[10], need_in = w.counters_host[11];
  if (c->out.pool_cap - w.counters_host[8] < need_out)
    API_HIP(c, csr_compact(c, c->out, c->cfg.graph_slack, 2 * need_out), "CSR compaction");
  if (c->in.pool_cap - w.counters_host[9] < need_in)
    API_HIP(c, csr_compact(c, c->in, c->cfg.graph_slack, 2 * need_in), "CSR^T compaction");
  if (c->ppr_on && fixup) {
    API_HIP(c, launch_r_rows(c, w.rows_out, h.n_rows_out, 0, false), "undo log (R)");
    API_HIP(c, ppr_fixup(c, h.n_rows_out), "PPR structural fix-up");
  }
  API_HIP(c, launch_csr_edit(c, c->out, w.net, w.rows_out, w.rowpos_out, h.n_rows_out, false), "CSR edit");
  API_HIP(c, launch_csr_edit(c, c->in, w.net_t, w.rows_in, w.rowpos_in, h.n_rows_in, true), "CSR^T edit");
  return DAMF_OK;
}

}  // namespace

damf_status step_graph(damf_ctx *c, const BatchHeader &h) { return graph_edit(c, h, true); }

damf_status step_chain(damf_ctx *c, const BatchHeader &h, int nseg) {
  if (h.n_chunks <= 0) return DAMF_OK;
  hipStream_t s = c->stream;
  // a request's first chunk that meets the previous request's last chunk
  // waits for that chunk's scatter (see chain_hold)
  std::memset(c->chain_hold, 0, sizeof(c->chain_hold));
  for (int i = 0, ch0 = 0; i < nseg; ++i) {
    if (ch0 > 0 && ch0 < h.n_chunks && ((h.meets_prev[ch0 >> 6] >> (ch0 & 63)) & 1))
      c->chain_hold[ch0 >> 6] |= 1ull << (ch0 & 63);
    ch0 += c->ws.seg_stats_host[2 * i + 1];
  }
  // undo log: the touched rows of U_b, V_b and R, and P, Sigma before the chunks
  const size_t dd = 2 * (size_t)c->d * c->d;
  API_HIP(c, launch_undo_rows(c, 0, h.s1_total, 0, h.s2_total, false), "undo log");
  API_HIP(c, launch_r_rows(c, c->ws.chunk_s1, h.s1_total, kRLogS1, false), "undo log (R)");
  API_HIP(c, hipMemcpyAsync(c->ws.psave, c->P, dd * sizeof(double), hipMemcpyDeviceToDevice, s), "undo log");
  API_HIP(c, hipMemcpyAsync(c->ws.psave + dd, c->sigma, kMaxCore * sizeof(double), hipMemcpyDeviceToDevice, s),
          "undo log");
  API_HIP(c, hipEventRecord(c->ev[4], s), "event");
  bool graphed = false;
  API_HIP(c, launch_chain_graph(c, h.n_chunks, h.meets_prev, &graphed), "chain (graph)");
  if (graphed)
    ++c->graph_launches;
  else
    API_HIP(c, launch_chain(c, 0, h.n_chunks, h.n_chunks, h.meets_prev), "chain");
  API_HIP(c, hipEventRecord(c->ev[5], s), "event");
  return DAMF_OK;
}

namespace {

void add_stats(ChainStats &a, const ChainStats &b, bool with_cond) {
  a.max_core = std::max(a.max_core, b.max_core);
  a.dropped += b.dropped;
  a.sweeps += b.sweeps;
  a.flops += b.flops;
  a.core_flops += b.core_flops;
  a.core_flops_model += b.core_flops_model;
  a.small_sv_columns += b.small_sv_columns;
  for (int i = 0; i < 8; ++i) a.phase_ticks[i] += b.phase_ticks[i];
  if (with_cond) a.p_cond_bits = std::max(a.p_cond_bits, b.p_cond_bits);
}

// A chunk left a projection P F too ill-conditioned for the lazy scatter (a
// kept direction with little or no component in span(U_b P), e.g. an edge
// between two nodes without basis weight while a zero singular value is
// kept): its solve would amplify the FP32 rounding of the rows it writes by
// cond(P F), or fail.  Undo the batch's chunks and run them again one by
// one; a chunk whose new projection passes the limit is applied explicitly,
// U_b <- U_b P F + dU (the flush rotation by P F over all rows, then the row
// corrections with P = I), which is the update of Theorem 2 without the lazy
// projection.
damf_status chain_recover(damf_ctx *c, const BatchHeader &h, ChainStats *out) {
  hipStream_t s = c->stream;
  Workspace &w = c->ws;
  const size_t dd = 2 * (size_t)c->d * c->d;
  API_HIP(c, launch_undo_rows(c, 0, h.s1_total, 0, h.s2_total, true), "undo");
  API_HIP(c, hipMemcpyAsync(c->P, w.psave, dd * sizeof(double), hipMemcpyDeviceToDevice, s), "undo");
  API_HIP(c, hipMemcpyAsync(c->sigma, w.psave + dd, kMaxCore * sizeof(double), hipMemcpyDeviceToDevice, s),
          "undo");
  std::vector<ChunkDesc> desc;
  try {
    desc.resize(h.n_chunks);
  } catch (...) {
    return fail(c, DAMF_E_OOM, "host memory");
  }
  API_HIP(c, hipMemcpyAsync(desc.data(), w.chunks, h.n_chunks * sizeof(ChunkDesc), hipMemcpyDeviceToHost, s),
          "chunk list");
  API_HIP(c, hipStreamSynchronize(s), "chunk list");
  ChainStats acc{};
  for (int ch = 0; ch < h.n_chunks; ++ch) {
    // the chunk's own rows, so that a side whose scatter went through while
    // the other refused can be taken back
    const ChunkDesc &cd = desc[ch];
    API_HIP(c, launch_undo_rows(c, cd.s1_off, cd.s1, cd.s2_off, cd.s2, false), "undo log (chunk)");
    API_HIP(c, launch_chain(c, ch, ch + 1, h.n_chunks, h.meets_prev), "chain (one chunk)");
    API_HIP(c, hipMemcpyAsync(w.cstats_host, w.cstats, sizeof(ChainStats), hipMemcpyDeviceToHost, s), "stats");
    API_HIP(c, hipStreamSynchronize(s), "chain (one chunk)");
    const ChainStats one = *w.cstats_host;
    if (one.numeric_error & kNumericCore) {
      // the per-chunk undo log has overwritten the batch's, and an explicit
      // chunk may have rotated every row: no exact undo is left
      c->poisoned = true;
      return fail(c, DAMF_E_NUMERIC, "non-finite core in the update");
    }
    const bool singular = (one.numeric_error & kNumericSingularP) != 0;
    add_stats(acc, one, !singular);
    if (singular) {
      // one side's scatter may have run: take its rows back; then c->P holds
      // P F: rotate every basis by it (P <- I) and add the row corrections of
      // this chunk with the identity projection
      API_HIP(c, launch_undo_rows(c, cd.s1_off, cd.s1, cd.s2_off, cd.s2, true), "undo (chunk)");
      API_HIP(c, flush_projections(c), "explicit chunk (rotation)");
      API_HIP(c, launch_chunk_scatter(c, ch, h.n_chunks, c->P), "explicit chunk (rows)");
      c->enhance_pending = c->enhance_pending || c->ppr_on;  // R rotated
      ++c->last_explicit;
    }
  }
  API_HIP(c, hipStreamSynchronize(s), "explicit chunks");
  acc.numeric_error = 0;
  *out = acc;
  *w.cstats_host = acc;
  API_HIP(c, hipMemcpyAsync(w.cstats, w.cstats_host, sizeof(ChainStats), hipMemcpyHostToDevice, s), "stats");
  API_HIP(c, hipStreamSynchronize(s), "stats");
  return DAMF_OK;
}

}  // namespace

namespace {

// A core came out non-finite (NaN or infinite values, e.g. from singular
// values near the top of the double range): undo the whole batch instead of
// leaving a corrupt state.  The rows of U_b and V_b and P, Sigma come back
// from the undo log.  With the graph already edited (damf_update: edit,
// chain, check), R's rows come back from their copies, the chunks' S1 rows
// first (saved after the fix-up) and then the edited rows (saved before it),
// and the graph from the inverse edit: the context is then bit for bit what
// it was before the call.  Otherwise (the server: chain, check, edit) the
// previous step's push ran beside the chain, so R's saved rows are stale;
// the PPR state is seeded again from the restored basis (Z = 0, R = X, pushed
// to eps / 2), which is as valid an approximation as the one it replaces.
damf_status rollback_batch(damf_ctx *c, const BatchHeader &h, bool graph_edited) {
  hipStream_t s = c->stream;
  Workspace &w = c->ws;
  const size_t dd = 2 * (size_t)c->d * c->d;
  API_HIP(c, launch_undo_rows(c, 0, h.s1_total, 0, h.s2_total, true, false), "undo");
  API_HIP(c, hipMemcpyAsync(c->P, w.psave, dd * sizeof(double), hipMemcpyDeviceToDevice, s), "undo");
  API_HIP(c, hipMemcpyAsync(c->sigma, w.psave + dd, kMaxCore * sizeof(double), hipMemcpyDeviceToDevice, s),
          "undo");
  if (graph_edited) {
    API_HIP(c, launch_r_rows(c, w.chunk_s1, h.s1_total, kRLogS1, true), "undo (R)");
    API_HIP(c, launch_r_rows(c, w.rows_out, h.n_rows_out, 0, true), "undo (R)");
    if (h.n_net > 0) {
      API_HIP(c, launch_negate_net(c, h.n_net), "undo (graph)");
      const damf_status st = graph_edit(c, h, false);
      if (st != DAMF_OK) return st;
    }
  } else if (c->ppr_on) {
    API_HIP(c, hipDeviceSynchronize(), "undo");
    API_HIP(c, ppr_init(c), "undo (PPR seed)");
  }
  API_HIP(c, hipStreamSynchronize(s), "undo");
  return fail(c, DAMF_E_NUMERIC, "non-finite core in the update: the batch was undone");
}

}  // namespace

damf_status step_check(damf_ctx *c, const BatchHeader &h, bool graph_edited) {
  c->last_p_cond = 0.0;
  c->last_flushed = 0;
  c->last_explicit = 0;
  if (h.n_chunks <= 0) return DAMF_OK;
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  API_HIP(c, hipMemcpyAsync(w.cstats_host, w.cstats, sizeof(ChainStats), hipMemcpyDeviceToHost, s), "stats");
  API_HIP(c, hipStreamSynchronize(s), "chain");
  ChainStats cs = *w.cstats_host;
  if (cs.numeric_error & kNumericCore) return rollback_batch(c, h, graph_edited);
  if (cs.numeric_error & kNumericSingularP) {
    const damf_status st = chain_recover(c, h, &cs);
    if (st != DAMF_OK) return st;
  }
  double cond;
  std::memcpy(&cond, &cs.p_cond_bits, sizeof(double));
  c->last_p_cond = cond;
  // the lazy projection's conditioning bounds how much FP32 rounding of the
  // stored bases is amplified in U = U_b P: flush once it passes the limit
  const double limit = c->cfg.flush_cond == 0.0 ? kDefaultFlushCond : c->cfg.flush_cond;
  if (limit > 0.0 && cond > limit) {
    API_HIP(c, flush_projections(c), "flush");
    c->enhance_pending = c->enhance_pending || c->ppr_on;  // R rotated
    c->last_flushed = 1;
    c->last_p_cond = 1.0;
  }
  return DAMF_OK;
}

damf_status step_finish(damf_ctx *c, const BatchHeader &h) {
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  API_HIP(c, hipMemcpyAsync(w.cstats_host, w.cstats, sizeof(ChainStats), hipMemcpyDeviceToHost, s), "stats");
  API_HIP(c, hipMemcpyAsync(w.hdr_host, w.hdr, sizeof(BatchHeader), hipMemcpyDeviceToHost, s), "header");
  API_HIP(c, hipMemcpyAsync(w.counters_host + 8, c->out.top, sizeof(int64_t), hipMemcpyDeviceToHost, s), "pool");
  API_HIP(c, hipMemcpyAsync(w.counters_host + 9, c->in.top, sizeof(int64_t), hipMemcpyDeviceToHost, s), "pool");
  API_HIP(c, hipStreamSynchronize(s), "update");
  if (w.hdr_host->pool_overflow) {
    c->poisoned = true;
    return fail(c, DAMF_E_OOM, "graph pool exhausted");
  }
  // rows that moved left their old space behind: compact a pool once less
  // than an eighth of it is free
  if (c->out.pool_cap - w.counters_host[8] < c->out.pool_cap / 8)
    API_HIP(c, csr_compact(c, c->out, c->cfg.graph_slack, 0), "CSR compaction");
  if (c->in.pool_cap - w.counters_host[9] < c->in.pool_cap / 8)
    API_HIP(c, csr_compact(c, c->in, c->cfg.graph_slack, 0), "CSR^T compaction");
  return DAMF_OK;
}

void step_info(damf_ctx *c, const BatchHeader &h, int64_t k, damf_batch_info *info) {
  Workspace &w = c->ws;
  const bool ch = h.n_chunks > 0;
  info->ops = k;
  info->net_entries = h.n_net;
  info->chunks = h.n_chunks;
  info->max_core = ch ? w.cstats_host->max_core : 0;
  info->dropped = ch ? w.cstats_host->dropped : 0;
  info->ms_prepare = ms_between(c->ev[0], c->ev[1]);
  info->ms_chain_kernel = ch ? ms_between(c->ev[4], c->ev[5]) : 0.0;
  info->chain_flops = ch ? w.cstats_host->flops : 0.0;
  info->core_flops = ch ? w.cstats_host->core_flops : 0.0;
  info->core_flops_model = ch ? w.cstats_host->core_flops_model : 0.0;
  info->ms_core_kernel = 0.0;
  info->core_launches = ch ? c->core_timed : 0;
  for (int i = 0; ch && i < c->core_timed; ++i)
    info->ms_core_kernel += ms_between(c->ev_core[2 * i], c->ev_core[2 * i + 1]);
  info->sweeps = ch ? w.cstats_host->sweeps : 0;
  info->p_cond = c->last_p_cond;
  info->flushed = c->last_flushed;
  info->explicit_chunks = c->last_explicit;
  info->graph_launches = c->graph_launches;
  info->small_sv_columns = ch ? w.cstats_host->small_sv_columns : 0;
  for (int i = 0; i < 8; ++i)
    info->chain_phase_ms[i] = ch ? (double)w.cstats_host->phase_ticks[i] / c->wall_khz : 0.0;
}

damf_status step_push_rows(damf_ctx *c, const BatchHeader &h, int nseg, int64_t *count) {
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  *count = 0;
  if (h.n_rows_out > 0)
    API_HIP(c, hipMemcpyAsync(w.pend_rows, w.rows_out, h.n_rows_out * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, s), "push rows");
  *count = h.n_rows_out;
  if (nseg > 1 && h.s1_total > 0) {
    API_HIP(c, hipMemcpyAsync(w.pend_rows + *count, w.chunk_s1, h.s1_total * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, s), "push rows");
    *count += h.s1_total;
  }
  return DAMF_OK;
}

damf_status update_impl(damf_ctx *c, int64_t k, const int32_t *src, const int32_t *dst,
                        const int8_t *op, int32_t flags, int nseg, const int32_t *seg_end,
                        damf_batch_info *info, damf_request_stats *per_request) {
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  if (k < 0 || k > kMaxBatch) return fail(c, DAMF_E_INVALID_ARG, "batch size out of range");
  if (info) std::memset(info, 0, sizeof(*info));
  if (info) info->ops = k;
  if (per_request) std::memset(per_request, 0, nseg * sizeof(damf_request_stats));
  if (k == 0) return DAMF_OK;
  BatchHeader h{};
  damf_status st = step_prepare(c, k, src, dst, op, flags, nseg, seg_end, &h);
  if (st != DAMF_OK) return st;
  if (per_request)
    for (int i = 0; i < nseg; ++i) {
      per_request[i].net_entries = c->ws.seg_stats_host[2 * i];
      per_request[i].chunks = c->ws.seg_stats_host[2 * i + 1];
    }
  return update_apply(c, h, k, nseg, info);
}

damf_status update_apply(damf_ctx *c, const BatchHeader &h, int64_t k, int nseg,
                         damf_batch_info *info) {
  hipStream_t s = c->stream;
  damf_status st;
  if ((st = step_graph(c, h)) != DAMF_OK) return st;
  if ((st = step_chain(c, h, nseg)) != DAMF_OK) return st;
  if ((st = step_check(c, h, true)) != DAMF_OK) return st;
  // re-orthogonalisation due: before Step 4, so the push restores max |R| <= eps
  bool reorth_refused = false;
  double ms_reorth = 0.0;
  if (h.n_chunks > 0 && c->cfg.reorth_every > 0 &&
      ++c->batches_since_reorth >= c->cfg.reorth_every) {
    c->batches_since_reorth = 0;
    API_HIP(c, hipEventRecord(c->ev[6], s), "event");
    int bad = 0;
    API_HIP(c, reorthogonalize(c, &bad), "re-orthogonalisation");
    c->enhance_pending = c->enhance_pending || c->ppr_on;  // R was rotated: every row may exceed eps
    API_HIP(c, hipEventRecord(c->ev[7], s), "event");
    API_HIP(c, hipEventSynchronize(c->ev[7]), "event");
    ms_reorth = ms_between(c->ev[6], c->ev[7]);
    reorth_refused = bad != 0;
  }
  API_HIP(c, hipEventRecord(c->ev[2], s), "event");
  int64_t rounds = 0, pushes = 0, edges = 0;
  c->push_ms = 0.0;
  c->push_bytes = 0.0;
  if (c->ppr_on && c->cfg.auto_enhance) {
    // from this batch's rows, or from every node when R changed elsewhere
    // (a re-orthogonalisation or flush rotates every row of R)
    int64_t nrows = 0;
    if ((st = step_push_rows(c, h, nseg, &nrows)) != DAMF_OK) return st;
    const bool all = c->enhance_pending;
    API_HIP(c, ppr_push(c, s, all ? nullptr : c->ws.pend_rows, all ? 0 : nrows, &rounds, &pushes, &edges),
            "PPR push");
    c->enhance_pending = false;
  } else if (c->ppr_on) {
    c->enhance_pending = true;  // the next Z query or damf_enhance pushes from every node
  }
  API_HIP(c, hipEventRecord(c->ev[3], s), "event");
  if ((st = step_finish(c, h)) != DAMF_OK) return st;
  if (info) {
    step_info(c, h, k, info);
    info->push_rounds = rounds;
    info->pushes = pushes;
    info->push_edges = edges;
    info->ms_chain = ms_between(c->ev[1], c->ev[2]);
    info->ms_enhance = ms_between(c->ev[2], c->ev[3]);
    info->ms_push_kernel = c->push_ms;
    info->push_bytes = c->push_bytes;
    info->ms_reorth = ms_reorth;
  }
  if (reorth_refused)
    return fail(c, DAMF_E_NUMERIC,
                "batch applied; re-orthogonalisation refused: basis far from orthonormal");
  return DAMF_OK;
}

}  // namespace damf

extern "C" {

void damf_config_default(damf_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->n = 0;
  cfg->d = 128;
  cfg->directed = 1;
  cfg->oversample = 10;
  cfg->power_iters = 2;
  cfg->seed = 1;
  cfg->alpha = 0.15;
  cfg->eps = 1e-5;
  cfg->max_core_rank = 64;
  cfg->max_side = 64;
  cfg->tau = 1e-6;
  cfg->auto_enhance = 1;
  cfg->graph_slack = 1.25;
  cfg->hip_stream = nullptr;
}

const char *damf_status_string(damf_status s) {
  switch (s) {
    case DAMF_OK: return "ok";
    case DAMF_E_INVALID_ARG: return "invalid argument";
    case DAMF_E_OUT_OF_RANGE: return "node id or op out of range";
    case DAMF_E_OOM: return "out of device memory";
    case DAMF_E_DEVICE: return "device error";
    case DAMF_E_NUMERIC: return "numerical failure";
    case DAMF_E_STATE: return "context poisoned by an earlier device error";
    case DAMF_E_BUSY: return "admission cap reached";
    case DAMF_E_TIMEOUT: return "timed out";
  }
  return "unknown status";
}

const char *damf_last_error(const damf_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

damf_status damf_init_factors(const damf_config *cfg, int64_t m, const int32_t *src,
                              const int32_t *dst, const double *U, const double *S,
                              const double *V, int32_t flags, damf_ctx **out) {
  damf_ctx *c = nullptr;
  damf_status st = new_ctx(cfg, out, &c);
  if (st != DAMF_OK) return st;
  if (!U || !S || !V) {
    free_ctx(c);
    return DAMF_E_INVALID_ARG;
  }
  const int64_t n = c->n;
  const int d = c->d;
  for (int i = 0; i < d; ++i)
    if (!std::isfinite(S[i]) || S[i] < 0.0 || (i > 0 && S[i] > S[i - 1] * (1.0 + 1e-12))) {
      free_ctx(c);
      return DAMF_E_INVALID_ARG;
    }
  if ((st = alloc_state(c)) != DAMF_OK || (st = build_graph(c, m, src, dst, flags)) != DAMF_OK) {
    free_ctx(c);
    return st;
  }
  std::vector<float> buf;
  try {
    buf.resize((size_t)n * d);
  } catch (...) {
    free_ctx(c);
    return DAMF_E_OOM;
  }
  for (int side = 0; side < 2; ++side) {
    const double *M = side ? V : U;
    for (size_t i = 0; i < buf.size(); ++i) {
      const float f = (float)M[i];
      if (c->split) {
        const uint32_t w = split_encode(f);
        std::memcpy(&buf[i], &w, 4);
      } else {
        buf[i] = f;
      }
    }
    if (hipMemcpy(side ? c->Vb : c->Ub, buf.data(), buf.size() * sizeof(float),
                  hipMemcpyHostToDevice) != hipSuccess) {
      free_ctx(c);
      return DAMF_E_DEVICE;
    }
  }
  std::vector<double> P(2 * (size_t)d * d, 0.0);
  for (int s = 0; s < 2; ++s)
    for (int i = 0; i < d; ++i) P[s * d * d + i * d + i] = 1.0;
  std::vector<double> sig(kMaxCore, 0.0);
  std::copy(S, S + d, sig.begin());
  if (hipMemcpy(c->P, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->sigma, sig.data(), sig.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess) {
    free_ctx(c);
    return DAMF_E_DEVICE;
  }
  if (c->ppr_on) {
    if (ppr_init(c) != hipSuccess) {
      free_ctx(c);
      return DAMF_E_DEVICE;
    }
    if (c->nonfinite) {
      free_ctx(c);
      return DAMF_E_NUMERIC;
    }
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    free_ctx(c);
    return DAMF_E_DEVICE;
  }
  *out = c;
  return DAMF_OK;
}

damf_status damf_init(const damf_config *cfg, int64_t m, const int32_t *src, const int32_t *dst,
                      int32_t flags, damf_ctx **out) {
  damf_ctx *c = nullptr;
  damf_status st = new_ctx(cfg, out, &c);
  if (st != DAMF_OK) return st;
  auto t0 = std::chrono::steady_clock::now();
  if ((st = alloc_state(c)) != DAMF_OK || (st = build_graph(c, m, src, dst, flags)) != DAMF_OK) {
    free_ctx(c);
    return st;
  }
  auto t1 = std::chrono::steady_clock::now();
  hipError_t e = rsvd_init(c);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  auto t2 = std::chrono::steady_clock::now();
  if (e == hipSuccess && c->ppr_on) e = ppr_init(c);
  auto t3 = std::chrono::steady_clock::now();
  c->init_info.ms_graph = std::chrono::duration<double, std::milli>(t1 - t0).count();
  c->init_info.ms_rsvd = std::chrono::duration<double, std::milli>(t2 - t1).count();
  c->init_info.ms_ppr = std::chrono::duration<double, std::milli>(t3 - t2).count();
  c->init_info.nnz = m;
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    free_ctx(c);
    return (e == hipErrorOutOfMemory) ? DAMF_E_OOM : DAMF_E_DEVICE;
  }
  if (c->nonfinite) {  // the factorisation produced NaN or Inf
    free_ctx(c);
    return DAMF_E_NUMERIC;
  }
  *out = c;
  return DAMF_OK;
}

damf_status damf_update(damf_ctx *c, int64_t k, const int32_t *src, const int32_t *dst,
                        const int8_t *op, int32_t flags, damf_batch_info *info) {
  if (!c) return DAMF_E_INVALID_ARG;
  const int32_t seg_end = (int32_t)std::max<int64_t>(k, 0);
  return update_impl(c, k, src, dst, op, flags, 1, &seg_end, info, nullptr);
}

damf_status damf_update_requests(damf_ctx *c, int32_t nreq, const int64_t *req_ops,
                                 const int32_t *src, const int32_t *dst, const int8_t *op,
                                 int32_t flags, damf_batch_info *info,
                                 damf_request_stats *per_request) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (nreq < 1 || nreq > kMaxRequests || !req_ops)
    return fail(c, DAMF_E_INVALID_ARG, "request count out of range");
  int32_t seg_end[kMaxRequests];
  int64_t k = 0;
  for (int i = 0; i < nreq; ++i) {
    if (req_ops[i] < 0) return fail(c, DAMF_E_INVALID_ARG, "negative request size");
    k += req_ops[i];
    if (k > kMaxBatch) return fail(c, DAMF_E_INVALID_ARG, "batch size out of range");
    seg_end[i] = (int32_t)k;
  }
  return update_impl(c, k, src, dst, op, flags, nreq, seg_end, info, per_request);
}

damf_status damf_add_node(damf_ctx *c, int32_t node, int64_t k_in, const int32_t *in_nbrs,
                          int64_t k_out, const int32_t *out_nbrs, damf_batch_info *info) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (info) std::memset(info, 0, sizeof(*info));
  if (info) info->ops = k_in + k_out;
  BatchHeader h{};
  API_HIP(c, hipEventRecord(c->ev[0], c->stream), "event");
  damf_status st = node_prepare(c, node, k_in, in_nbrs, k_out, out_nbrs, &h);
  if (st != DAMF_OK) return st;
  API_HIP(c, hipEventRecord(c->ev[1], c->stream), "event");
  if (h.n_net == 0) return DAMF_OK;
  return update_apply(c, h, k_in + k_out, 1, info);
}

damf_status damf_set_chunk_rank(damf_ctx *c, int32_t r) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (r < 1 || r > c->cfg.max_side || c->d + r > kMaxCore)
    return fail(c, DAMF_E_INVALID_ARG, "chunk rank out of range");
  c->cfg.max_core_rank = r;
  return DAMF_OK;
}

damf_status damf_enhance(damf_ctx *c) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  if (!c->ppr_on) return DAMF_OK;
  int64_t r, p, e;
  API_HIP(c, ppr_push(c, c->stream, nullptr, 0, &r, &p, &e), "PPR push");
  API_HIP(c, hipStreamSynchronize(c->stream), "PPR push");
  c->enhance_pending = false;
  return DAMF_OK;
}

damf_status damf_flush(damf_ctx *c) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  API_HIP(c, flush_projections(c), "flush");
  c->enhance_pending = c->enhance_pending || c->ppr_on;  // R rotated
  return DAMF_OK;
}

damf_status damf_reorthogonalize(damf_ctx *c) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  int bad = 0;
  API_HIP(c, reorthogonalize(c, &bad), "re-orthogonalisation");
  if (bad) return fail(c, DAMF_E_NUMERIC, "re-orthogonalisation refused: basis far from orthonormal");
  c->batches_since_reorth = 0;
  c->enhance_pending = c->enhance_pending || c->ppr_on;  // R rotated
  return DAMF_OK;
}

damf_status damf_query(damf_ctx *c, damf_which which, int64_t q, const int32_t *nodes,
                       float *out, int32_t flags) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  if (which < DAMF_X || which > DAMF_Z || q < 0 || !out) return fail(c, DAMF_E_INVALID_ARG, "bad query");
  if (!nodes && q != c->n) return fail(c, DAMF_E_INVALID_ARG, "q must be n without a node list");
  if (q == 0) return DAMF_OK;
  const int d = c->d;
  hipStream_t s = c->stream;
  if (which == DAMF_Z && !c->ppr_on) which = DAMF_X;  // alpha = 1: Z = X
  if (which == DAMF_Z && c->enhance_pending) {          // Z within eps of PPR(X) when read
    const damf_status st = damf_enhance(c);
    if (st != DAMF_OK) return st;
  }
  const int32_t *dn = nodes;
  float *dout = out;
  int32_t *own_n = nullptr;
  float *own_o = nullptr;
  if ((flags & DAMF_DEVICE_PTRS) && nodes) {
    // device list: a read-only counting pass before any row is read
    int64_t *bad = c->ws.counters + 12;
    API_HIP(c, launch_count_bad_ids(nodes, q, c->n, bad, s), "query id check");
    API_HIP(c, hipMemcpyAsync(c->ws.counters_host + 12, bad, sizeof(int64_t), hipMemcpyDeviceToHost, s),
            "query id check");
    API_HIP(c, hipStreamSynchronize(s), "query id check");
    if (c->ws.counters_host[12] != 0) return fail(c, DAMF_E_OUT_OF_RANGE, "query id out of range");
  }
  if (!(flags & DAMF_DEVICE_PTRS)) {
    if (nodes) {
      for (int64_t i = 0; i < q; ++i)
        if (nodes[i] < 0 || nodes[i] >= c->n) return fail(c, DAMF_E_OUT_OF_RANGE, "query id out of range");
      API_HIP(c, dalloc(&own_n, q), "alloc query");
      API_HIP(c, hipMemcpyAsync(own_n, nodes, q * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy query");
      dn = own_n;
    }
    API_HIP(c, dalloc(&own_o, q * d), "alloc query");
    dout = own_o;
  }
  API_HIP(c, launch_query(c, which, q, dn, dout), "query");
  if (own_o) {
    API_HIP(c, hipMemcpyAsync(out, own_o, q * d * sizeof(float), hipMemcpyDeviceToHost, s), "copy query");
  }
  API_HIP(c, hipStreamSynchronize(s), "query");
  if (own_n) (void)hipFree(own_n);
  if (own_o) (void)hipFree(own_o);
  return DAMF_OK;
}

damf_status damf_query_static(damf_ctx *c, damf_which which, int64_t q, const int32_t *nodes,
                              float *out, int32_t flags) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  if (which < DAMF_X || which > DAMF_Z || q < 0 || !out) return fail(c, DAMF_E_INVALID_ARG, "bad query");
  if (!nodes && q != c->n) return fail(c, DAMF_E_INVALID_ARG, "q must be n without a node list");
  if (q == 0) return DAMF_OK;
  const int d = c->d;
  hipStream_t s = c->stream;
  if (which == DAMF_Z && !c->ppr_on) which = DAMF_X;  // alpha = 1: Z = X
  // Step 4 may grow its workspace, so a pending enhancement is not run here
  if (which == DAMF_Z && c->enhance_pending)
    return fail(c, DAMF_E_INVALID_ARG, "Z query with Step 4 pending: call damf_enhance first");
  const bool dev = (flags & DAMF_DEVICE_PTRS) != 0;
  // scratch layout: counter slot [0, 256); ids from 256; rows after the ids
  const size_t ids_bytes = (!dev && nodes) ? (((size_t)q * sizeof(int32_t) + 255) / 256) * 256 : 0;
  const size_t need = dev ? 256 : 256 + ids_bytes + (size_t)q * d * sizeof(float);
  if (need > kStaticScratchBytes)
    return fail(c, DAMF_E_INVALID_ARG, "query larger than the 4 MiB static scratch (host pointers)");
  unsigned char *base = static_cast<unsigned char *>(static_scratch_ptr(c->device));
  if (!base) return fail(c, DAMF_E_STATE, "static scratch not set up on this device");
  int64_t *bad = reinterpret_cast<int64_t *>(base);
  const int32_t *dn = nodes;
  float *dout = out;
  if (dev && nodes) {
    API_HIP(c, launch_count_bad_ids(nodes, q, c->n, bad, s), "query id check");
    API_HIP(c, hipMemcpyAsync(c->ws.counters_host + 12, bad, sizeof(int64_t), hipMemcpyDeviceToHost, s),
            "query id check");
    API_HIP(c, hipStreamSynchronize(s), "query id check");
    if (c->ws.counters_host[12] != 0) return fail(c, DAMF_E_OUT_OF_RANGE, "query id out of range");
  }
  if (!dev) {
    if (nodes) {
      for (int64_t i = 0; i < q; ++i)
        if (nodes[i] < 0 || nodes[i] >= c->n) return fail(c, DAMF_E_OUT_OF_RANGE, "query id out of range");
      int32_t *ids = reinterpret_cast<int32_t *>(base + 256);
      API_HIP(c, hipMemcpyAsync(ids, nodes, q * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy query");
      dn = ids;
    }
    dout = reinterpret_cast<float *>(base + 256 + ids_bytes);
  }
  API_HIP(c, launch_query(c, which, q, dn, dout), "query");
  if (!dev)
    API_HIP(c, hipMemcpyAsync(out, dout, (size_t)q * d * sizeof(float), hipMemcpyDeviceToHost, s), "copy query");
  API_HIP(c, hipStreamSynchronize(s), "query");
  return DAMF_OK;
}

damf_status damf_score_pairs(damf_ctx *c, damf_which which_a, damf_which which_b, int64_t q,
                             const int32_t *u, const int32_t *v, float *out, int32_t flags) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  if (which_a < DAMF_X || which_a > DAMF_Z || which_b < DAMF_X || which_b > DAMF_Z || q < 0 ||
      (q > 0 && (!u || !v || !out)))
    return fail(c, DAMF_E_INVALID_ARG, "bad pair scoring arguments");
  if (q == 0) return DAMF_OK;
  hipStream_t s = c->stream;
  if (!c->ppr_on) {  // alpha = 1: Z = X
    if (which_a == DAMF_Z) which_a = DAMF_X;
    if (which_b == DAMF_Z) which_b = DAMF_X;
  }
  if ((which_a == DAMF_Z || which_b == DAMF_Z) && c->enhance_pending) {
    const damf_status st = damf_enhance(c);
    if (st != DAMF_OK) return st;
  }
  const bool both = (flags & DAMF_SCORE_BOTH_WAYS) != 0;
  const int32_t *du = u, *dv = v;
  float *dout = out;
  int32_t *own = nullptr;
  float *own_o = nullptr;
  if (flags & DAMF_DEVICE_PTRS) {
    int64_t *bad = c->ws.counters + 12;
    API_HIP(c, launch_count_bad_ids(u, q, c->n, bad, s), "pair id check");
    API_HIP(c, hipMemcpyAsync(c->ws.counters_host + 12, bad, sizeof(int64_t), hipMemcpyDeviceToHost, s),
            "pair id check");
    API_HIP(c, hipStreamSynchronize(s), "pair id check");
    if (c->ws.counters_host[12] != 0) return fail(c, DAMF_E_OUT_OF_RANGE, "pair id out of range");
    API_HIP(c, launch_count_bad_ids(v, q, c->n, bad, s), "pair id check");
    API_HIP(c, hipMemcpyAsync(c->ws.counters_host + 12, bad, sizeof(int64_t), hipMemcpyDeviceToHost, s),
            "pair id check");
    API_HIP(c, hipStreamSynchronize(s), "pair id check");
    if (c->ws.counters_host[12] != 0) return fail(c, DAMF_E_OUT_OF_RANGE, "pair id out of range");
  } else {
    for (int64_t i = 0; i < q; ++i)
      if (u[i] < 0 || u[i] >= c->n || v[i] < 0 || v[i] >= c->n)
        return fail(c, DAMF_E_OUT_OF_RANGE, "pair id out of range");
    API_HIP(c, dalloc(&own, 2 * q), "alloc pairs");
    API_HIP(c, dalloc(&own_o, q), "alloc pairs");
    API_HIP(c, hipMemcpyAsync(own, u, q * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy pairs");
    API_HIP(c, hipMemcpyAsync(own + q, v, q * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy pairs");
    du = own;
    dv = own + q;
    dout = own_o;
  }
  API_HIP(c, launch_score_pairs(c, which_a, which_b, q, du, dv, dout, both), "score pairs");
  if (own_o) API_HIP(c, hipMemcpyAsync(out, own_o, q * sizeof(float), hipMemcpyDeviceToHost, s), "copy scores");
  API_HIP(c, hipStreamSynchronize(s), "score pairs");
  if (own) (void)hipFree(own);
  if (own_o) (void)hipFree(own_o);
  return DAMF_OK;
}

damf_status damf_singular_values(damf_ctx *c, double *out) {
  if (!c || !out) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  API_HIP(c, hipMemcpyAsync(out, c->sigma, c->d * sizeof(double), hipMemcpyDeviceToHost, c->stream), "sigma");
  API_HIP(c, hipStreamSynchronize(c->stream), "sigma");
  return DAMF_OK;
}

damf_status damf_export_csr(damf_ctx *c, int32_t transpose, int64_t *indptr, int32_t *indices,
                            int64_t *m_out) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  API_HIP(c, csr_export(c, transpose ? c->in : c->out, indptr, indices, m_out), "export CSR");
  return DAMF_OK;
}

damf_status damf_export_state(damf_ctx *c, double *Ub, double *Vb, double *PU, double *PV,
                              double *Zb, double *R) {
  if (!c) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  const size_t nd = (size_t)c->n * c->d;
  const int d = c->d;
  API_HIP(c, hipStreamSynchronize(c->stream), "export");
  std::vector<float> buf;
  try {
    buf.resize(nd);
  } catch (...) {
    return fail(c, DAMF_E_OOM, "export: host memory");
  }
  bool split = c->split;
  auto pull = [&](const float *src, double *dst) -> hipError_t {
    if (!dst) return hipSuccess;
    if (!src) {
      std::fill(dst, dst + nd, 0.0);
      return hipSuccess;
    }
    hipError_t e = hipMemcpy(buf.data(), src, nd * sizeof(float), hipMemcpyDeviceToHost);
    for (size_t i = 0; i < nd; ++i) {
      if (split) {
        uint32_t w;
        std::memcpy(&w, &buf[i], 4);
        dst[i] = split_decode(w);
      } else {
        dst[i] = buf[i];
      }
    }
    return e;
  };
  API_HIP(c, pull(c->Ub, Ub), "export U_b");
  API_HIP(c, pull(c->Vb, Vb), "export V_b");
  split = false;  // Z_b and the residual R are FP32 in both forms
  API_HIP(c, pull(c->Zb, Zb), "export Z_b");
  API_HIP(c, pull(c->R, R), "export R");
  if (PU) API_HIP(c, hipMemcpy(PU, c->P, (size_t)d * d * sizeof(double), hipMemcpyDeviceToHost), "export P");
  if (PV) API_HIP(c, hipMemcpy(PV, c->P + (size_t)d * d, (size_t)d * d * sizeof(double), hipMemcpyDeviceToHost), "export P");
  return DAMF_OK;
}

damf_status damf_get_init_info(damf_ctx *c, damf_init_info *info) {
  if (!c || !info) return DAMF_E_INVALID_ARG;
  *info = c->init_info;
  return DAMF_OK;
}

damf_status damf_residual_max(damf_ctx *c, double *out) {
  if (!c || !out) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  if (!c->ppr_on) {
    *out = 0.0;
    return DAMF_OK;
  }
  API_HIP(c, ppr_residual_max(c, out), "residual max");
  return DAMF_OK;
}

damf_status damf_sync(damf_ctx *c) {
  if (!c) return DAMF_E_INVALID_ARG;
  API_HIP(c, hipStreamSynchronize(c->stream), "sync");
  return DAMF_OK;
}

// ---- checkpoint: the whole state of a context in one file
//
// Layout (host byte order): CkptHeader; out-CSR indptr (n + 1 int64) and
// indices (m int32), canonical; P (2 d d FP64); Sigma (kMaxCore FP64);
// U_b, V_b (n d 32-bit words each, as stored: FP32 or BF16 pairs); with PPR,
// Z_b and R (n d FP32 each).  Matrices stream through a pinned buffer.

namespace {

struct CkptHeader {
  char magic[8];
  int64_t version, n, m, batches_since_reorth, round_counter;
  int32_t d, directed, precision, ppr_on, enhance_pending, pad;
  double alpha;
};
constexpr char kCkptMagic[8] = {'D', 'A', 'M', 'F', 'C', 'K', 'P', '1'};
constexpr size_t kCkptChunk = size_t(64) << 20;  // bytes per staged copy

// Device <-> file in chunks through one pinned buffer.
hipError_t stream_out(FILE *f, const void *dev, size_t bytes, void *pin, hipStream_t s, bool *io_ok) {
  for (size_t off = 0; off < bytes; off += kCkptChunk) {
    const size_t len = std::min(kCkptChunk, bytes - off);
    hipError_t e = hipMemcpyAsync(pin, (const char *)dev + off, len, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (std::fwrite(pin, 1, len, f) != len) {
      *io_ok = false;
      return hipSuccess;
    }
  }
  return hipSuccess;
}
hipError_t stream_in(FILE *f, void *dev, size_t bytes, void *pin, hipStream_t s, bool *io_ok) {
  for (size_t off = 0; off < bytes; off += kCkptChunk) {
    const size_t len = std::min(kCkptChunk, bytes - off);
    if (std::fread(pin, 1, len, f) != len) {
      *io_ok = false;
      return hipSuccess;
    }
    hipError_t e = hipMemcpyAsync((char *)dev + off, pin, len, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

damf_status damf_save(damf_ctx *c, const char *path) {
  if (!c || !path) return DAMF_E_INVALID_ARG;
  if (c->poisoned) return fail(c, DAMF_E_STATE, "context poisoned");
  const int64_t n = c->n;
  const int d = c->d;
  int64_t m = 0;
  API_HIP(c, csr_export(c, c->out, nullptr, nullptr, &m), "checkpoint CSR");
  std::vector<int64_t> indptr;
  std::vector<int32_t> indices;
  try {
    indptr.resize(n + 1);
    indices.resize(m > 0 ? m : 1);
  } catch (...) {
    return fail(c, DAMF_E_OOM, "checkpoint: host memory for the CSR");
  }
  API_HIP(c, csr_export(c, c->out, indptr.data(), indices.data(), &m), "checkpoint CSR");
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(c, DAMF_E_INVALID_ARG, "cannot open the checkpoint file for writing");
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = 1;
  h.n = n;
  h.m = m;
  h.batches_since_reorth = c->batches_since_reorth;
  h.round_counter = c->round_counter;
  h.d = d;
  h.directed = c->cfg.directed;
  h.precision = c->split ? 1 : 0;
  h.ppr_on = c->ppr_on ? 1 : 0;
  h.enhance_pending = c->enhance_pending ? 1 : 0;
  h.alpha = c->cfg.alpha;
  bool io = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
            std::fwrite(indptr.data(), sizeof(int64_t), n + 1, f) == (size_t)(n + 1) &&
            (m == 0 || std::fwrite(indices.data(), sizeof(int32_t), m, f) == (size_t)m);
  void *pin = nullptr;
  hipError_t e = io ? hipHostMalloc(&pin, kCkptChunk) : hipSuccess;
  const size_t nd = (size_t)n * d * sizeof(float);
  if (io && e == hipSuccess) e = stream_out(f, c->P, 2 * (size_t)d * d * sizeof(double), pin, c->stream, &io);
  if (io && e == hipSuccess) e = stream_out(f, c->sigma, kMaxCore * sizeof(double), pin, c->stream, &io);
  if (io && e == hipSuccess) e = stream_out(f, c->Ub, nd, pin, c->stream, &io);
  if (io && e == hipSuccess) e = stream_out(f, c->Vb, nd, pin, c->stream, &io);
  if (c->ppr_on && io && e == hipSuccess) e = stream_out(f, c->Zb, nd, pin, c->stream, &io);
  if (c->ppr_on && io && e == hipSuccess) e = stream_out(f, c->R, nd, pin, c->stream, &io);
  if (pin) (void)hipHostFree(pin);
  io = (std::fclose(f) == 0) && io;
  if (e != hipSuccess) return dev_fail(c, e, "checkpoint");
  if (!io) return fail(c, DAMF_E_INVALID_ARG, "checkpoint file write failed");
  return DAMF_OK;
}

damf_status damf_load(const char *path, const damf_config *cfg, damf_ctx **out) {
  if (!path || !cfg || !out) return DAMF_E_INVALID_ARG;
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return DAMF_E_INVALID_ARG;
  CkptHeader h{};
  const bool hdr_ok = std::fread(&h, sizeof(h), 1, f) == 1 &&
                      std::memcmp(h.magic, kCkptMagic, 8) == 0 && h.version == 1;
  const bool ppr_on = cfg->alpha < 1.0;
  if (!hdr_ok || h.n != cfg->n || h.d != cfg->d || h.directed != cfg->directed ||
      h.precision != cfg->precision || h.ppr_on != (ppr_on ? 1 : 0) ||
      (ppr_on && h.alpha != cfg->alpha) || h.m < 0 || check_config(cfg) != DAMF_OK) {
    std::fclose(f);
    return DAMF_E_INVALID_ARG;
  }
  // the file must hold exactly what the header promises: this bounds m
  // before anything is allocated from it
  {
    const int64_t nd_bytes = h.n * (int64_t)h.d * (int64_t)sizeof(float);
    const int64_t fixed = (int64_t)sizeof(CkptHeader) + 8 * (h.n + 1) +
                          2 * (int64_t)h.d * h.d * (int64_t)sizeof(double) +
                          kMaxCore * (int64_t)sizeof(double) + (ppr_on ? 4 : 2) * nd_bytes;
    int64_t size = -1;
    if (fseeko(f, 0, SEEK_END) == 0) size = (int64_t)ftello(f);
    if (size < fixed || (size - fixed) % 4 != 0 || (size - fixed) / 4 != h.m ||
        fseeko(f, (off_t)sizeof(CkptHeader), SEEK_SET) != 0) {
      std::fclose(f);
      return DAMF_E_INVALID_ARG;
    }
  }
  const int64_t n = h.n, m = h.m;
  std::vector<int64_t> indptr;
  std::vector<int32_t> dst, src;
  try {
    indptr.resize(n + 1);
    dst.resize(m > 0 ? m : 1);
    src.resize(m > 0 ? m : 1);
  } catch (...) {
    std::fclose(f);
    return DAMF_E_OOM;
  }
  bool io = std::fread(indptr.data(), sizeof(int64_t), n + 1, f) == (size_t)(n + 1) &&
            (m == 0 || std::fread(dst.data(), sizeof(int32_t), m, f) == (size_t)m) &&
            indptr[0] == 0 && indptr[n] == m;
  // every row range inside [0, m] and in order, before src is written
  for (int64_t u = 0; io && u < n; ++u)
    if (indptr[u + 1] < indptr[u] || indptr[u + 1] > m) io = false;
  for (int64_t u = 0; io && u < n; ++u)
    for (int64_t e = indptr[u]; e < indptr[u + 1]; ++e) src[e] = (int32_t)u;
  if (!io) {
    std::fclose(f);
    return DAMF_E_INVALID_ARG;
  }
  damf_ctx *c = nullptr;
  damf_status st = new_ctx(cfg, out, &c);
  if (st != DAMF_OK) {
    std::fclose(f);
    return st;
  }
  if ((st = alloc_state(c)) != DAMF_OK || (st = build_graph(c, m, src.data(), dst.data(), 0)) != DAMF_OK) {
    std::fclose(f);
    free_ctx(c);
    return st;
  }
  void *pin = nullptr;
  hipError_t e = hipHostMalloc(&pin, kCkptChunk);
  const size_t nd = (size_t)n * h.d * sizeof(float);
  if (e == hipSuccess) e = stream_in(f, c->P, 2 * (size_t)h.d * h.d * sizeof(double), pin, c->stream, &io);
  if (io && e == hipSuccess) e = stream_in(f, c->sigma, kMaxCore * sizeof(double), pin, c->stream, &io);
  if (io && e == hipSuccess) e = stream_in(f, c->Ub, nd, pin, c->stream, &io);
  if (io && e == hipSuccess) e = stream_in(f, c->Vb, nd, pin, c->stream, &io);
  if (ppr_on && io && e == hipSuccess) e = stream_in(f, c->Zb, nd, pin, c->stream, &io);
  if (ppr_on && io && e == hipSuccess) e = stream_in(f, c->R, nd, pin, c->stream, &io);
  if (pin) (void)hipHostFree(pin);
  std::fclose(f);
  if (e != hipSuccess || !io) {
    free_ctx(c);
    return e != hipSuccess ? DAMF_E_DEVICE : DAMF_E_INVALID_ARG;
  }
  c->batches_since_reorth = h.batches_since_reorth;
  c->round_counter = h.round_counter;
  c->enhance_pending = h.enhance_pending != 0;
  *out = c;
  return DAMF_OK;
}

void damf_destroy(damf_ctx *c) { free_ctx(c); }

}  // extern "C"
