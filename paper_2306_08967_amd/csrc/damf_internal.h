// damf_internal.h -- device state and kernel entry points shared by the
// library's translation units.  Not part of the public ABI (include/damf.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <map>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/damf.h"

namespace damf {

constexpr int64_t kMaxNodes = int64_t(1) << 30;  // nodes per context
constexpr int kMaxBatch = 8192;     // ops per damf_update call (sorted in LDS)
constexpr int kMaxCore = 192;       // d + chunk rank <= kMaxCore (Jacobi in VGPRs)
constexpr int kMaxD = 128;          // embedding width
constexpr int kMaxSide = 64;        // |S1|, |S2| per chunk
constexpr int kChainThreads = 512;  // one workgroup (8 waves) runs Steps 1-3
constexpr int kMaxRequests = 256;   // request segments per batch
constexpr int64_t kEditStagePool = 1 << 24;  // staging entries for long-row edits
constexpr double kDefaultFlushCond = 1e3;    // flush P once its condition estimate passes this

// Dynamic CSR with per-row slack.  Row u occupies col[start[u] .. start[u] +
// len[u]) in ascending order; cap[u] >= len[u] entries are reserved there.
// Rows that outgrow their reservation move to fresh space taken from the pool
// by a device-side bump pointer (*top).
struct Csr {
  int64_t *start = nullptr;
  int32_t *len = nullptr;
  int32_t *cap = nullptr;
  int32_t *col = nullptr;
  int64_t pool_cap = 0;
  int64_t *top = nullptr;  // device counter: first free pool entry
  int64_t nnz_built = 0;    // entries when the CSR was built
};

// One net edit of A (after set semantics), sorted by (row, col).
struct NetEntry {
  int32_t row, col;
  int32_t delta;  // +1 / -1
  int32_t pad;
};

// Chunk descriptor (Sec. 4.3 with B, C of several columns): rows S1 and
// columns S2 as index ranges into the chunk lists, entries as a range of
// NetEntry.
struct ChunkDesc {
  int32_t s1_off, s1, s2_off, s2;
  int32_t e_off, ne;
  int32_t pad0, pad1;
};

// Written by the batch-preparation kernel, read back by the host.
struct BatchHeader {
  int32_t bad_ops;        // ops with an id out of range or op not +1/-1
  int32_t n_net;          // net entries (both orientations for undirected)
  int32_t n_chunks;
  int32_t n_rows_out;     // distinct rows touched in A
  int32_t n_rows_in;      // distinct rows touched in A^T
  int32_t max_s;          // largest |S1| or |S2|
  int32_t pool_overflow;  // CSR rows that found no pool space (set by edits)
  int32_t s1_total;       // entries of all chunks' S1 lists
  int32_t s2_total;       // entries of all chunks' S2 lists
  int32_t pad_;
  // bit j: chunk j's S1 meets chunk j-1's S1, or its S2 meets chunk j-1's S2
  uint64_t meets_prev[kMaxBatch / 64];
};

// ChainStats::numeric_error bits
constexpr int32_t kNumericSingularP = 1;  // new P past the chunk limit: scatter refused
constexpr int32_t kNumericCore = 2;       // non-finite core (corrupt state)

// Per-chunk results written by the chain kernels (for batch info).
struct ChainStats {
  int32_t max_core;
  int32_t dropped;
  int32_t sweeps;
  int32_t numeric_error;  // kNumeric* bits
  double flops;  // FP64 flops executed (counted per phase)
  uint64_t phase_ticks[8];  // wall-clock ticks per phase (see chain.hip)
  double core_flops;        // the core-SVD kernel's share of flops
  double core_flops_model;  // 9 N^3 per sweep (one-sided Jacobi with V accumulated)
  uint64_t p_cond_bits;     // max over chunks of the new P's condition estimate (double bits)
  int32_t small_sv_columns; // right-vector columns re-orthogonalised (small singular value)
  int32_t pad_;
};

struct Workspace {
  // batch preparation
  int32_t *ops_src = nullptr, *ops_dst = nullptr;
  int8_t *ops_op = nullptr;
  uint64_t *units = nullptr;     // edit units per request, (request, edge) order
  int32_t *unit_seg = nullptr;   // request of each unit
  uint64_t *units_comb = nullptr;  // units of the whole batch's net change
  int32_t *seg_end = nullptr;    // request segments (exclusive op ends)
  int32_t *seg_stats = nullptr;  // per request: net entries, chunks
  int32_t *seg_stats_host = nullptr;  // pinned
  int32_t *pend_rows = nullptr;  // first push candidates of a deferred Step 4
  float *hbuf = nullptr;         // Step 4: taken residuals of heavy frontier nodes
  int32_t *hnode = nullptr;      // their node ids
  void *hseg = nullptr;          // (heavy node, segment) pairs (int2)
  int64_t heavy_cap = 0, hseg_cap = 0;
  int64_t *push_ring = nullptr;  // per-round push counters (ring of sets)
  int64_t *push_log = nullptr;   // per round: frontier size, edges
  int64_t *push_log_host = nullptr;  // pinned
  int32_t *edit_stage = nullptr;     // staging pool for in-place edits of long rows
  int64_t *edit_stage_top = nullptr; // its bump counter (reset per edit launch)
  NetEntry *chunk_ent = nullptr; // entries of each chunk, chunk after chunk
  NetEntry *net = nullptr;       // sorted by (row, col)
  NetEntry *net_t = nullptr;     // same entries sorted by (col, row)
  int32_t *rows_out = nullptr;   // distinct rows of net (CSR edit list)
  int32_t *rowpos_out = nullptr; // start of each row's run in net (+1 sentinel)
  int32_t *rows_in = nullptr;
  int32_t *rowpos_in = nullptr;
  ChunkDesc *chunks = nullptr;
  int32_t *chunk_s1 = nullptr;   // concatenated sorted S1 lists
  int32_t *chunk_s2 = nullptr;
  BatchHeader *hdr = nullptr;    // device
  BatchHeader *hdr_host = nullptr;  // pinned
  ChainStats *cstats = nullptr;
  ChainStats *cstats_host = nullptr;
  // chain kernels' scratch (float64, L2 resident)
  double *scratch = nullptr;
  size_t scratch_doubles = 0;
  // state before the chunks of a batch, for the explicit re-run of a batch in
  // which a projection turned singular: U_b rows of every chunk's S1 and V_b
  // rows of every chunk's S2 (as stored, in chunk-list order), P and Sigma
  float *undo_u = nullptr, *undo_v = nullptr;
  // rows of R the update touches before Step 4: the edited rows before the
  // structural fix-up (from row 0), the chunks' S1 rows before the chain
  // (from row kRLogS1)
  float *undo_r = nullptr;
  double *psave = nullptr;  // 2 d^2 + kMaxCore
  // PPR push
  int32_t *stamp = nullptr;      // per node: last round it was queued
  int32_t *cand = nullptr;       // candidate list (n)
  int32_t *cand2 = nullptr;      // next round's candidates (n)
  int32_t *frontier = nullptr;   // frontier list (n)
  int64_t *counters = nullptr;   // device counters: 0-7 Step 4 (cand, frontier, edges, ...),
                                 // 8-11 CSR pool tops and needs, 12 bad query ids,
                                 // 13 a joining node's two degrees (node.hip)
  int64_t *counters_host = nullptr;
  double *dscratch_host = nullptr;
};

}  // namespace damf

struct damf_ctx {
  damf_config cfg{};
  int64_t n = 0;
  int d = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  bool poisoned = false;
  bool nonfinite = false;  // a residual maximum came out NaN or infinite
  bool enhance_pending = false;  // batches ran without Step 4 since the last push
  std::string err;
  damf::Csr out, in;
  float *Ub = nullptr, *Vb = nullptr, *Zb = nullptr, *R = nullptr;
  double *P = nullptr;     // [P_U | P_V] (2 d x d, row-major)
  double *Pnext = nullptr; // double buffer for the chain kernels
  double *sigma = nullptr; // d
  damf::Workspace ws;
  int64_t round_counter = 0;
  bool ppr_on = true;
  hipEvent_t ev[8] = {};
  hipEvent_t ev_k[2] = {};  // per-kernel timing inside multi-launch stages
  static constexpr int kCoreTimed = 256;  // core-SVD launches timed per batch
  hipEvent_t ev_core[2 * kCoreTimed] = {};  // created only with cfg.kernel_timing
  int core_timed = 0;                       // launches timed by the last chain
  // Step 3's solve-and-scatter runs on scatter_stream, beside the next
  // chunk's core; ev_back / ev_front / ev_scatter order the two streams
  // (rings of 4)
  hipStream_t scatter_stream = nullptr;
  hipEvent_t ev_back[4] = {}, ev_front[4] = {}, ev_scatter[4] = {};
  damf_init_info init_info{};
  double push_ms = 0.0, push_bytes = 0.0;  // accumulated by ppr_push
  double wall_khz = 100000.0;               // device wall-clock rate (kHz)
  int64_t batches_since_reorth = 0;
  double last_p_cond = 0.0;  // condition estimate of P after the last batch's chunks
  int last_flushed = 0;      // the last batch flushed P (condition limit)
  int last_explicit = 0;     // chunks of the last batch applied explicitly
  // captured chain launch sequences (graph_chunks), keyed by chunk count and
  // the chunks that wait for their predecessor
  // captured chains by (bits of chunks that meet their predecessor, bits of
  // chunks that wait for its scatter, chunk count)
  std::map<std::tuple<uint64_t, uint64_t, int>, hipGraphExec_t> graphs;
  // chunks of this batch whose front waits for the previous chunk's
  // solve-and-scatter instead of adding its corrections: the first chunk of a
  // request (after the first) that meets the previous request's last chunk,
  // so that a request's result does not depend on being served with others
  uint64_t chain_hold[damf::kMaxBatch / 64] = {};
  int64_t graph_launches = 0;
  bool split = false;  // U_b, V_b as BF16 pairs (precision form)
};

namespace damf {

// ---- api.hip: the steps of one update, shared by damf_update and the server
damf_status api_fail(damf_ctx *c, damf_status s, const char *msg);
damf_status api_dev_fail(damf_ctx *c, hipError_t e, const char *where);
// Copies ops and request segments to the device, validates, prepares the
// batch and reads its header back (no state changes).
damf_status step_prepare(damf_ctx *c, int64_t k, const int32_t *src, const int32_t *dst,
                         const int8_t *op, int32_t flags, int nseg, const int32_t *seg_end,
                         BatchHeader *h);
// Structural PPR fix-up and CSR edits of A and A^T (asynchronous).
damf_status step_graph(damf_ctx *c, const BatchHeader &h);
// Steps 1-3 over every chunk (asynchronous).
damf_status step_chain(damf_ctx *c, const BatchHeader &h, int nseg);
// Waits for the chunks, re-runs a batch whose projection turned singular
// (explicit chunks), poisons on a non-finite core, and flushes the lazy
// projections when their condition estimate passes the configured limit.
damf_status step_check(damf_ctx *c, const BatchHeader &h, bool graph_edited);
// Waits for the stream, checks pool overflow and compacts the CSR pools.
damf_status step_finish(damf_ctx *c, const BatchHeader &h);
void step_info(damf_ctx *c, const BatchHeader &h, int64_t k, damf_batch_info *info);
// First-round Step 4 candidates into ws.pend_rows: rows of the net change and,
// with several requests, every chunk's S1 rows (rows whose R got a signal).
damf_status step_push_rows(damf_ctx *c, const BatchHeader &h, int nseg, int64_t *count);
// The steps after batch preparation (graph edits, Steps 1-3, checks,
// re-orthogonalisation when due, Step 4, statistics) for a prepared header.
damf_status update_apply(damf_ctx *c, const BatchHeader &h, int64_t k, int nseg,
                         damf_batch_info *info);
// ---- node.hip: node change (Theorem 1) prepared as chunks on the host
damf_status node_prepare(damf_ctx *c, int32_t node, int64_t k_in, const int32_t *in_nbrs,
                         int64_t k_out, const int32_t *out_nbrs, BatchHeader *h);
damf_status update_impl(damf_ctx *c, int64_t k, const int32_t *src, const int32_t *dst,
                        const int8_t *op, int32_t flags, int nseg, const int32_t *seg_end,
                        damf_batch_info *info, damf_request_stats *per_request);

// ---- graph.hip
hipError_t csr_build(damf_ctx *c, Csr &g, const int32_t *d_rows,
                     const int32_t *d_cols, int64_t m, double slack);
hipError_t csr_free(Csr &g);
hipError_t csr_export(damf_ctx *c, const Csr &g, int64_t *h_indptr,
                      int32_t *h_indices, int64_t *m_out);
hipError_t launch_validate_edges(const int32_t *src, const int32_t *dst,
                                 int64_t m, int64_t n, int32_t *bad,
                                 hipStream_t s);
hipError_t launch_batch_prepare(damf_ctx *c, int k, int nseg);
hipError_t csr_compact(damf_ctx *c, Csr &g, double slack, int64_t min_free);
hipError_t launch_csr_need(damf_ctx *c, const Csr &g, const NetEntry *net, const int32_t *rows,
                           const int32_t *rowpos, int nrows, int64_t *need);
hipError_t launch_csr_edit(damf_ctx *c, Csr &g, const NetEntry *net,
                           const int32_t *rows, const int32_t *rowpos,
                           int nrows, bool transposed);

// ---- chain.hip
// Steps 1-3 for chunks [first, last) of the n_chunks prepared ones, starting
// from c->P and leaving the last projection in c->P.
hipError_t launch_chain(damf_ctx *c, int first, int last, int n_chunks, const uint64_t *meets);
// All n_chunks chunks as one captured HIP graph when n_chunks <= graph_chunks
// and kernel timing is off (*used = true); the graph is built on first use of
// its shape and replayed after.  Otherwise nothing is launched (*used = false).
hipError_t launch_chain_graph(damf_ctx *c, int n_chunks, const uint64_t *meets, bool *used);
// The solve-and-scatter of chunk ch alone with projection Pn (2 d x d), on
// the context stream: rows += (row corrections of ch) Pn^-1.
hipError_t launch_chunk_scatter(damf_ctx *c, int ch, int n_chunks, const double *Pn);

// ---- ppr.hip
hipError_t ppr_init(damf_ctx *c);
hipError_t ppr_fixup(damf_ctx *c, int n_rows);
hipError_t ppr_push(damf_ctx *c, hipStream_t s, const int32_t *first_rows, int64_t nfirst,
                    int64_t *rounds, int64_t *pushes, int64_t *edges);
hipError_t ppr_residual_max(damf_ctx *c, double *out);

// ---- spmm.hip: Y = A X with long rows split into fixed segments
struct SpmmPlan {
  int64_t nlong = 0, nseg = 0;     // rows longer than one segment, their segments
  int32_t *long_row = nullptr;     // long rows
  int64_t *long_seg0 = nullptr;    // first segment of each long row
  int32_t *seg_row = nullptr, *seg_idx = nullptr;  // row and index of each segment
  float *part = nullptr;           // partial row sums, nseg x ld_max
  int ld_max = 0;
};
hipError_t spmm_plan_build(damf_ctx *c, const Csr &g, int kmax, SpmmPlan *p);
void spmm_plan_free(SpmmPlan &p);
hipError_t csr_spmm(const Csr &g, const SpmmPlan &p, const float *X, float *Y, int64_t n, int k,
                    int ld, hipStream_t s);
// One PPR propagation round: Rnew = (1 - alpha) D^-1 A Rold, Z += alpha Rold,
// max |Rnew| into *maxbits (float bits, atomicMax).
hipError_t ppr_pull_round(const Csr &g, const SpmmPlan &p, const float *Rold, float *Rnew,
                          float *Z, int64_t n, int d, float alpha, unsigned *maxbits,
                          hipStream_t s);

// ---- rsvd.hip
hipError_t rsvd_init(damf_ctx *c);
hipError_t gemm_tall(const float *A, int64_t n, int l, int lda, const float *B,
                     int d, float *C, int ldc, hipStream_t s);

// ---- reorth.hip
hipError_t flush_projections(damf_ctx *c);
hipError_t reorthogonalize(damf_ctx *c, int *numeric_bad);

// ---- state.hip
hipError_t launch_query(damf_ctx *c, int which, int64_t q,
                        const int32_t *d_nodes, float *d_out);
// Undo log over a stretch of the chunk lists (S1 entries [s1_off, s1_off +
// n_s1) for U_b, S2 entries for V_b; a row may appear several times): save
// copies the rows into the log; restore removes the chain's signal additions
// from R (R -= U_b - log) and copies the rows back, entry by entry in list
// order, so a repeated row is corrected once.
// With r_delta false the restore leaves R alone.
hipError_t launch_undo_rows(damf_ctx *c, int s1_off, int n_s1, int s2_off, int n_s2, bool restore,
                            bool r_delta = true);
// save (restore = false) or put back the rows `rows` of R (one FP32 row of d
// per list entry, list order) at row `at` of undo_r; a no-op without PPR
constexpr int kRLogS1 = 2 * kMaxBatch + 1;
hipError_t launch_r_rows(damf_ctx *c, const int32_t *rows, int n, int at, bool restore);
// flip the sign of the batch's net entries (both sort orders), so that the
// graph edit applies the inverse change
hipError_t launch_negate_net(damf_ctx *c, int n_net);
// out[i] = <rows of which_a at u[i], rows of which_b at v[i]> (device lists)
hipError_t launch_score_pairs(damf_ctx *c, int which_a, int which_b, int64_t q, const int32_t *d_u,
                              const int32_t *d_v, float *d_out, bool both_ways);
// *d_bad = number of ids of d_nodes[0..q) outside [0, n) (cleared first)
hipError_t launch_count_bad_ids(const int32_t *d_nodes, int64_t q, int64_t n, int64_t *d_bad,
                                hipStream_t s);
// Fixed per-device scratch of damf_query_static: a 256-byte counter slot,
// then (host pointers only) the node ids and the output rows.
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
// Looks up this device's address of the scratch array (once per device;
// the device must be current).  Called by context creation.
hipError_t static_scratch_setup(int device);
// That address, or nullptr before static_scratch_setup(device) succeeded.
void *static_scratch_ptr(int device);

}  // namespace damf

#define DAMF_HIP(expr)                              \
  do {                                              \
    hipError_t _e = (expr);                         \
    if (_e != hipSuccess) return _e;                \
  } while (0)
