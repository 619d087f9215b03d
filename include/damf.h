/*
 * damf.h -- C ABI of libdamf, an MI355X (gfx950) implementation of DAMF,
 * Dynamic Adjacency Matrix Factorization (Deng, Yang, Li, Cai, Pu, Jiang,
 * "Accelerating Dynamic Network Embedding with Billions of Parameter Updates
 * to Milliseconds", KDD 2023, arXiv 2306.08967).
 *
 * The library keeps a rank-d factorisation A ~ U Sigma V^T of a graph's 0/1
 * adjacency matrix, its embeddings X = U Sigma^(1/2), Y = V Sigma^(1/2)
 * (Sec. 4.1) and the PPR-enhanced context embedding Z = PPR(X) (Sec. 4.4),
 * all resident in GPU memory, and updates them under batches of edge
 * insertions and deletions by space projection (Sec. 4.3, Theorem 2;
 * Algorithm 1 and Algorithm 2, edge branch) followed by dynamic PPR push.
 *
 * Conventions for every entry point:
 *   - Every call returns a damf_status; no C++ exception crosses the ABI.
 *     damf_last_error(ctx) describes the last failure of that context.
 *   - Pointer arguments are host pointers unless the call's `flags` include
 *     DAMF_DEVICE_PTRS, in which case they are device pointers (for example
 *     torch tensors' data_ptr()) readable/writable on the context's device.
 *     Input arrays are only read during the call; the caller owns them.
 *     Output arrays are caller-allocated with the sizes stated below.
 *   - Ids are 0-based int32 node ids in [0, n).
 *   - Calls on one context are serialised by the caller (one thread at a
 *     time); separate contexts are independent.
 *   - After a device error the context is poisoned: later calls return
 *     DAMF_E_STATE (DAMF_E_NUMERIC from an update undoes the batch and
 *     leaves the context usable, see damf_update).  An input error (DAMF_E_INVALID_ARG,
 *     DAMF_E_OUT_OF_RANGE) is detected before any state changes, so the
 *     context is unchanged.
 */
#ifndef DAMF_H
#define DAMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct damf_ctx damf_ctx; /* opaque; owns all device state */

typedef enum {
  DAMF_OK = 0,
  DAMF_E_INVALID_ARG = 1,  /* bad size, null pointer, bad config value      */
  DAMF_E_OUT_OF_RANGE = 2, /* node id outside [0, n) or op not +1/-1         */
  DAMF_E_OOM = 3,          /* device allocation failed                       */
  DAMF_E_DEVICE = 4,       /* a HIP call failed                              */
  DAMF_E_NUMERIC = 5,      /* non-finite value or failed factorisation       */
  DAMF_E_STATE = 6,        /* context poisoned by an earlier device error    */
  DAMF_E_BUSY = 7,         /* server admission cap reached (damf_serve.h)    */
  DAMF_E_TIMEOUT = 8       /* wait ended before the request completed        */
} damf_status;

typedef enum { DAMF_X = 0, DAMF_Y = 1, DAMF_Z = 2 } damf_which;

enum { DAMF_DEVICE_PTRS = 1, DAMF_SCORE_BOTH_WAYS = 2 };

/* Configuration.  Fill with damf_config_default() and override fields. */
typedef struct {
  int64_t n;             /* number of nodes, 1..2^30                          */
  int32_t d;             /* t-SVD rank = embedding width (Sec. 4.1); 1..128   */
  int32_t directed;      /* 0: an op on (u,v) edits A[u,v] and A[v,u]         */
  int32_t oversample;    /* randomized t-SVD oversampling p (default 10)      */
  int32_t power_iters;   /* randomized t-SVD power iterations q (default 2)   */
  uint64_t seed;         /* seed of the Rademacher sketch                     */
  double alpha;          /* PPR damping factor (Sec. 4.4); 1.0 disables Step 4 */
  double eps;            /* PPR error tolerance: max |R| <= eps after Step 4  */
  int32_t max_core_rank; /* r: chunk rank bound, min(|S1|,|S2|) <= r          */
  int32_t max_side;      /* r_max: max(|S1|,|S2|) <= r_max; d + r_max <= 192  */
  double tau;            /* residual Gram eigenvalue drop threshold           */
  int32_t auto_enhance;  /* 1: damf_update runs Step 4 before returning       */
  int32_t reorth_every;  /* > 0: damf_update re-orthogonalises after every
                            reorth_every-th batch that changed A; 0: never */
  double graph_slack;    /* CSR pool: rows reserve len + len/4 + 4 entries; the
                            pool holds max(reservations, slack * m) plus a
                            free quarter of the reservations; compacted when
                            less than an eighth is free                      */
  void *hip_stream;      /* hipStream_t to run on; NULL = a context stream    */
  int32_t precision;     /* 0: bases U_b, V_b in FP32.  1: the precision form:
                            each basis element stored as a BF16 pair
                            hi = bf16(x), lo = bf16(x - hi) in one 32-bit word
                            (about 16 significant bits); flush / re-
                            orthogonalisation rotate them with BF16 MFMA
                            (hi*hi + hi*lo + lo*hi, FP32 accumulation).  The
                            core, Grams, projections, re-orthogonalisation and
                            the eps test stay FP64; Z_b and the PPR residual R
                            stay FP32 (Z_b sums many small pushes).          */
  int32_t kernel_timing; /* 1: time every Step 2 core-SVD kernel launch with a
                            pair of HIP events (up to 256 chunks per batch) and
                            report the sum in damf_batch_info.ms_core_kernel;
                            0 (default): no per-launch events              */
  double jacobi_tol;     /* Step 2 core SVD (one-sided Jacobi): a column pair
                            is rotated while |a_i . a_j| > jacobi_tol
                            ||a_i|| ||a_j||.  0 (default) means 1e-9 for FP32
                            bases, which keeps the products at FP32 rounding,
                            and 1e-8 for the precision form, whose stored
                            bases carry about 16 significant bits.  Valid:
                            0, or 1e-14 .. 1e-6                            */
  double flush_cond;     /* lazy projection limit (Sec. 4.1 lazy update): after
                            a batch whose new P has a condition estimate
                            (LU pivot spread) above flush_cond, damf_update
                            flushes (as damf_flush) before Step 4, since the
                            FP32 rounding of the stored bases is amplified by
                            up to cond(P) in U = U_b P.  0 (default) means
                            1e3; a negative value never flushes; else >= 1.
                            A single chunk whose new P passes max(flush_cond,
                            1e3) is applied explicitly (see damf_update)   */
  int32_t graph_chunks;  /* 0 (default): Steps 1-3 are launched kernel by kernel.
                            1..64: a batch of at most graph_chunks chunks runs
                            its Steps 1-3 launches (four per chunk on two
                            streams) as one captured HIP graph, built on the
                            first batch of its shape (chunk count and which
                            chunks wait for their predecessor) and replayed
                            after; results are bit-identical.  Ignored while
                            kernel_timing = 1                               */
  int32_t pad0_;
} damf_config;

/* Per-batch statistics written by damf_update when `info` is non-NULL. */
typedef struct {
  int64_t ops;            /* ops submitted                                     */
  int64_t net_entries;    /* nonzero entries of the net change of A            */
  int64_t chunks;         /* chunks the net change was cut into                */
  int32_t max_core;       /* largest core dimension (d + rank) used            */
  int32_t dropped;        /* residual directions dropped by tau                */
  int64_t push_rounds;    /* Step 4 rounds                                     */
  int64_t pushes;         /* Step 4 node pushes                                */
  int64_t push_edges;     /* Step 4 edge traversals                            */
  double ms_prepare;      /* batch sort / net change / chunking                */
  double ms_chain;        /* Steps 1-3 over all chunks (with CSR edits)        */
  double ms_enhance;      /* Step 4                                            */
  double ms_chain_kernel; /* the Steps 1-3 kernel alone (HIP events)           */
  double chain_flops;     /* FP64 flops that kernel executed (counted model)   */
  double ms_push_kernel;  /* Step 4 push kernels, summed over rounds          */
  double push_bytes;      /* compulsory HBM bytes of those push kernels        */
  int64_t sweeps;         /* Jacobi sweeps over all chunks                     */
  double chain_phase_ms[8]; /* inside the Steps 1-3 kernel: 0 gather/project,
                               1 Jacobi sweeps, 2 core SVD (incl. 1), 3 basis
                               completion, 4 rotations/row corrections,
                               5 P <- P F, 6 LU solve + scatter, 7 Grams   */
  double ms_reorth;       /* re-orthogonalisation run by this batch (0: none)  */
  double ms_core_kernel;  /* Step 2 core-SVD kernel launches, summed (HIP events
                             around each launch; needs kernel_timing = 1)     */
  int64_t core_launches;  /* launches timed into ms_core_kernel                */
  double core_flops;      /* counted FP64 flops of all core-SVD launches: Jacobi
                             sweeps x N(N-1)/2 pairs x (2N for the dot + 6N f
                             for the rotation, f the share of steps in which
                             any pair rotated) + 2N^2 d (H) + 2N^2 k (K)      */
  double core_flops_model; /* the same launches priced by the textbook count of
                             one-sided Jacobi: 9 N^3 FP64 flops per sweep (the
                             dots, the column rotation and the accumulation of
                             the right vectors, which this kernel forms after
                             the sweeps as H = K^T E instead)              */
  double p_cond;          /* condition estimate of the projections after the
                             chunks (largest LU pivot spread; 1 after a flush) */
  int32_t flushed;        /* 1: this batch flushed P (flush_cond reached)      */
  int32_t explicit_chunks;/* chunks whose new projection was too ill-conditioned
                             and that were applied explicitly (damf_update)    */
  int64_t graph_launches; /* batches of the context so far whose Steps 1-3 ran
                             as a captured graph (graph_chunks)                */
  int32_t small_sv_columns;/* right singular vectors of the cores that were
                             re-orthogonalised because their singular value
                             was below 1e5 jacobi_tol sigma_1 (H = K^T E
                             Theta^-1 amplifies E's residual non-orthogonality
                             by sigma_1 / theta there)                        */
  int32_t pad1_;
} damf_batch_info;

/* Statistics of the initialisation (damf_init / damf_init_factors). */
typedef struct {
  double ms_graph;        /* CSR build of A and A^T                            */
  double ms_rsvd;         /* randomized t-SVD                                  */
  double ms_ppr;          /* initial PPR propagation                           */
  int64_t ppr_rounds;     /* propagation rounds (CSR SpMM passes)              */
  double ms_spmm_kernel;  /* propagation SpMM kernels, summed                  */
  double spmm_bytes;      /* compulsory HBM bytes of those SpMM kernels        */
  int64_t nnz;            /* edges of A                                        */
  int64_t qr_fallbacks;   /* tall QRs of the t-SVD that took the Householder
                             TSQR because the sketch's Gram was not clearly
                             positive definite (rank below d + p, or cond above
                             about 1e5); the others ran as CholeskyQR2         */
} damf_init_info;

/* Defaults: d=128, directed, p=10, q=2, alpha=0.15, eps=1e-5, r=64,
 * r_max=64, tau=1e-6, auto_enhance=1, slack=1.25. */
void damf_config_default(damf_config *cfg);

/* Create a context from an initial edge list (Appendix A, Algorithm 3):
 * builds the graph, takes the randomized rank-d t-SVD of A (sketch
 * Omega[i,j] = +/-1 from SplitMix64, Q = qr(A Omega), q rounds of
 * Q = qr(A^T Q), Q = qr(A Q), then B^T = A^T Q = Q2 R2 and svd(R2^T)), sets
 * the projections to the identity and propagates PPR until max |R| <= eps / 2
 * (headroom for the first updates' pushes).
 * src/dst: m edges (duplicates collapse; self-loops are entries).
 * Errors: DAMF_E_INVALID_ARG (n outside 1..2^30, d out of range, m < 0, null arrays with
 * m > 0), DAMF_E_OUT_OF_RANGE (id outside [0,n)), DAMF_E_OOM, DAMF_E_NUMERIC
 * (the factorisation or the PPR residual came out NaN or infinite). */
damf_status damf_init(const damf_config *cfg, int64_t m, const int32_t *src,
                      const int32_t *dst, int32_t flags, damf_ctx **out);

/* As damf_init, but takes the rank-d factorisation from the caller instead
 * of computing it: U, V are n x d row-major float64, S has d values sorted
 * descending (host pointers; flags only govern src/dst). */
damf_status damf_init_factors(const damf_config *cfg, int64_t m,
                              const int32_t *src, const int32_t *dst,
                              const double *U, const double *S,
                              const double *V, int32_t flags, damf_ctx **out);

/* Apply one batch of k edits (Algorithm 2, edge branch, for all events of
 * the batch).  op[i] = +1 inserts (src[i], dst[i]), -1 deletes it; ops apply
 * in order with set semantics (inserting a present edge or deleting an
 * absent one changes nothing).  The net change of A is cut into chunks of
 * rank <= r; each chunk is one Steps 1-3 update (Theorem 2 with B, C of k
 * columns).  Then Step 4 runs if auto_enhance.  0 <= k <= 8192; k == 0 is a
 * no-op.  The lazy update keeps U = U_b P and solves with the new P, so the
 * FP32 rounding of the rows it writes is amplified by up to cond(P).  When a
 * chunk's new P has a condition estimate (LU pivot spread) above
 * max(flush_cond, 1e3) (above 1e10 when flushing is off), such as when a kept
 * direction has almost no component in span(U) (an edge between two nodes
 * without basis weight while a zero singular value is kept), the batch's
 * chunks are undone and re-run one by one, and that chunk is applied
 * explicitly (every row rotated by P F, then its row corrections with P = I);
 * info->explicit_chunks counts them.  Errors: DAMF_E_INVALID_ARG,
 * DAMF_E_OUT_OF_RANGE (state unchanged), DAMF_E_NUMERIC (non-finite values
 * in a chunk's core, e.g. from singular values near the top of the double
 * range: the batch is undone, bases, P, Sigma, R and the graph are bit for
 * bit as before the call and the context stays usable; only when it comes
 * up during the one-by-one re-run of explicit chunks is the context
 * poisoned), DAMF_E_DEVICE. */
damf_status damf_update(damf_ctx *ctx, int64_t k, const int32_t *src,
                        const int32_t *dst, const int8_t *op, int32_t flags,
                        damf_batch_info *info);

/* Per-request results of damf_update_requests. */
typedef struct {
  int64_t net_entries;    /* nonzero entries of the request's net change       */
  int64_t chunks;         /* chunks the request was cut into                   */
} damf_request_stats;

/* Several requests in one update step, with the result of applying them one
 * after another by damf_update without Step 4 in between (Algorithm 2 applied
 * to each request's events in order).  Request i is ops [sum_{j<i} req_ops[j],
 * sum_{j<=i} req_ops[j]) of src/dst/op.  Each request's net change is taken
 * against the graph the earlier requests leave, and its chunks never contain
 * another request's edits, so U, Sigma, V after the step are those of the
 * one-by-one sequence; the graph is edited once with the step's net change and
 * Step 4 runs once (auto_enhance).  nreq in 1..256, sum of req_ops <= 8192;
 * req_ops is a host array.  per_request (nullable, host, nreq entries)
 * receives each request's net entries and chunks.  Errors as damf_update. */
damf_status damf_update_requests(damf_ctx *ctx, int32_t nreq, const int64_t *req_ops,
                                 const int32_t *src, const int32_t *dst,
                                 const int8_t *op, int32_t flags,
                                 damf_batch_info *info,
                                 damf_request_stats *per_request);

/* Node change (Sec. 4.2, Theorem 1; Algorithm 2, node branch).  Node `node`,
 * which must have no edges yet (a free slot of the fixed node range), joins
 * with in-edges (v, node) for v in in_nbrs and out-edges (node, w) for w in
 * out_nbrs.  The update runs Theorem 1's two steps: the column step
 * A' = [A, B1] with B1 the in-edges (a self-loop excluded), then the row step
 * with B2 the out-edges and the self-loop (node, node) when either list
 * names `node`.  Each step is one rank-1 space projection ((d+1) x (d+1)
 * core); a step with more than max_side (r_max) entries is applied as
 * consecutive rank-1 pieces of at most r_max entries, the first Theorem 1's
 * step and the later ones edge updates of the existing column (row).  Then
 * Step 4 runs if auto_enhance.  Undirected graphs: the neighbours go in
 * in_nbrs and k_out must be 0 (the row step takes the same list).  Host
 * arrays; duplicates collapse; k_in + k_out <= 8192.  Errors:
 * DAMF_E_OUT_OF_RANGE (an id outside [0, n)), DAMF_E_INVALID_ARG (the node
 * has edges, bad sizes or lists), both with the state unchanged; otherwise as
 * damf_update.  info (nullable) as damf_update's. */
damf_status damf_add_node(damf_ctx *ctx, int32_t node, int64_t k_in, const int32_t *in_nbrs,
                          int64_t k_out, const int32_t *out_nbrs, damf_batch_info *info);

/* Chunk rank r (max_core_rank) for the batches that follow: 1 <= r <= max_side
 * and d + r <= 192, else DAMF_E_INVALID_ARG.  The chunking of a batch depends
 * on r, so the factorisation after a batch does too (the serving tuner
 * changes it; a replay sets the rank each request reports). */
damf_status damf_set_chunk_rank(damf_ctx *ctx, int32_t r);

/* Step 4 (Sec. 4.4): push PPR residuals until max |R| <= eps. */
damf_status damf_enhance(damf_ctx *ctx);

/* Flush of the lazy projections (Sec. 4.1, the lazy update equation):
 * U_b <- U_b P_U, Z_b <- Z_b P_U, R <- R P_U, V_b <- V_b P_V, P_U = P_V = I.
 * X, Y, Z and the PPR invariant are unchanged up to FP32 rounding of the
 * rotated bases.  Cost: one n x d by d x d MFMA product per basis.
 * Errors: DAMF_E_STATE (poisoned), DAMF_E_DEVICE (poisons the context). */
damf_status damf_flush(damf_ctx *ctx);

/* FP64 re-orthogonalisation of the factorisation, keeping U Sigma V^T
 * (Sec. 4.1: U and V are the orthonormal factors of the t-SVD, which FP32
 * rounding over many updates erodes).  With U = U_b P_U, V = V_b P_V:
 * U^T U = R_U^T R_U and V^T V = R_V^T R_V (FP64 Grams, Cholesky), then
 * R_U Sigma R_V^T = Ut S Vt^T (FP64 Jacobi SVD), U <- U R_U^-1 Ut,
 * V <- V R_V^-1 Vt, Sigma <- S, with Z_b and R rotated like U_b and the
 * projections reset to I.  Directions with S = 0 (rank(A) < d) are completed
 * to orthonormal columns.  Max |R| may exceed eps afterwards: damf_update
 * re-orthogonalises before its Step 4; a direct caller runs damf_enhance.
 * Errors: DAMF_E_NUMERIC when a Cholesky pivot of U^T U or V^T V is below
 * 0.25 (a basis far from orthonormal, not rounding drift): the state is left
 * unchanged and the context stays usable.  DAMF_E_DEVICE poisons it. */
damf_status damf_reorthogonalize(damf_ctx *ctx);

/* Rows of X, Y or Z for q nodes (nodes == NULL: all n rows, q must be n):
 * out is q x d row-major float32.  Row of X = U_b[u] P_U Sigma^(1/2)
 * (Sec. 4.6, O(d^2) per query).  A Z query after batches applied without
 * Step 4 (auto_enhance = 0) runs damf_enhance first, so Z is within eps of
 * PPR(X) for the current state. */
damf_status damf_query(damf_ctx *ctx, damf_which which, int64_t q,
                       const int32_t *nodes, float *out, int32_t flags);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc): damf_query without any
 * allocation.  Same arguments, layout and results as damf_query.  Its
 * temporaries live in a fixed 4 MiB array that the library holds on each
 * device for the life of the process: a 256-byte counter slot, then, with
 * host pointers only, the q node ids (rounded up to 256 bytes) and the q x d
 * output rows.  Limits: with host pointers 256 + round256(4 q) + 4 q d must
 * not exceed 4 MiB (q <= 8,128 rows at d = 128, nodes given), else
 * DAMF_E_INVALID_ARG; with DAMF_DEVICE_PTRS only the counter is used and q is
 * not limited.  A Z query while Step 4 is pending (auto_enhance = 0) returns
 * DAMF_E_INVALID_ARG (call damf_enhance first, which may allocate).  Every
 * call on one device shares that array: calls that overlap on one device
 * (contexts on different streams or threads) race and must be serialised by
 * the caller.  Errors otherwise as damf_query. */
damf_status damf_query_static(damf_ctx *ctx, damf_which which, int64_t q,
                              const int32_t *nodes, float *out, int32_t flags);

/* Link scores (Sec. 5.2 link prediction and graph reconstruction; the
 * appendix on link prediction): out[i] = <A[u[i]], B[v[i]]> where A and B
 * are the rows of X, Y or Z chosen by which_a and which_b (the paper scores a
 * pair (u, v) by u's context vector, Z, against v's content vector, Y).
 * With DAMF_SCORE_BOTH_WAYS in flags, out[i] = max(<A[u], B[v]>,
 * <A[v], B[u]>), the paper's score for undirected graphs.  u, v: q int32 ids;
 * out: q float32 (host, or device with DAMF_DEVICE_PTRS).  Rows are formed
 * as in damf_query (FP64 accumulation); a Z side runs a pending Step 4
 * first.  Errors: DAMF_E_OUT_OF_RANGE (an id outside [0, n)),
 * DAMF_E_INVALID_ARG, DAMF_E_DEVICE. */
damf_status damf_score_pairs(damf_ctx *ctx, damf_which which_a, damf_which which_b, int64_t q,
                             const int32_t *u, const int32_t *v, float *out, int32_t flags);

/* The d singular values, descending (host float64 array of d). */
damf_status damf_singular_values(damf_ctx *ctx, double *out);

/* Canonical CSR of A (transpose = 0) or A^T (transpose = 1): indptr has n+1
 * int64 entries, indices m int32 entries ascending within each row.  Call
 * with indices == NULL to get m in *m_out only.  Host pointers. */
damf_status damf_export_csr(damf_ctx *ctx, int32_t transpose, int64_t *indptr,
                            int32_t *indices, int64_t *m_out);

/* Internal state for tests, as host float64: Ub, Vb, Zb, R are n x d
 * row-major (any may be NULL), PU, PV are d x d row-major. */
damf_status damf_export_state(damf_ctx *ctx, double *Ub, double *Vb,
                              double *PU, double *PV, double *Zb, double *R);

/* Statistics of the context's initialisation. */
damf_status damf_get_init_info(damf_ctx *ctx, damf_init_info *info);

/* Current max |R| entry (float64); <= eps after Step 4. */
damf_status damf_residual_max(damf_ctx *ctx, double *out);

/* Wait for all work of the context. */
damf_status damf_sync(damf_ctx *ctx);

/* Checkpoint (not part of the paper's method; it lets a long-running
 * context stop and resume).  damf_save writes the whole state to `path`: the
 * graph as the canonical out-CSR, P_U, P_V, Sigma, U_b, V_b (as stored, FP32
 * or BF16 pairs) and, with PPR, Z_b and R, plus the re-orthogonalisation and
 * push counters; host byte order, streamed through a 64 MiB pinned buffer.
 * damf_load creates a context from such a file: cfg supplies the run-time
 * options (stream, eps, chunk ranks, ...) and must agree with the file on n,
 * d, directed, precision and alpha (else DAMF_E_INVALID_ARG).  The loaded
 * context rebuilds its CSR pools compactly; every later result equals the
 * saved context's bit for bit, except where float atomics of Step 4 order
 * differently.  Errors: DAMF_E_INVALID_ARG (path, mismatch, short or corrupt
 * file), DAMF_E_STATE (save of a poisoned context), DAMF_E_OOM, DAMF_E_DEVICE. */
damf_status damf_save(damf_ctx *ctx, const char *path);
damf_status damf_load(const char *path, const damf_config *cfg, damf_ctx **out);

void damf_destroy(damf_ctx *ctx);

const char *damf_last_error(const damf_ctx *ctx);
const char *damf_status_string(damf_status s);

#ifdef __cplusplus
}
#endif
#endif /* DAMF_H */
