// state.hip -- small kernels on the embedding state: node queries
// (Sec. 4.6: X[u] = X_b[u] P_X at O(d^2) per node) and the range check of
// device node lists.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"
#include "damf_internal.h"

namespace damf {

// *bad = 0; a kernel rather than a memset, so the sequence stays valid inside
// a captured HIP graph.
__global__ void clear_counter_kernel(int64_t *bad) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *bad = 0;
}

// *bad += number of ids outside [0, n).  Reads the list only.
__global__ __launch_bounds__(256) void count_bad_ids_kernel(const int32_t *nodes, int64_t q,
                                                            int64_t n, int64_t *bad) {
  int64_t cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = nodes[i];
    cnt += (v < 0 || (int64_t)v >= n) ? 1 : 0;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if ((threadIdx.x & 63) == 0 && cnt)
    atomicAdd((unsigned long long *)bad, (unsigned long long)cnt);
}

// out[i][c] = sum_k M_b[node_i][k] P[k][c] * sqrt(sigma_c), FP64 accumulate.
// One wave per queried row, rows taken in a grid-stride loop; lanes own
// columns c = lane + 64 j.
__global__ __launch_bounds__(256) void query_kernel(const float *Mb, const double *P,
                                                    const double *sigma, int d, int64_t q,
                                                    const int32_t *nodes, float *out,
                                                    bool split) {
  __shared__ double row[4][kMaxD];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < q; i += (int64_t)gridDim.x * 4) {
    const int64_t node = nodes ? nodes[i] : i;
    for (int k = lane; k < d; k += 64) row[w][k] = (double)basis_ld(Mb, node * d + k, split);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int c = lane; c < d; c += 64) {
      double acc = 0.0;
      for (int k = 0; k < d; ++k) acc = fma(row[w][k], P[k * d + c], acc);
      out[i * d + c] = (float)(acc * sqrt(sigma[c]));
    }
    // the row buffer is rewritten by the next pass
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
}

// Undo log of one basis over a row list that may repeat rows.  Save (one
// wave per entry, any order): log[i] = M[rows[i]], the stored words.
__global__ __launch_bounds__(256) void undo_save_kernel(const int32_t *rows, int nrows,
                                                        const float *M, float *log, int d) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < nrows;
       i += (int64_t)gridDim.x * 4) {
    const int64_t row = rows[i];
    for (int c = lane; c < d; c += 64) log[i * d + c] = M[row * d + c];
  }
}

// Restore, by one wave walking the list in order: with R,
// R[row] -= M[row] - log[i] (what the chain's scatters added to R along with
// U_b), then M[row] = log[i].  Every entry of a row logged the same pre-chain
// words, so after its first entry the difference is zero: a repeated row is
// corrected once.  A lane always handles the same columns, so the entries of
// one row are ordered by program order.
__global__ __launch_bounds__(64) void undo_restore_kernel(const int32_t *rows, int nrows, float *M,
                                                          const float *log, float *R, int d,
                                                          bool split) {
  const int lane = threadIdx.x;
  for (int i = 0; i < nrows; ++i) {
    const int64_t row = rows[i];
    for (int c = lane; c < d; c += 64) {
      const int64_t at = row * d + c, li = (int64_t)i * d + c;
      if (R) R[at] -= basis_ld(M, at, split) - basis_ld(log, li, split);
      M[at] = log[li];
    }
  }
}

hipError_t launch_undo_rows(damf_ctx *c, int s1_off, int n_s1, int s2_off, int n_s2, bool restore,
                            bool r_delta) {
  const Workspace &w = c->ws;
  hipStream_t s = c->stream;
  const int32_t *l1 = w.chunk_s1 + s1_off, *l2 = w.chunk_s2 + s2_off;
  if (!restore) {
    if (n_s1 > 0) {
      const Grid g = geom_rows(n_s1);
      undo_save_kernel<<<g.blocks, g.threads, 0, s>>>(l1, n_s1, c->Ub, w.undo_u, c->d);
    }
    if (n_s2 > 0) {
      const Grid g = geom_rows(n_s2);
      undo_save_kernel<<<g.blocks, g.threads, 0, s>>>(l2, n_s2, c->Vb, w.undo_v, c->d);
    }
  } else {
    if (n_s1 > 0)
      undo_restore_kernel<<<1, 64, 0, s>>>(l1, n_s1, c->Ub, w.undo_u,
                                           (c->ppr_on && r_delta) ? c->R : nullptr, c->d, c->split);
    if (n_s2 > 0)
      undo_restore_kernel<<<1, 64, 0, s>>>(l2, n_s2, c->Vb, w.undo_v, nullptr, c->d, c->split);
  }
  return hipGetLastError();
}

// Rows of R as they were before the structural fix-up or the chain changed
// them, saved into undo_r or put back from it.  A list may repeat a row
// (S1 over several chunks); its copies all hold the same saved words, so the
// restore can write them in parallel.
__global__ __launch_bounds__(256) void r_rows_restore_kernel(const int32_t *rows, int nrows, float *R,
                                                             const float *log, int d) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < nrows;
       i += (int64_t)gridDim.x * 4) {
    const int64_t row = rows[i];
    for (int c = lane; c < d; c += 64) R[row * d + c] = log[i * d + c];
  }
}

hipError_t launch_r_rows(damf_ctx *c, const int32_t *rows, int n, int at, bool restore) {
  if (n <= 0 || !c->ppr_on) return hipSuccess;
  const Grid g = geom_rows(n);
  float *log = c->ws.undo_r + (size_t)at * c->d;
  if (restore)
    r_rows_restore_kernel<<<g.blocks, g.threads, 0, c->stream>>>(rows, n, c->R, log, c->d);
  else
    undo_save_kernel<<<g.blocks, g.threads, 0, c->stream>>>(rows, n, c->R, log, c->d);
  return hipGetLastError();
}

// The inverse of a net change: every insert becomes a delete and back, and
// pad (the inserts before an entry in its sorted list) becomes the deletes
// before it, i - pad.
__global__ void negate_net_kernel(NetEntry *a, NetEntry *b, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    a[i].delta = -a[i].delta;
    a[i].pad = i - a[i].pad;
    b[i].delta = -b[i].delta;
    b[i].pad = i - b[i].pad;
  }
}

hipError_t launch_negate_net(damf_ctx *c, int n_net) {
  if (n_net <= 0) return hipSuccess;
  const Grid g = geom_elementwise(n_net);
  negate_net_kernel<<<g.blocks, g.threads, 0, c->stream>>>(c->ws.net, c->ws.net_t, n_net);
  return hipGetLastError();
}

// score[i] = <A[u_i], B[v_i]> with A, B rows of X, Y or Z (Sec. 5.2: the
// inner product of u's context vector and v's content vector), and with
// both_ways max(<A[u], B[v]>, <A[v], B[u]>) (undirected graphs).  A row of A
// is Ma_b[u] Pa Sigma^(1/2) as in the query; one wave per pair, FP64
// accumulation, pairs in a grid-stride loop.
__global__ __launch_bounds__(256) void score_pairs_kernel(const float *Ma, const double *Pa, bool split_a,
                                                          const float *Mb, const double *Pb, bool split_b,
                                                          const double *sigma, int d, int64_t q,
                                                          const int32_t *u, const int32_t *v,
                                                          float *out, bool both_ways) {
  __shared__ double ra[4][kMaxD], rb[4][kMaxD];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < q; i += (int64_t)gridDim.x * 4) {
    double best = -INFINITY;
    for (int dir = 0; dir < (both_ways ? 2 : 1); ++dir) {
      const int64_t a = dir ? v[i] : u[i], b = dir ? u[i] : v[i];
      for (int k = lane; k < d; k += 64) {
        ra[w][k] = (double)basis_ld(Ma, a * d + k, split_a);
        rb[w][k] = (double)basis_ld(Mb, b * d + k, split_b);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      double dot = 0.0;
      for (int c = lane; c < d; c += 64) {
        double xa = 0.0, xb = 0.0;
        for (int k = 0; k < d; ++k) {
          xa = fma(ra[w][k], Pa[k * d + c], xa);
          xb = fma(rb[w][k], Pb[k * d + c], xb);
        }
        dot = fma(xa * sigma[c], xb, dot);  // sqrt(sigma_c)^2
      }
      dot = wave_sum(dot);
      best = fmax(best, dot);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    if (lane == 0) out[i] = (float)best;
  }
}

hipError_t launch_score_pairs(damf_ctx *c, int which_a, int which_b, int64_t q, const int32_t *d_u,
                              const int32_t *d_v, float *d_out, bool both_ways) {
  if (q <= 0) return hipSuccess;
  auto mat = [&](int which, const float **M, const double **P, bool *split) {
    *M = (which == DAMF_X) ? c->Ub : (which == DAMF_Y) ? c->Vb : c->Zb;
    *P = (which == DAMF_Y) ? c->P + (size_t)c->d * c->d : c->P;
    *split = c->split && which != DAMF_Z;
  };
  const float *Ma, *Mb;
  const double *Pa, *Pb;
  bool sa, sb;
  mat(which_a, &Ma, &Pa, &sa);
  mat(which_b, &Mb, &Pb, &sb);
  const Grid g = geom_query(q);
  score_pairs_kernel<<<g.blocks, g.threads, 0, c->stream>>>(Ma, Pa, sa, Mb, Pb, sb, c->sigma, c->d, q,
                                                            d_u, d_v, d_out, both_ways);
  return hipGetLastError();
}

hipError_t launch_count_bad_ids(const int32_t *d_nodes, int64_t q, int64_t n, int64_t *d_bad,
                                hipStream_t s) {
  clear_counter_kernel<<<1, 64, 0, s>>>(d_bad);
  if (q > 0) {
    const Grid g = geom_check_ids(q);
    count_bad_ids_kernel<<<g.blocks, g.threads, 0, s>>>(d_nodes, q, n, d_bad);
  }
  return hipGetLastError();
}

hipError_t launch_query(damf_ctx *c, int which, int64_t q, const int32_t *d_nodes,
                        float *d_out) {
  const float *Mb = (which == DAMF_X) ? c->Ub : (which == DAMF_Y) ? c->Vb : c->Zb;
  const double *P = (which == DAMF_Y) ? c->P + (size_t)c->d * c->d : c->P;
  if (q <= 0) return hipSuccess;
  const Grid g = geom_query(q);
  query_kernel<<<g.blocks, g.threads, 0, c->stream>>>(Mb, P, c->sigma, c->d, q, d_nodes, d_out,
                                                      c->split && which != DAMF_Z);
  return hipGetLastError();
}

// ---- fixed scratch of damf_query_static, for callers that cannot allocate.
// Each device holds its own copy of the array until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns on
// that device (static_scratch_setup, called once per device by context
// creation with the device current).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void *static_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace damf
