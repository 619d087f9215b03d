// ppr.hip -- Step 4, dynamic embedding enhancement by Personalized PageRank
// (Sec. 4.4; Algorithm 2; Algorithm 3 for the initial propagation).
//
// PPR(X) = sum_i alpha (1 - alpha)^i (D^-1 A)^i X with D the out-degree.  The
// enhanced embedding is kept in base coordinates, Z_b ~ PPR(U_b), together
// with a residual R such that PPR(U_b) = Z_b + Pi R, Pi = alpha (I - (1 -
// alpha) P)^-1, P = D^-1 A (rows of dangling nodes are zero).
//
//   initial propagation: R = U_b, Z_b = 0, then synchronous rounds
//       Z_b += alpha R,  R <- (1 - alpha) P R        (CSR SpMM over out-rows)
//   signal change dU_b at rows S:  R[S] += dU_b       (added by the chain kernel)
//   structure change of row u:     R[u] += (1-alpha)/alpha (P'Z_b - P Z_b)[u]
//   push of node v:  Z_b[v] += alpha R[v];  R[u] += (1-alpha) R[v] / deg(u) for
//       every in-neighbour u of v;  R[v] = 0
//
// Every step keeps the invariant exactly (Pi = alpha I + (1 - alpha) Pi P), and
// since Pi >= 0 has row sums <= 1, max |R| <= eps gives |Z_b - PPR(U_b)| <= eps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>

#include "common.h"
#include "damf_internal.h"

namespace damf {

namespace {

constexpr int kRowsPerBlock = 4;  // one wave per row
constexpr int kPushCounters = 8;  // per round: [1] frontier, [2] next candidates,
                                  // [3] edges, [4] heavy nodes, [5] heavy segments
constexpr int kPushRing = 4;      // rounds in flight share a ring of counter sets
constexpr int kPushGroup = 4;     // rounds queued per host check
constexpr int kMaxPushRounds = 65536;

// Structural fix-up for each changed out-row u (before the CSR edit; before
// or after the chain kernel, which adds the same change to U_b and R, so
// alpha (R - X) is unchanged; never while a push runs):
//   P Z_b[u] from the invariant, (alpha (R - X) + Z_b)[u] / (1 - alpha)
//   P'Z_b[u] = (deg_old P Z_b[u] + sum_added Z_b[v] - sum_removed Z_b[v]) / deg_new
__global__ __launch_bounds__(256) void fixup_kernel(Csr g, const NetEntry *net,
                                                    const int32_t *rows, const int32_t *rowpos,
                                                    int nrows, const float *X, const float *Z,
                                                    float *R, int d, float alpha, bool split) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
  if (j >= nrows) return;
  const int32_t u = rows[j];
  const int e0 = rowpos[j], e1 = rowpos[j + 1];
  const int32_t deg_old = g.len[u];
  int32_t ddeg = 0;
  for (int e = e0; e < e1; ++e) ddeg += net[e].delta;
  const int32_t deg_new = deg_old + ddeg;
  const float k = (1.f - alpha) / alpha;
  for (int c = lane; c < d; c += 64) {
    const int64_t i = (int64_t)u * d + c;
    const float pz = (alpha * (R[i] - basis_ld(X, i, split)) + Z[i]) / (1.f - alpha);
    float s = (float)deg_old * pz;
    for (int e = e0; e < e1; ++e) {
      const NetEntry en = net[e];
      const float z = Z[(int64_t)en.col * d + c];
      s += (en.delta > 0) ? z : -z;
    }
    const float pz_new = (deg_new > 0) ? s / (float)deg_new : 0.f;
    R[i] += k * (pz_new - pz);
  }
}

// Frontier selection: candidates with max |R| > eps (compared in FP64).
// Appends are compacted per block (one global atomic per block).  With
// dedup_round >= 0 a candidate listed twice is taken once (stamp exchange):
// a node pushed twice in one round would race on its Z_b row.  The candidate
// count comes from the previous round's counters on the device (or from the
// host for the first round), so rounds queue without host round trips.
// Block 0 also clears the next round's counters and logs the previous
// round's frontier and edge counts.
__global__ __launch_bounds__(256) void select_kernel(const int32_t *cand, const int64_t *ncand_dev,
                                                     int64_t ncand_host, const float *R, int d,
                                                     double eps, int32_t *stamp,
                                                     int32_t dedup_round, int32_t *frontier,
                                                     int64_t *cnt_r, int64_t *cnt_next,
                                                     const int64_t *cnt_prev, int64_t *log_prev) {
  __shared__ int s_cnt;
  __shared__ int32_t s_list[kRowsPerBlock];
  __shared__ unsigned long long s_base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (blockIdx.x == 0 && threadIdx.x < kPushCounters) {
    cnt_next[threadIdx.x] = 0;
    if (cnt_prev && threadIdx.x == 0) {
      log_prev[0] = cnt_prev[1];
      log_prev[1] = cnt_prev[3];
    }
  }
  const int64_t ncand = ncand_dev ? *ncand_dev : ncand_host;
  for (int64_t base = (int64_t)blockIdx.x * kRowsPerBlock; base < ncand;
       base += (int64_t)gridDim.x * kRowsPerBlock) {
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int64_t j = base + w;
    bool take = j < ncand;
    int32_t v = 0;
    if (take) {
      v = cand ? cand[j] : (int32_t)j;
      if (dedup_round >= 0) {
        int first = 0;
        if (lane == 0) first = atomicExch(&stamp[v], dedup_round) != dedup_round;
        take = __shfl(first, 0, 64) != 0;
      }
    }
    if (take) {
      float m = 0.f;
      for (int c = lane; c < d; c += 64) m = fmaxf(m, fabsf(R[(int64_t)v * d + c]));
      m = wave_max(m);
      if (lane == 0 && (double)m > eps) s_list[atomicAdd(&s_cnt, 1)] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt > 0)
      s_base = atomicAdd((unsigned long long *)&cnt_r[1], (unsigned long long)s_cnt);
    __syncthreads();
    if (threadIdx.x < s_cnt) frontier[s_base + threadIdx.x] = s_list[threadIdx.x];
    __syncthreads();
  }
}

constexpr int kCandBuf = 1024;  // per-block LDS list of new candidates

// Spreads (1 - alpha) r / deg(u) into R[u] for the in-neighbours u in
// row[0 .. cnt) of a pushed node (cnt <= 64, one neighbour per lane for the
// first-touch stamp).  New candidates go to the block's LDS list (overflow
// straight to next_cand).
__device__ __forceinline__ void spread64(const int32_t *row, int cnt, const int32_t *outdeg,
                                         float *R, int d, float alpha, float r0, float r1,
                                         int32_t round, int32_t *stamp, int32_t *s_list,
                                         int *s_cnt, int32_t *next_cand, int64_t *counters) {
  const int lane = threadIdx.x & 63;
  const bool c0 = lane < d, c1 = lane + 64 < d;
  const int32_t myu = (lane < cnt) ? row[lane] : -1;
  // the 64 scale factors load in parallel, one per lane
  const float mysc = (myu >= 0) ? (1.f - alpha) / (float)outdeg[myu] : 0.f;
  bool fresh = false;
  if (myu >= 0) fresh = atomicExch(&stamp[myu], round) != round;
  const unsigned long long fm = __ballot(fresh);
  if (fm) {
    int base = 0;
    if (lane == 0) base = atomicAdd(s_cnt, __popcll(fm));
    base = __shfl(base, 0, 64);
    if (fresh) {
      const int at = base + __popcll(fm & ((1ull << lane) - 1ull));
      if (at < kCandBuf) {
        s_list[at] = myu;
      } else {
        const unsigned long long g = atomicAdd((unsigned long long *)&counters[2], 1ull);
        next_cand[g] = myu;
      }
    }
  }
  for (int q = 0; q < cnt; ++q) {  // q is wave-uniform: lane reads, no LDS
    const int32_t u = __builtin_amdgcn_readlane(myu, q);
    const float sc = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mysc), q));
    if (c0) atomicAdd(&R[(int64_t)u * d + lane], sc * r0);
    if (c1) atomicAdd(&R[(int64_t)u * d + lane + 64], sc * r1);
  }
}

__device__ __forceinline__ void flush_candidates(const int32_t *s_list, int s_cnt,
                                                 unsigned long long s_edges,
                                                 int32_t *next_cand, int64_t *counters,
                                                 unsigned long long *s_base) {
  const int cnt = min(s_cnt, kCandBuf);
  if (threadIdx.x == 0) {
    *s_base = cnt ? atomicAdd((unsigned long long *)&counters[2], (unsigned long long)cnt) : 0;
    if (s_edges) atomicAdd((unsigned long long *)&counters[3], s_edges);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < cnt; i += 256) next_cand[*s_base + i] = s_list[i];
}

// Push every frontier node: take R[v] atomically, Z_b[v] += alpha R[v], and
// spread (1 - alpha) R[v] / deg(u) to each in-neighbour u (in-CSR row v).
// A node with more than kHeavy in-neighbours is not spread here: its taken
// residual goes to hbuf and its row to segments of kSegEdges neighbours that
// spread_heavy_kernel spreads with one wave each.  Counters: [1] frontier,
// [2] next candidates, [3] edges, [4] heavy nodes, [5] heavy segments.
constexpr int kHeavy = 64;
constexpr int kSegEdges = 64;
__global__ __launch_bounds__(256) void push_kernel(Csr gin, const int32_t *outdeg,
                                                   const int32_t *frontier, float *R,
                                                   float *Z, int d, float alpha, int32_t round,
                                                   int32_t *stamp, int32_t *next_cand,
                                                   int64_t *counters, float *hbuf,
                                                   int32_t *hnode, int2 *hseg) {
  __shared__ int32_t s_list[kCandBuf];
  __shared__ int s_cnt;
  __shared__ unsigned long long s_edges, s_base;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) {
    s_cnt = 0;
    s_edges = 0;
  }
  __syncthreads();
  const int64_t nf = counters[1];
  for (int64_t j = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6); j < nf;
       j += (int64_t)gridDim.x * kRowsPerBlock) {
    const int32_t v = frontier[j];
    const bool c0 = lane < d, c1 = lane + 64 < d;
    float r0 = 0.f, r1 = 0.f;
    if (c0) {
      const int64_t i = (int64_t)v * d + lane;
      r0 = atomicExch(&R[i], 0.f);
      Z[i] += alpha * r0;
    }
    if (c1) {
      const int64_t i = (int64_t)v * d + lane + 64;
      r1 = atomicExch(&R[i], 0.f);
      Z[i] += alpha * r1;
    }
    const int32_t L = gin.len[v];
    const int32_t *row = gin.col + gin.start[v];
    if (L > kHeavy) {
      int h = 0, sg = 0;
      const int ns = (L + kSegEdges - 1) / kSegEdges;
      if (lane == 0) {
        h = (int)atomicAdd((unsigned long long *)&counters[4], 1ull);
        sg = (int)atomicAdd((unsigned long long *)&counters[5], (unsigned long long)ns);
      }
      h = __shfl(h, 0, 64);
      sg = __shfl(sg, 0, 64);
      if (c0) hbuf[(int64_t)h * d + lane] = r0;
      if (c1) hbuf[(int64_t)h * d + lane + 64] = r1;
      if (lane == 0) hnode[h] = v;
      for (int q = lane; q < ns; q += 64) hseg[sg + q] = make_int2(h, q);
    } else {
      for (int32_t e0 = 0; e0 < L; e0 += 64)
        spread64(row + e0, min(64, L - e0), outdeg, R, d, alpha, r0, r1, round, stamp, s_list,
                 &s_cnt, next_cand, counters);
      if (lane == 0) atomicAdd(&s_edges, (unsigned long long)L);
    }
  }
  __syncthreads();
  flush_candidates(s_list, s_cnt, s_edges, next_cand, counters, &s_base);
}

// One wave per segment of a heavy node's in-row (grid-stride over the
// segments the push kernel listed; the count is read on the device).
__global__ __launch_bounds__(256) void spread_heavy_kernel(Csr gin, const int32_t *outdeg,
                                                           float *R, int d, float alpha,
                                                           int32_t round, int32_t *stamp,
                                                           int32_t *next_cand, int64_t *counters,
                                                           const float *hbuf,
                                                           const int32_t *hnode,
                                                           const int2 *hseg) {
  __shared__ int32_t s_list[kCandBuf];
  __shared__ int s_cnt;
  __shared__ unsigned long long s_edges, s_base;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) {
    s_cnt = 0;
    s_edges = 0;
  }
  __syncthreads();
  const int64_t nseg = counters[5];
  for (int64_t sgi = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6); sgi < nseg;
       sgi += (int64_t)gridDim.x * kRowsPerBlock) {
    const int2 sg = hseg[sgi];
    const int32_t v = hnode[sg.x];
    const float r0 = (lane < d) ? hbuf[(int64_t)sg.x * d + lane] : 0.f;
    const float r1 = (lane + 64 < d) ? hbuf[(int64_t)sg.x * d + lane + 64] : 0.f;
    const int32_t L = gin.len[v];
    const int32_t b = sg.y * kSegEdges, e = min(L, b + kSegEdges);
    const int32_t *row = gin.col + gin.start[v];
    for (int32_t e0 = b; e0 < e; e0 += 64)
      spread64(row + e0, min(64, e - e0), outdeg, R, d, alpha, r0, r1, round, stamp, s_list,
               &s_cnt, next_cand, counters);
    if (lane == 0) atomicAdd(&s_edges, (unsigned long long)(e - b));
  }
  __syncthreads();
  flush_candidates(s_list, s_cnt, s_edges, next_cand, counters, &s_base);
}

// FP32 copy of a basis stored as BF16 pairs.
__global__ void decode_kernel(const float *M, float *out, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = split_decode(__float_as_uint(M[i]));
}

__global__ void abs_max_kernel(const float *R, int64_t count, unsigned *maxbits) {
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, nan_to_inf(fabsf(R[i])));
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0 && m > 0.f) atomicMax(maxbits, __float_as_uint(m));
}

}  // namespace

hipError_t ppr_init(damf_ctx *c) {
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  const int d = c->d;
  const size_t bytes = (size_t)n * d * sizeof(float);
  if (c->split) {
    decode_kernel<<<stride_grid((int64_t)n * d, 256), 256, 0, s>>>(c->Ub, c->R, (int64_t)n * d);
    DAMF_HIP(hipGetLastError());
  } else {
    DAMF_HIP(hipMemcpyAsync(c->R, c->Ub, bytes, hipMemcpyDeviceToDevice, s));
  }
  DAMF_HIP(hipMemsetAsync(c->Zb, 0, bytes, s));
  float *Rn = nullptr;
  DAMF_HIP(hipMalloc(&Rn, bytes));
  unsigned *maxbits = reinterpret_cast<unsigned *>(c->ws.counters);
  unsigned h = 0;
  const float alpha = (float)c->cfg.alpha;
  // initial max |R|
  DAMF_HIP(hipMemsetAsync(maxbits, 0, sizeof(unsigned), s));
  abs_max_kernel<<<1024, 256, 0, s>>>(c->R, (int64_t)n * d, maxbits);
  DAMF_HIP(hipMemcpyAsync(&h, maxbits, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  SpmmPlan plan;
  DAMF_HIP(spmm_plan_build(c, c->out, d, &plan));
  float *Rcur = c->R, *Rnxt = Rn;
  for (int round = 0; round < 100000; ++round) {
    float mx;
    std::memcpy(&mx, &h, sizeof(float));
    if (!std::isfinite(mx)) {  // NaN or Inf in the factors: stop, do not iterate on it
      c->nonfinite = true;
      break;
    }
    // to eps / 2: a synchronous round lowers every residual together, so
    // stopping at eps would leave many nodes just under it, and the first
    // update's push would cascade through them
    if (!((double)mx > 0.5 * c->cfg.eps)) break;
    DAMF_HIP(hipMemsetAsync(maxbits, 0, sizeof(unsigned), s));
    DAMF_HIP(hipEventRecord(c->ev_k[0], s));
    DAMF_HIP(ppr_pull_round(c->out, plan, Rcur, Rnxt, c->Zb, n, d, alpha, maxbits, s));
    DAMF_HIP(hipEventRecord(c->ev_k[1], s));
    DAMF_HIP(hipMemcpyAsync(&h, maxbits, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    DAMF_HIP(hipStreamSynchronize(s));
    float kms = 0.f;
    DAMF_HIP(hipEventElapsedTime(&kms, c->ev_k[0], c->ev_k[1]));
    c->init_info.ms_spmm_kernel += kms;
    c->init_info.ppr_rounds += 1;
    // compulsory bytes: CSR (start, len, indices), R read once, R' written, Z read + written
    c->init_info.spmm_bytes += 12.0 * n + 4.0 * (double)c->out.nnz_built +
                               4.0 * 4.0 * (double)n * d;
    float *t = Rcur;
    Rcur = Rnxt;
    Rnxt = t;
  }
  if (Rcur != c->R) DAMF_HIP(hipMemcpyAsync(c->R, Rcur, bytes, hipMemcpyDeviceToDevice, s));
  DAMF_HIP(hipStreamSynchronize(s));
  spmm_plan_free(plan);
  DAMF_HIP(hipFree(Rn));
  return hipSuccess;
}

hipError_t ppr_fixup(damf_ctx *c, int n_rows) {
  if (n_rows <= 0) return hipSuccess;
  fixup_kernel<<<ceil_div(n_rows, kRowsPerBlock), 256, 0, c->stream>>>(
      c->out, c->ws.net, c->ws.rows_out, c->ws.rowpos_out, n_rows, c->Ub, c->Zb, c->R, c->d,
      (float)c->cfg.alpha, c->split);
  return hipGetLastError();
}

// first_rows: candidate rows of the first round (device list), or nullptr to
// start from every node.  Runs on stream s (the server overlaps it with the
// next step's chain kernel; R is only ever changed by atomics meanwhile).
constexpr int kPushGrid = 512;

hipError_t ppr_push(damf_ctx *c, hipStream_t s, const int32_t *first_rows, int64_t nfirst,
                    int64_t *rounds, int64_t *pushes, int64_t *edges) {
  Workspace &w = c->ws;
  const int d = c->d;
  *rounds = *pushes = *edges = 0;
  const bool all = (first_rows == nullptr);
  const int64_t ncand0 = all ? c->n : nfirst;
  if (ncand0 <= 0) return hipSuccess;
  // heavy-node buffers: at most edges / kHeavy nodes have more than kHeavy
  // in-neighbours, and their rows hold at most edges / kSegEdges + nodes segments
  const int64_t edges_cap = c->in.pool_cap;
  const int64_t hcap = edges_cap / kHeavy + 64;
  const int64_t scap = edges_cap / kSegEdges + hcap;
  if (w.heavy_cap < hcap || w.hseg_cap < scap) {
    (void)hipFree(w.hbuf);
    (void)hipFree(w.hnode);
    (void)hipFree(w.hseg);
    w.hbuf = nullptr;
    w.hnode = nullptr;
    w.hseg = nullptr;
    w.heavy_cap = w.hseg_cap = 0;
    DAMF_HIP(hipMalloc(&w.hbuf, hcap * d * sizeof(float)));
    DAMF_HIP(hipMalloc(&w.hnode, hcap * sizeof(int32_t)));
    DAMF_HIP(hipMalloc(&w.hseg, scap * sizeof(int2)));
    w.heavy_cap = hcap;
    w.hseg_cap = scap;
  }
  if (!w.push_ring) {
    DAMF_HIP(hipMalloc(&w.push_ring, kPushRing * kPushCounters * sizeof(int64_t)));
    DAMF_HIP(hipMalloc(&w.push_log, 2 * (size_t)kMaxPushRounds * sizeof(int64_t)));
    DAMF_HIP(hipHostMalloc((void **)&w.push_log_host, 2 * (size_t)kMaxPushRounds * sizeof(int64_t)));
  }
  int32_t *cand[2] = {w.cand, w.cand2};
  if (!all) DAMF_HIP(hipMemcpyAsync(cand[0], first_rows, nfirst * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  DAMF_HIP(hipMemsetAsync(w.push_ring, 0, kPushRing * kPushCounters * sizeof(int64_t), s));
  auto ring = [&](int r) { return w.push_ring + (size_t)(r % kPushRing) * kPushCounters; };
  const int32_t id0 = (int32_t)(++c->round_counter & 0x7fffffff);  // first-round dedup stamp
  const float alpha = (float)c->cfg.alpha;
  DAMF_HIP(hipEventRecord(c->ev_k[0], s));
  int r = 0;
  int64_t *last = w.counters_host;  // pinned copy of the last queued round's counters
  for (;;) {
    for (int g = 0; g < kPushGroup; ++g, ++r) {
      const int32_t round = (int32_t)((id0 + 1 + r) & 0x7fffffff);
      // two workgroups per CU: the grids stride over the round's candidates and
      // frontier, and larger grids only cost dispatch time in the late rounds
      // (select and push at 2048, 512 and 256 workgroups: 0.74, 0.69 and 0.77 ms
      // of push kernels per C2 batch)
      select_kernel<<<kPushGrid, 256, 0, s>>>(
          (r == 0 && all) ? nullptr : cand[r & 1], r == 0 ? nullptr : ring(r - 1) + 2, ncand0,
          c->R, d, c->cfg.eps, w.stamp, (r == 0 && !all) ? id0 : -1, w.frontier, ring(r),
          ring(r + 1), r == 0 ? nullptr : ring(r - 1), w.push_log + 2 * (size_t)(r > 0 ? r - 1 : 0));
      push_kernel<<<kPushGrid, 256, 0, s>>>(c->in, c->out.len, w.frontier, c->R, c->Zb, d, alpha,
                                       round, w.stamp, cand[(r + 1) & 1], ring(r), w.hbuf,
                                       w.hnode, reinterpret_cast<int2 *>(w.hseg));
      spread_heavy_kernel<<<kPushGrid / 2, 256, 0, s>>>(c->in, c->out.len, c->R, d, alpha, round, w.stamp,
                                               cand[(r + 1) & 1], ring(r), w.hbuf, w.hnode,
                                               reinterpret_cast<const int2 *>(w.hseg));
    }
    DAMF_HIP(hipGetLastError());
    DAMF_HIP(hipMemcpyAsync(last, ring(r - 1), kPushCounters * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DAMF_HIP(hipStreamSynchronize(s));
    if (last[2] == 0) break;  // no candidates left for another round
    if (r + kPushGroup >= kMaxPushRounds) return hipErrorUnknown;
  }
  DAMF_HIP(hipEventRecord(c->ev_k[1], s));
  if (r > 1)
    DAMF_HIP(hipMemcpyAsync(w.push_log_host, w.push_log, 2 * (size_t)(r - 1) * sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  float kms = 0.f;
  DAMF_HIP(hipEventElapsedTime(&kms, c->ev_k[0], c->ev_k[1]));
  c->push_ms += kms;
  c->round_counter = id0 + 1 + r;
  for (int q = 0; q < r; ++q) {
    const int64_t nf = (q < r - 1) ? w.push_log_host[2 * q] : last[1];
    const int64_t ne = (q < r - 1) ? w.push_log_host[2 * q + 1] : last[3];
    if (nf == 0) continue;
    // compulsory bytes: per pushed node R[v] and Z_b[v] read + written and
    // its in-row metadata; per traversed edge the index, deg(u), R[u] read +
    // written and the stamp word
    c->push_bytes += (double)nf * (4.0 * 4.0 * d + 12.0) + (double)ne * (4.0 + 4.0 + 2.0 * 4.0 * d + 8.0);
    ++*rounds;
    *pushes += nf;
    *edges += ne;
  }
  return hipSuccess;
}

hipError_t ppr_residual_max(damf_ctx *c, double *out) {
  hipStream_t s = c->stream;
  unsigned *maxbits = reinterpret_cast<unsigned *>(c->ws.counters);
  unsigned h = 0;
  DAMF_HIP(hipMemsetAsync(maxbits, 0, sizeof(unsigned), s));
  abs_max_kernel<<<1024, 256, 0, s>>>(c->R, c->n * c->d, maxbits);
  DAMF_HIP(hipGetLastError());
  DAMF_HIP(hipMemcpyAsync(&h, maxbits, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  float f;
  std::memcpy(&f, &h, sizeof(float));
  *out = (double)f;
  return hipSuccess;
}

}  // namespace damf
