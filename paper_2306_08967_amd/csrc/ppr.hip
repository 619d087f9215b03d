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

// One synchronous propagation round over all rows (pull form, out-CSR).
// Waves stride over rows; the block's max |R'| goes out with one atomic.
__global__ __launch_bounds__(256) void pull_round_kernel(Csr g, const float *__restrict__ Rold,
                                                         float *__restrict__ Rnew,
                                                         float *__restrict__ Z, int64_t n, int d,
                                                         float alpha, unsigned *maxbits) {
  __shared__ float bmax[4];
  const int lane = threadIdx.x & 63;
  const bool c0 = lane < d, c1 = lane + 64 < d;
  float m = 0.f;
  const int64_t stride = (int64_t)gridDim.x * kRowsPerBlock;
  for (int64_t u = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6); u < n; u += stride) {
    const int32_t L = g.len[u];
    const int32_t *row = g.col + g.start[u];
    float a0 = 0.f, a1 = 0.f;
    int32_t e = 0;
    for (; e + 4 <= L; e += 4) {
      const int64_t v0 = row[e], v1 = row[e + 1], v2 = row[e + 2], v3 = row[e + 3];
      if (c0) {
        a0 += Rold[v0 * d + lane] + Rold[v1 * d + lane];
        a0 += Rold[v2 * d + lane] + Rold[v3 * d + lane];
      }
      if (c1) {
        a1 += Rold[v0 * d + lane + 64] + Rold[v1 * d + lane + 64];
        a1 += Rold[v2 * d + lane + 64] + Rold[v3 * d + lane + 64];
      }
    }
    for (; e < L; ++e) {
      const int64_t v = row[e];
      if (c0) a0 += Rold[v * d + lane];
      if (c1) a1 += Rold[v * d + lane + 64];
    }
    const float scale = (L > 0) ? (1.f - alpha) / (float)L : 0.f;
    if (c0) {
      const int64_t i = u * d + lane;
      Z[i] += alpha * Rold[i];
      const float r = a0 * scale;
      Rnew[i] = r;
      m = fmaxf(m, fabsf(r));
    }
    if (c1) {
      const int64_t i = u * d + lane + 64;
      Z[i] += alpha * Rold[i];
      const float r = a1 * scale;
      Rnew[i] = r;
      m = fmaxf(m, fabsf(r));
    }
  }
  m = wave_max(m);
  if (lane == 0) bmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float b = fmaxf(fmaxf(bmax[0], bmax[1]), fmaxf(bmax[2], bmax[3]));
    if (b > 0.f) atomicMax(maxbits, __float_as_uint(b));
  }
}

// Structural fix-up for each changed out-row u (before the CSR edit; before
// or after the chain kernel, which adds the same change to U_b and R, so
// alpha (R - X) is unchanged; never while a push runs):
//   P Z_b[u] from the invariant, (alpha (R - X) + Z_b)[u] / (1 - alpha)
//   P'Z_b[u] = (deg_old P Z_b[u] + sum_added Z_b[v] - sum_removed Z_b[v]) / deg_new
__global__ __launch_bounds__(256) void fixup_kernel(Csr g, const NetEntry *net,
                                                    const int32_t *rows, const int32_t *rowpos,
                                                    int nrows, const float *X, const float *Z,
                                                    float *R, int d, float alpha) {
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
    const float pz = (alpha * (R[i] - X[i]) + Z[i]) / (1.f - alpha);
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
// a node pushed twice in one round would race on its Z_b row.
__global__ __launch_bounds__(256) void select_kernel(const int32_t *cand, int64_t ncand,
                                                     const float *R, int d, double eps,
                                                     int32_t *stamp, int32_t dedup_round,
                                                     int32_t *frontier, int64_t *counters) {
  __shared__ int s_cnt;
  __shared__ int32_t s_list[kRowsPerBlock];
  __shared__ unsigned long long s_base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * kRowsPerBlock + w;
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
    s_base = atomicAdd((unsigned long long *)&counters[1], (unsigned long long)s_cnt);
  __syncthreads();
  if (threadIdx.x < s_cnt) frontier[s_base + threadIdx.x] = s_list[threadIdx.x];
}

// Push every frontier node: take R[v] atomically, Z_b[v] += alpha R[v], and
// spread (1 - alpha) R[v] / deg(u) to each in-neighbour u (in-CSR row v).
// New candidates (first touch of u in this round, by stamp) are gathered in
// LDS and appended with one global atomic per block.
constexpr int kCandBuf = 1024;
__global__ __launch_bounds__(256) void push_kernel(Csr gin, const int32_t *outdeg,
                                                   const int32_t *frontier, int64_t nf, float *R,
                                                   float *Z, int d, float alpha, int32_t round,
                                                   int32_t *stamp, int32_t *next_cand,
                                                   int64_t *counters) {
  __shared__ int32_t s_list[kCandBuf];
  __shared__ int s_cnt;
  __shared__ unsigned long long s_edges, s_base;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) {
    s_cnt = 0;
    s_edges = 0;
  }
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
  if (j < nf) {
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
    for (int32_t e0 = 0; e0 < L; e0 += 64) {
      // one neighbour per lane for the stamp check, then the wave updates rows
      const int32_t myu = (e0 + lane < L) ? row[e0 + lane] : -1;
      bool fresh = false;
      if (myu >= 0) fresh = atomicExch(&stamp[myu], round) != round;
      const unsigned long long fm = __ballot(fresh);
      if (fm) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_cnt, __popcll(fm));
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
      const int cnt = min(64, L - e0);
      for (int q = 0; q < cnt; ++q) {
        const int32_t u = __shfl(myu, q, 64);
        const float s = (1.f - alpha) / (float)outdeg[u];
        if (c0) atomicAdd(&R[(int64_t)u * d + lane], s * r0);
        if (c1) atomicAdd(&R[(int64_t)u * d + lane + 64], s * r1);
      }
    }
    if (lane == 0) atomicAdd(&s_edges, (unsigned long long)L);
  }
  __syncthreads();
  const int cnt = min(s_cnt, kCandBuf);
  if (threadIdx.x == 0) {
    s_base = cnt ? atomicAdd((unsigned long long *)&counters[2], (unsigned long long)cnt) : 0;
    if (s_edges) atomicAdd((unsigned long long *)&counters[3], s_edges);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < cnt; i += 256) next_cand[s_base + i] = s_list[i];
}

__global__ void abs_max_kernel(const float *R, int64_t count, unsigned *maxbits) {
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(R[i]));
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0 && m > 0.f) atomicMax(maxbits, __float_as_uint(m));
}

}  // namespace

hipError_t ppr_init(damf_ctx *c) {
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  const int d = c->d;
  const size_t bytes = (size_t)n * d * sizeof(float);
  DAMF_HIP(hipMemcpyAsync(c->R, c->Ub, bytes, hipMemcpyDeviceToDevice, s));
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
  float *Rcur = c->R, *Rnxt = Rn;
  for (int round = 0; round < 100000; ++round) {
    float mx;
    std::memcpy(&mx, &h, sizeof(float));
    if (!((double)mx > c->cfg.eps)) break;
    DAMF_HIP(hipMemsetAsync(maxbits, 0, sizeof(unsigned), s));
    DAMF_HIP(hipEventRecord(c->ev_k[0], s));
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n, kRowsPerBlock), 8192);
    pull_round_kernel<<<grid, 256, 0, s>>>(c->out, Rcur, Rnxt, c->Zb, n, d, alpha, maxbits);
    DAMF_HIP(hipGetLastError());
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
  DAMF_HIP(hipFree(Rn));
  return hipSuccess;
}

hipError_t ppr_fixup(damf_ctx *c, int n_rows) {
  if (n_rows <= 0) return hipSuccess;
  fixup_kernel<<<ceil_div(n_rows, kRowsPerBlock), 256, 0, c->stream>>>(
      c->out, c->ws.net, c->ws.rows_out, c->ws.rowpos_out, n_rows, c->Ub, c->Zb, c->R, c->d,
      (float)c->cfg.alpha);
  return hipGetLastError();
}

// first_rows: candidate rows of the first round (device list), or nullptr to
// start from every node.  Runs on stream s (the server overlaps it with the
// next step's chain kernel; R is only ever changed by atomics meanwhile).
hipError_t ppr_push(damf_ctx *c, hipStream_t s, const int32_t *first_rows, int64_t nfirst,
                    int64_t *rounds, int64_t *pushes, int64_t *edges) {
  Workspace &w = c->ws;
  const int d = c->d;
  *rounds = *pushes = *edges = 0;
  int64_t ncand = first_rows ? nfirst : c->n;
  int32_t *cand = w.cand, *next = w.cand2, *front = w.frontier;
  if (first_rows && ncand > 0)
    DAMF_HIP(hipMemcpyAsync(cand, first_rows, ncand * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  bool all = (first_rows == nullptr);
  bool first = true;
  while (ncand > 0) {
    DAMF_HIP(hipMemsetAsync(w.counters, 0, 4 * sizeof(int64_t), s));
    // the caller's list may repeat rows; later rounds' lists are unique by stamp
    const int32_t dedup = (first && !all) ? (int32_t)(++c->round_counter & 0x7fffffff) : -1;
    select_kernel<<<ceil_div(ncand, kRowsPerBlock), 256, 0, s>>>(
        all ? nullptr : cand, ncand, c->R, d, c->cfg.eps, w.stamp, dedup, front, w.counters);
    all = false;
    first = false;
    DAMF_HIP(hipGetLastError());
    DAMF_HIP(hipMemcpyAsync(w.counters_host, w.counters, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DAMF_HIP(hipStreamSynchronize(s));
    const int64_t nf = w.counters_host[1];
    if (nf == 0) break;
    const int32_t round = (int32_t)(++c->round_counter & 0x7fffffff);
    DAMF_HIP(hipEventRecord(c->ev_k[0], s));
    push_kernel<<<ceil_div(nf, kRowsPerBlock), 256, 0, s>>>(c->in, c->out.len, front, nf, c->R,
                                                            c->Zb, d, (float)c->cfg.alpha, round,
                                                            w.stamp, next, w.counters);
    DAMF_HIP(hipGetLastError());
    DAMF_HIP(hipEventRecord(c->ev_k[1], s));
    DAMF_HIP(hipMemcpyAsync(w.counters_host, w.counters, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DAMF_HIP(hipStreamSynchronize(s));
    float kms = 0.f;
    DAMF_HIP(hipEventElapsedTime(&kms, c->ev_k[0], c->ev_k[1]));
    c->push_ms += kms;
    // compulsory bytes: per pushed node R[v] and Z_b[v] read + written and
    // its in-row metadata; per traversed edge the index, deg(u), R[u] read +
    // written and the stamp word
    c->push_bytes += (double)nf * (4.0 * 4.0 * d + 12.0) +
                     (double)w.counters_host[3] * (4.0 + 4.0 + 2.0 * 4.0 * d + 8.0);
    ++*rounds;
    *pushes += nf;
    *edges += w.counters_host[3];
    ncand = w.counters_host[2];
    int32_t *t = cand;
    cand = next;
    next = t;
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
