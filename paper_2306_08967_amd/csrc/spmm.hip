// spmm.hip -- CSR SpMM Y = A X over dense n x k row blocks (k <= 192), the
// sparse work of the initialisation (Appendix A, Algorithm 3): the products of
// the randomized t-SVD and the synchronous PPR propagation rounds.
//
// Rows with at most kSegLen entries take one wave each (waves stride over the
// rows; with long rows out of the way no wave can collect several hubs).
// Longer rows are cut into segments of kSegLen entries, one wave per segment
// writing a partial row sum; an epilogue wave per long row adds its partials
// in segment order, so the result does not depend on scheduling.  A bounded
// grid keeps the per-block max reduction to a few thousand atomics.
// Lane l of a wave owns columns l, l + 64, l + 128 of the row.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "damf_internal.h"

namespace damf {

namespace {

constexpr int kSegLen = 256;

template <int NC>
__device__ __forceinline__ void gather_sum(const int32_t *row, int32_t L, const float *X, int ld,
                                           int k, float (&acc)[NC]) {
  const int lane = threadIdx.x & 63;
  // columns past k read column k - 1 of the same row (a valid address) and
  // count zero, so every gather of a group can be in flight at once
  int colc[NC];
  float msk[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = lane + 64 * c;
    colc[c] = min(col, k - 1);
    msk[c] = (col < k) ? 1.f : 0.f;
    acc[c] = 0.f;
  }
  int32_t e = 0;
  for (; e + 8 <= L; e += 8) {
    int64_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (int64_t)row[e + q] * ld;
    float x[NC][8];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < 8; ++q) x[c][q] = X[v[q] + colc[c]];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      acc[c] += msk[c] * (((x[c][0] + x[c][1]) + (x[c][2] + x[c][3])) +
                          ((x[c][4] + x[c][5]) + (x[c][6] + x[c][7])));
  }
  for (; e < L; ++e) {
    const int64_t v = (int64_t)row[e] * ld;
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += msk[c] * X[v + colc[c]];
  }
}

// Epilogue shared by the plain product and the PPR round.  mode 0: Y = sum.
// mode 1: Y = (1 - alpha) sum / deg, Z += alpha Xold (Xold = X), max |Y|.
template <int NC>
__device__ __forceinline__ float finish_row(int64_t u, int32_t L, const float (&acc)[NC],
                                            const float *X, float *Y, float *Z, int ld, int k,
                                            int mode, float alpha) {
  const int lane = threadIdx.x & 63;
  float m = 0.f;
  const float scale = (mode == 1) ? ((L > 0) ? (1.f - alpha) / (float)L : 0.f) : 1.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = lane + 64 * c;
    if (col < k) {
      const int64_t i = u * ld + col;
      const float r = acc[c] * scale;
      Y[i] = r;
      if (mode == 1) {
        Z[i] += alpha * X[i];
        m = fmaxf(m, nan_to_inf(fabsf(r)));
      }
    }
  }
  return m;
}

__device__ __forceinline__ void block_max_out(float m, unsigned *maxbits) {
  __shared__ float bmax[4];
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) bmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float b = fmaxf(fmaxf(bmax[0], bmax[1]), fmaxf(bmax[2], bmax[3]));
    if (b > 0.f) atomicMax(maxbits, __float_as_uint(b));
  }
}

template <int NC>
__global__ __launch_bounds__(256) void spmm_rows_kernel(Csr g, const float *__restrict__ X,
                                                        float *__restrict__ Y, float *Z,
                                                        int64_t n, int k, int ld, int mode,
                                                        float alpha, unsigned *maxbits) {
  float m = 0.f;
  for (int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); u < n;
       u += (int64_t)gridDim.x * 4) {
    const int32_t L = g.len[u];
    if (L <= kSegLen) {
      float acc[NC];
      gather_sum<NC>(g.col + g.start[u], L, X, ld, k, acc);
      m = fmaxf(m, finish_row<NC>(u, L, acc, X, Y, Z, ld, k, mode, alpha));
    }
  }
  if (mode == 1) block_max_out(m, maxbits);
}

// One wave per segment of a long row: partial sums into part[seg].
template <int NC>
__global__ __launch_bounds__(256) void spmm_segments_kernel(Csr g, const int32_t *seg_row,
                                                            const int32_t *seg_idx, int64_t nseg,
                                                            const float *__restrict__ X,
                                                            float *__restrict__ part, int k,
                                                            int ld) {
  const int64_t sgi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (sgi >= nseg) return;
  const int32_t u = seg_row[sgi];
  const int32_t L = g.len[u];
  const int32_t b = seg_idx[sgi] * kSegLen;
  float acc[NC];
  gather_sum<NC>(g.col + g.start[u] + b, min(kSegLen, L - b), X, ld, k, acc);
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (lane + 64 * c < k) part[sgi * ld + lane + 64 * c] = acc[c];
}

// One wave per long row: add its partials in segment order, then finish.
template <int NC>
__global__ __launch_bounds__(256) void spmm_long_finish_kernel(
    Csr g, const int32_t *long_row, const int64_t *long_seg0, int64_t nlong,
    const float *__restrict__ part, const float *X, float *Y, float *Z, int k, int ld, int mode,
    float alpha, unsigned *maxbits) {
  const int64_t h = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  float m = 0.f;
  if (h < nlong) {
    const int32_t u = long_row[h];
    const int32_t L = g.len[u];
    const int64_t s0 = long_seg0[h];
    const int ns = (L + kSegLen - 1) / kSegLen;
    float acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.f;
    for (int j = 0; j < ns; ++j) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (lane + 64 * c < k) acc[c] += part[(s0 + j) * ld + lane + 64 * c];
    }
    m = finish_row<NC>(u, L, acc, X, Y, Z, ld, k, mode, alpha);
  }
  if (mode == 1) block_max_out(m, maxbits);
}

// Plan: long rows (append order), their first segment, and the segment list.
__global__ void count_long_kernel(Csr g, int64_t n, int64_t *counts) {
  int64_t rows = 0, segs = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t L = g.len[u];
    if (L > kSegLen) {
      rows += 1;
      segs += (L + kSegLen - 1) / kSegLen;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    rows += __shfl_down(rows, off, 64);
    segs += __shfl_down(segs, off, 64);
  }
  if ((threadIdx.x & 63) == 0 && rows) {
    atomicAdd((unsigned long long *)&counts[0], (unsigned long long)rows);
    atomicAdd((unsigned long long *)&counts[1], (unsigned long long)segs);
  }
}

__global__ void fill_long_kernel(Csr g, int64_t n, int64_t *cursor, int32_t *long_row,
                                 int64_t *long_seg0, int32_t *seg_row, int32_t *seg_idx) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t L = g.len[u];
    if (L <= kSegLen) continue;
    const int32_t ns = (L + kSegLen - 1) / kSegLen;
    const int64_t h = (int64_t)atomicAdd((unsigned long long *)&cursor[0], 1ull);
    const int64_t s0 = (int64_t)atomicAdd((unsigned long long *)&cursor[1], (unsigned long long)ns);
    long_row[h] = (int32_t)u;
    long_seg0[h] = s0;
    for (int32_t j = 0; j < ns; ++j) {
      seg_row[s0 + j] = (int32_t)u;
      seg_idx[s0 + j] = j;
    }
  }
}

}  // namespace

hipError_t spmm_plan_build(damf_ctx *c, const Csr &g, int kmax, SpmmPlan *p) {
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  *p = SpmmPlan{};
  p->ld_max = kmax;
  int64_t *counts = nullptr;
  DAMF_HIP(hipMalloc(&counts, 4 * sizeof(int64_t)));
  DAMF_HIP(hipMemsetAsync(counts, 0, 4 * sizeof(int64_t), s));
  count_long_kernel<<<stride_grid(n, 256), 256, 0, s>>>(g, n, counts);
  DAMF_HIP(hipGetLastError());
  int64_t h[2] = {0, 0};
  DAMF_HIP(hipMemcpyAsync(h, counts, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  p->nlong = h[0];
  p->nseg = h[1];
  if (p->nlong > 0) {
    DAMF_HIP(hipMalloc(&p->long_row, p->nlong * sizeof(int32_t)));
    DAMF_HIP(hipMalloc(&p->long_seg0, p->nlong * sizeof(int64_t)));
    DAMF_HIP(hipMalloc(&p->seg_row, p->nseg * sizeof(int32_t)));
    DAMF_HIP(hipMalloc(&p->seg_idx, p->nseg * sizeof(int32_t)));
    DAMF_HIP(hipMalloc(&p->part, (size_t)p->nseg * kmax * sizeof(float)));
    DAMF_HIP(hipMemsetAsync(counts + 2, 0, 2 * sizeof(int64_t), s));
    fill_long_kernel<<<stride_grid(n, 256), 256, 0, s>>>(g, n, counts + 2, p->long_row, p->long_seg0,
                                                      p->seg_row, p->seg_idx);
    DAMF_HIP(hipGetLastError());
  }
  DAMF_HIP(hipStreamSynchronize(s));
  (void)hipFree(counts);
  return hipSuccess;
}

void spmm_plan_free(SpmmPlan &p) {
  for (void *q : {(void *)p.long_row, (void *)p.long_seg0, (void *)p.seg_row, (void *)p.seg_idx,
                  (void *)p.part})
    if (q) (void)hipFree(q);
  p = SpmmPlan{};
}

template <int NC>
static hipError_t spmm_launch(const Csr &g, const SpmmPlan &p, const float *X, float *Y, float *Z,
                              int64_t n, int k, int ld, int mode, float alpha, unsigned *maxbits,
                              hipStream_t s) {
  const Grid gr = geom_spmm_rows(n), gs = geom_spmm_segments(p.nseg), gl = geom_spmm_long(p.nlong);
  spmm_rows_kernel<NC><<<gr.blocks, gr.threads, 0, s>>>(g, X, Y, Z, n, k, ld, mode, alpha, maxbits);
  DAMF_HIP(hipGetLastError());
  if (p.nlong > 0) {
    spmm_segments_kernel<NC><<<gs.blocks, gs.threads, 0, s>>>(g, p.seg_row, p.seg_idx, p.nseg,
                                                              X, p.part, k, ld);
    spmm_long_finish_kernel<NC><<<gl.blocks, gl.threads, 0, s>>>(
        g, p.long_row, p.long_seg0, p.nlong, p.part, X, Y, Z, k, ld, mode, alpha, maxbits);
    DAMF_HIP(hipGetLastError());
  }
  return hipSuccess;
}

static hipError_t spmm_dispatch(const Csr &g, const SpmmPlan &p, const float *X, float *Y,
                                float *Z, int64_t n, int k, int ld, int mode, float alpha,
                                unsigned *maxbits, hipStream_t s) {
  if (k > 192 || ld > p.ld_max) return hipErrorInvalidValue;
  if (k <= 64) return spmm_launch<1>(g, p, X, Y, Z, n, k, ld, mode, alpha, maxbits, s);
  if (k <= 128) return spmm_launch<2>(g, p, X, Y, Z, n, k, ld, mode, alpha, maxbits, s);
  return spmm_launch<3>(g, p, X, Y, Z, n, k, ld, mode, alpha, maxbits, s);
}

hipError_t csr_spmm(const Csr &g, const SpmmPlan &p, const float *X, float *Y, int64_t n, int k,
                    int ld, hipStream_t s) {
  return spmm_dispatch(g, p, X, Y, nullptr, n, k, ld, 0, 0.f, nullptr, s);
}

hipError_t ppr_pull_round(const Csr &g, const SpmmPlan &p, const float *Rold, float *Rnew,
                          float *Z, int64_t n, int d, float alpha, unsigned *maxbits,
                          hipStream_t s) {
  return spmm_dispatch(g, p, Rold, Rnew, Z, n, d, d, 1, alpha, maxbits, s);
}

}  // namespace damf
