// graph.hip -- device graph store: CSR build, batch preparation (set
// semantics, net change of A, chunking), in-place CSR row edits and canonical
// export.
//
// The paper stores the graph next to the embeddings (Sec. 4.6, O(nd + m)
// space) and turns each edge event into a low-rank change B C^T of A
// (Sec. 4.3).  A batch of ops is reduced to its net change with set
// semantics: the last op on an edge wins, inserting a present edge and
// deleting an absent one change nothing.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <climits>

#include "common.h"
#include "damf_internal.h"

namespace damf {

// ---------------------------------------------------------------------------
// exclusive scan (int64 output) of a per-index value functor

template <typename F>
__global__ __launch_bounds__(1024) void scan_blocks_kernel(F f, int64_t n,
                                                           int64_t *out,
                                                           int64_t *block_sums) {
  __shared__ int64_t wsum[16];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  int64_t v = (i < n) ? f(i) : 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int64_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (w == 0) {
    int64_t s = (lane < 16) ? wsum[lane] : 0;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      int64_t y = __shfl_up(s, off, 64);
      if (lane >= off) s += y;
    }
    if (lane < 16) wsum[lane] = s;
  }
  __syncthreads();
  int64_t base = (w > 0) ? wsum[w - 1] : 0;
  if (i < n) out[i] = base + x - v;
  if (threadIdx.x == 1023) block_sums[blockIdx.x] = base + x;
}

__global__ __launch_bounds__(1024) void scan_sums_kernel(int64_t *sums, int64_t nb,
                                                         int64_t *total) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    int64_t i = b0 + threadIdx.x;
    int64_t v = (i < nb) ? sums[i] : 0;
    int64_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
      int64_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
      int64_t s = (lane < 16) ? wsum[lane] : 0;
      for (int off = 1; off < 16; off <<= 1) {
        int64_t y = __shfl_up(s, off, 64);
        if (lane >= off) s += y;
      }
      if (lane < 16) wsum[lane] = s;
    }
    __syncthreads();
    int64_t base = carry + ((w > 0) ? wsum[w - 1] : 0);
    if (i < nb) sums[i] = base + x - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = base + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void scan_add_kernel(int64_t *out, int64_t n, const int64_t *sums) {
  int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i < n) out[i] += sums[blockIdx.x];
}

// out[i] = sum_{j<i} f(j) for i < n; *total = sum_j f(j).  `tmp` holds
// ceil(n/1024) int64.
template <typename F>
hipError_t exclusive_scan(F f, int64_t n, int64_t *out, int64_t *tmp, int64_t *total,
                          hipStream_t s) {
  if (n <= 0) return hipMemsetAsync(total, 0, sizeof(int64_t), s);
  const Grid g = geom_scan(n);
  const unsigned nb = g.blocks;
  scan_blocks_kernel<<<nb, g.threads, 0, s>>>(f, n, out, tmp);
  scan_sums_kernel<<<1, 1024, 0, s>>>(tmp, nb, total);
  scan_add_kernel<<<nb, g.threads, 0, s>>>(out, n, tmp);
  return hipGetLastError();
}

struct LenOf {
  const int32_t *len;
  __device__ int64_t operator()(int64_t i) const { return len[i]; }
};
struct CapOf {
  const int32_t *len;
  __device__ int64_t operator()(int64_t i) const {
    int64_t l = len[i];
    return l + (l >> 2) + 4;
  }
};

// ---------------------------------------------------------------------------
// CSR build

__global__ void validate_edges_kernel(const int32_t *src, const int32_t *dst, int64_t m,
                                      int64_t n, int32_t *bad) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || (int64_t)u >= n || (int64_t)v >= n) atomicAdd(bad, 1);
  }
}

hipError_t launch_validate_edges(const int32_t *src, const int32_t *dst, int64_t m,
                                 int64_t n, int32_t *bad, hipStream_t s) {
  DAMF_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
  if (m > 0) validate_edges_kernel<<<stride_grid(m, 256), 256, 0, s>>>(src, dst, m, n, bad);
  return hipGetLastError();
}

__global__ void count_rows_kernel(const int32_t *rows, const int32_t *cols, int64_t m,
                                  int32_t undirected, int32_t *cnt) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = rows[e], v = cols[e];
    atomicAdd(&cnt[u], 1);
    if (undirected && u != v) atomicAdd(&cnt[v], 1);
  }
}

__global__ void scatter_rows_kernel(const int32_t *rows, const int32_t *cols, int64_t m,
                                    int32_t undirected, const int64_t *off, int32_t *cursor,
                                    int32_t *tmp) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = rows[e], v = cols[e];
    int32_t p = atomicAdd(&cursor[u], 1);
    tmp[off[u] + p] = v;
    if (undirected && u != v) {
      p = atomicAdd(&cursor[v], 1);
      tmp[off[v] + p] = u;
    }
  }
}

// Sort one segment ascending in LDS and drop duplicates; writes the unique
// count to len[row] and the unique values back to the segment's start.
template <int NT, int CAP>
__device__ void sort_unique_segment(int32_t *seg, int32_t L, int32_t *buf, int32_t *out_len) {
  int P = 1;
  while (P < L) P <<= 1;
  for (int i = threadIdx.x; i < P; i += NT) buf[i] = (i < L) ? seg[i] : INT_MAX;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += NT) {
        int p = i ^ j;
        if (p > i) {
          int32_t a = buf[i], b = buf[p];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            buf[i] = b;
            buf[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // compact unique values (sequential chunks with a block scan)
  __shared__ int32_t wcount[NT / 64 + 1];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < L; base += NT) {
    int i = base + threadIdx.x;
    int keep = (i < L) && (i == 0 || buf[i] != buf[i - 1]);
    unsigned long long bal = __ballot(keep);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[w] = __popcll(bal);
    __syncthreads();
    int off = carry;
    for (int q = 0; q < w; ++q) off += wcount[q];
    int32_t val = (i < L) ? buf[i] : 0;
    __syncthreads();
    if (keep) seg[off + before] = val;
    if (threadIdx.x == 0) {
      int t = 0;
      for (int q = 0; q < NT / 64; ++q) t += wcount[q];
      carry += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out_len = carry;
  __syncthreads();
}

constexpr int kSmallRow = 2048;
constexpr int kLargeRow = 32768;

__global__ __launch_bounds__(256) void sort_rows_small_kernel(int64_t n, const int64_t *off,
                                                              int32_t *len, int32_t *tmp,
                                                              int32_t *big, int32_t *nbig) {
  __shared__ int32_t buf[kSmallRow];
  // rows are workgroup-uniform, so the early continues keep barriers aligned
  for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
    const int32_t L = len[r];
    if (L <= 1) continue;
    if (L > kSmallRow) {
      if (threadIdx.x == 0) big[atomicAdd(nbig, 1)] = (int32_t)r;
      continue;
    }
    sort_unique_segment<256, kSmallRow>(tmp + off[r], L, buf, &len[r]);
  }
}

__global__ __launch_bounds__(1024) void sort_rows_large_kernel(const int32_t *big, int32_t nbig,
                                                               const int64_t *off, int32_t *len,
                                                               int32_t *tmp) {
  __shared__ int32_t buf[kLargeRow];
  // rows are workgroup-uniform: the continue keeps barriers aligned
  for (int32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    __syncthreads();  // the previous row is done with buf
    const int32_t r = big[bi];
    const int32_t L = len[r];
    if (L > kLargeRow) {
      // rows beyond LDS: sorting network in global memory (rare: hub rows).
      // Every comparator is ascending (i < p): the first one of each merge
      // stage pairs i with its mirror i ^ (k - 1), the rest pair i with i ^ j.
      // Positions >= L are a virtual +inf pad that no comparator moves, so
      // nothing is ever written past the row.
      int32_t *seg = tmp + off[r];
      int P = 1;
      while (P < L) P <<= 1;
      for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int i = threadIdx.x; i < P; i += 1024) {
            const int p = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
            if (p > i && p < L) {
              const int32_t a = seg[i], b = seg[p];
              if (a > b) {
                seg[i] = b;
                seg[p] = a;
              }
            }
          }
          __syncthreads();
        }
      }
      // unique in place, single thread (rare path)
      if (threadIdx.x == 0) {
        int32_t w = 0;
        for (int32_t i = 0; i < L; ++i)
          if (i == 0 || seg[i] != seg[i - 1]) seg[w++] = seg[i];
        len[r] = w;
      }
      continue;
    }
    sort_unique_segment<1024, kLargeRow>(tmp + off[r], L, buf, &len[r]);
  }
}

__global__ void copy_rows_kernel(int64_t n, const int64_t *src_off, const int32_t *tmp,
                                 const int64_t *start, const int32_t *len, int32_t *col) {
  // one wave per row
  const int lane = threadIdx.x & 63;
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); r < n;
       r += (int64_t)gridDim.x * (blockDim.x / 64)) {
    const int32_t L = len[r];
    const int32_t *s = tmp + src_off[r];
    int32_t *d = col + start[r];
    for (int32_t j = lane; j < L; j += 64) d[j] = s[j];
  }
}

__global__ void sum_len_kernel(int64_t n, const int32_t *len, int64_t *total) {
  int64_t v = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x)
    v += len[r];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd((unsigned long long *)total, (unsigned long long)v);
}

__global__ void set_caps_kernel(int64_t n, const int32_t *len, int32_t *cap) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t l = len[r];
    cap[r] = l + (l >> 2) + 4;
  }
}

// Pool entries for `used` reserved entries and `edges` edges: at least
// slack * edges, and always a free quarter of the reservations (at least 2^20)
// for rows that outgrow their reservation.
int64_t pool_capacity(int64_t used, int64_t edges, double slack) {
  const int64_t want = (int64_t)(slack * (double)edges) + (1 << 20);
  return used + (want > used ? want - used : 0) + std::max<int64_t>(1 << 20, used / 4);
}

hipError_t csr_build(damf_ctx *c, Csr &g, const int32_t *d_rows, const int32_t *d_cols,
                     int64_t m, double slack) {
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  const int32_t und = c->cfg.directed ? 0 : 1;
  const int64_t m2 = und ? 2 * m : m;
  DAMF_HIP(hipMalloc(&g.start, n * sizeof(int64_t)));
  DAMF_HIP(hipMalloc(&g.len, n * sizeof(int32_t)));
  DAMF_HIP(hipMalloc(&g.cap, n * sizeof(int32_t)));
  DAMF_HIP(hipMalloc(&g.top, sizeof(int64_t)));
  int64_t *off = nullptr, *tmp_sums = nullptr, *total = nullptr;
  int32_t *tmpcol = nullptr, *big = nullptr, *nbig = nullptr;
  DAMF_HIP(hipMalloc(&off, (n + 1) * sizeof(int64_t)));
  DAMF_HIP(hipMalloc(&tmp_sums, (ceil_div(n, 1024) + 1) * sizeof(int64_t)));
  DAMF_HIP(hipMalloc(&total, 2 * sizeof(int64_t)));
  DAMF_HIP(hipMalloc(&tmpcol, (m2 > 0 ? m2 : 1) * sizeof(int32_t)));
  DAMF_HIP(hipMalloc(&big, n * sizeof(int32_t)));
  DAMF_HIP(hipMalloc(&nbig, sizeof(int32_t)));
  DAMF_HIP(hipMemsetAsync(g.len, 0, n * sizeof(int32_t), s));
  DAMF_HIP(hipMemsetAsync(g.cap, 0, n * sizeof(int32_t), s));
  DAMF_HIP(hipMemsetAsync(nbig, 0, sizeof(int32_t), s));
  if (m > 0) {
    count_rows_kernel<<<stride_grid(m, 256), 256, 0, s>>>(d_rows, d_cols, m, und, g.len);
    DAMF_HIP(hipGetLastError());
  }
  DAMF_HIP(exclusive_scan(LenOf{g.len}, n, off, tmp_sums, total, s));
  if (m > 0) {
    scatter_rows_kernel<<<stride_grid(m, 256), 256, 0, s>>>(d_rows, d_cols, m, und, off, g.cap,
                                                         tmpcol);
    DAMF_HIP(hipGetLastError());
  }
  sort_rows_small_kernel<<<stride_grid(n, 1), 256, 0, s>>>(n, off, g.len, tmpcol, big, nbig);
  DAMF_HIP(hipGetLastError());
  int32_t h_nbig = 0;
  DAMF_HIP(hipMemcpyAsync(&h_nbig, nbig, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  if (h_nbig > 0) {
    const Grid gl = geom_sort_large(h_nbig);
    sort_rows_large_kernel<<<gl.blocks, gl.threads, 0, s>>>(big, h_nbig, off, g.len, tmpcol);
    DAMF_HIP(hipGetLastError());
  }
  set_caps_kernel<<<stride_grid(n, 256), 256, 0, s>>>(n, g.len, g.cap);
  DAMF_HIP(hipMemsetAsync(total + 1, 0, sizeof(int64_t), s));
  sum_len_kernel<<<stride_grid(n, 256), 256, 0, s>>>(n, g.len, total + 1);
  DAMF_HIP(hipMemcpyAsync(&g.nnz_built, total + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DAMF_HIP(exclusive_scan(CapOf{g.len}, n, g.start, tmp_sums, total, s));
  int64_t pool_used = 0;
  DAMF_HIP(hipMemcpyAsync(&pool_used, total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  g.pool_cap = pool_capacity(pool_used, m2, slack);
  DAMF_HIP(hipMalloc(&g.col, g.pool_cap * sizeof(int32_t)));
  copy_rows_kernel<<<stride_grid(n, 4), 256, 0, s>>>(n, off, tmpcol, g.start, g.len, g.col);
  DAMF_HIP(hipGetLastError());
  DAMF_HIP(hipMemcpyAsync(g.top, &pool_used, sizeof(int64_t), hipMemcpyHostToDevice, s));
  DAMF_HIP(hipStreamSynchronize(s));
  (void)hipFree(off);
  (void)hipFree(tmp_sums);
  (void)hipFree(total);
  (void)hipFree(tmpcol);
  (void)hipFree(big);
  (void)hipFree(nbig);
  return hipSuccess;
}

hipError_t csr_free(Csr &g) {
  (void)hipFree(g.start);
  (void)hipFree(g.len);
  (void)hipFree(g.cap);
  (void)hipFree(g.col);
  (void)hipFree(g.top);
  g = Csr{};
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// canonical export

__global__ void gather_rows_kernel(int64_t n, const int64_t *start, const int32_t *len,
                                   const int32_t *col, const int64_t *indptr, int32_t *out) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); r < n;
       r += (int64_t)gridDim.x * (blockDim.x / 64)) {
    const int32_t L = len[r];
    const int32_t *s = col + start[r];
    int32_t *d = out + indptr[r];
    for (int32_t j = lane; j < L; j += 64) d[j] = s[j];
  }
}

hipError_t csr_export(damf_ctx *c, const Csr &g, int64_t *h_indptr, int32_t *h_indices,
                      int64_t *m_out) {
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  int64_t *indptr = nullptr, *tmp_sums = nullptr, *total = nullptr;
  DAMF_HIP(hipMalloc(&indptr, (n + 1) * sizeof(int64_t)));
  DAMF_HIP(hipMalloc(&tmp_sums, (ceil_div(n, 1024) + 1) * sizeof(int64_t)));
  DAMF_HIP(hipMalloc(&total, sizeof(int64_t)));
  DAMF_HIP(exclusive_scan(LenOf{g.len}, n, indptr, tmp_sums, total, s));
  DAMF_HIP(hipMemcpyAsync(indptr + n, total, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  int64_t m = 0;
  DAMF_HIP(hipMemcpyAsync(&m, total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  if (m_out) *m_out = m;
  if (h_indptr) DAMF_HIP(hipMemcpy(h_indptr, indptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (h_indices && m > 0) {
    int32_t *idx = nullptr;
    DAMF_HIP(hipMalloc(&idx, m * sizeof(int32_t)));
    gather_rows_kernel<<<stride_grid(n, 4), 256, 0, s>>>(n, g.start, g.len, g.col, indptr, idx);
    DAMF_HIP(hipGetLastError());
    DAMF_HIP(hipMemcpyAsync(h_indices, idx, m * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DAMF_HIP(hipStreamSynchronize(s));
    (void)hipFree(idx);
  }
  (void)hipFree(indptr);
  (void)hipFree(tmp_sums);
  (void)hipFree(total);
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// batch preparation: one workgroup turns k ops into the sorted net change of
// A, the row runs of A and A^T to edit, and the chunk list.

constexpr int kPrepThreads = 1024;

__device__ __forceinline__ bool csr_has(const Csr g, int32_t u, int32_t v) {
  const int32_t *row = g.col + g.start[u];
  int32_t L = g.len[u];
  int32_t lo = 0, hi = L;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (row[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < L && row[lo] == v;
}

// block-wide exclusive scan of one int per thread (1024 threads); returns the
// exclusive prefix, *total receives the sum.
__device__ int block_scan_excl(int v, int *wbuf, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wbuf[w] = x;
  __syncthreads();
  if (w == 0) {
    int s = (lane < 16) ? wbuf[lane] : 0;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      int y = __shfl_up(s, off, 64);
      if (lane >= off) s += y;
    }
    if (lane < 16) wbuf[lane] = s;
  }
  __syncthreads();
  int base = (w > 0) ? wbuf[w - 1] : 0;
  int tot = wbuf[15];
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// ascending bitonic sort of P (power of two) uint64 keys in LDS
__device__ void bitonic_u64(uint64_t *a, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += kPrepThreads) {
        int p = i ^ j;
        if (p > i) {
          uint64_t x = a[i], y = a[p];
          bool up = (i & k) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

struct PrepParams {
  const int32_t *src, *dst;
  const int8_t *op;
  int32_t k;
  int64_t n;
  int32_t directed;
  int32_t r, r_max;
  Csr out;
  const int32_t *seg_end;  // request segments: op ranges [seg_end[s-1], seg_end[s]); last == k
  int32_t nseg;
  uint64_t *units;       // per-request units (u << 33 | v << 1 | insert), (segment, edge) order
  int32_t *unit_seg;     // segment of each unit
  uint64_t *units_comb;  // units of the whole batch's net change, edge order
  int32_t *seg_stats;    // per segment: net entries, chunks
  NetEntry *net, *net_t;
  int32_t *rows_out, *rowpos_out, *rows_in, *rowpos_in;
  ChunkDesc *chunks;
  int32_t *chunk_s1, *chunk_s2;
  NetEntry *chunk_ent;
  BatchHeader *hdr;
};

// LDS layout: phase 1 uses keys (8192 x u64) + idx (8192 x u16) + two delta
// arrays (8192 x i8 each) + the unit order buffer (8192 x u32); phase 2
// reuses the same bytes for up to 16384 entry keys.
constexpr int kPrepLdsBytes = kMaxBatch * (8 + 2 + 1 + 1 + 4);
static_assert(kPrepLdsBytes >= 2 * kMaxBatch * 8, "entry keys must fit");


// Sort `ne` entry keys (hi << 33 | lo << 1 | insert) held in LDS and write
// them out as NetEntry in A's coordinates, with the runs of equal `hi`:
// rows[j] = hi of run j, rowpos[j] = its first entry, rowpos[nruns] = ne.
// NetEntry.pad receives the number of inserts before the entry in the whole
// sorted list; the inserts before it within its run are pad - pad(run start).
__device__ int emit_sorted_entries(uint64_t *ent, int ne, bool transposed, NetEntry *dst,
                                   int32_t *rows, int32_t *rowpos, int *wbuf) {
  int P = 1;
  while (P < ne) P <<= 1;
  for (int i = ne + threadIdx.x; i < P; i += kPrepThreads) ent[i] = ~0ull;
  __syncthreads();
  bitonic_u64(ent, P);
  int carry_runs = 0, carry_ins = 0;
  for (int base = 0; base < ne; base += kPrepThreads) {
    int i = base + threadIdx.x;
    int32_t hi = 0, lo = 0, ins = 0, start = 0;
    if (i < ne) {
      uint64_t e = ent[i];
      hi = (int32_t)(e >> 33);
      lo = (int32_t)((e >> 1) & 0x7fffffffu);
      ins = (int32_t)(e & 1u);
      start = (i == 0) || ((int32_t)(ent[i - 1] >> 33) != hi);
    }
    int tot_runs = 0, tot_ins = 0;
    int rs = block_scan_excl(start, wbuf, &tot_runs);
    int is = block_scan_excl(ins, wbuf, &tot_ins);
    if (i < ne) {
      if (start) {
        rows[carry_runs + rs] = hi;
        rowpos[carry_runs + rs] = i;
      }
      NetEntry en;
      en.row = transposed ? lo : hi;
      en.col = transposed ? hi : lo;
      en.delta = ins ? 1 : -1;
      en.pad = carry_ins + is;
      dst[i] = en;
    }
    carry_runs += tot_runs;
    carry_ins += tot_ins;
  }
  if (threadIdx.x == 0) rowpos[carry_runs] = ne;
  __syncthreads();
  return carry_runs;
}

__device__ __forceinline__ uint64_t entry_key(int32_t hi, int32_t lo, int ins) {
  return ((uint64_t)(uint32_t)hi << 33) | ((uint64_t)(uint32_t)lo << 1) | (uint64_t)(ins & 1);
}

// ascending bitonic sort of P (power of two) uint32 values in LDS
__device__ void bitonic_u32(uint32_t *a, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += kPrepThreads) {
        int q = i ^ j;
        if (q > i) {
          uint32_t x = a[i], y = a[q];
          bool up = (i & k) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[q] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

// The batch is a sequence of request segments applied in order.  Each
// request's net change is taken against the graph its predecessors leave
// (edge-set semantics: the last op of a request on an edge decides), its
// units are chunked on their own (a chunk never spans two requests), and the
// graph edits use the net change of the whole batch.  With one segment this
// is the plain batch.
__device__ void set_header(BatchHeader *h, int bad, int ne, int nchunks, int rows_out,
                           int rows_in, int maxs, int s1tot, int s2tot) {
  h->bad_ops = bad;
  h->n_net = ne;
  h->n_chunks = nchunks;
  h->n_rows_out = rows_out;
  h->n_rows_in = rows_in;
  h->max_s = maxs;
  h->pool_overflow = 0;
  h->s1_total = s1tot;
  h->s2_total = s2tot;
}

__global__ __launch_bounds__(kPrepThreads) void batch_prepare_kernel(PrepParams p) {
  __shared__ __align__(16) unsigned char lds[kPrepLdsBytes];
  __shared__ int wbuf[16];
  __shared__ int s_bad;
  __shared__ int s_segend[kMaxRequests];
  uint64_t *key = reinterpret_cast<uint64_t *>(lds);
  uint16_t *idx = reinterpret_cast<uint16_t *>(lds + kMaxBatch * 8);
  int8_t *dl = reinterpret_cast<int8_t *>(lds + kMaxBatch * 10);
  int8_t *dlc = reinterpret_cast<int8_t *>(lds + kMaxBatch * 11);
  uint32_t *order = reinterpret_cast<uint32_t *>(lds + kMaxBatch * 12);
  const int k = p.k;
  const int nseg = p.nseg;
  int P = 1;
  while (P < k) P <<= 1;
  if (threadIdx.x == 0) s_bad = 0;
  for (int s = threadIdx.x; s < nseg; s += kPrepThreads) s_segend[s] = p.seg_end[s];
  for (int s = threadIdx.x; s < 2 * nseg; s += kPrepThreads) p.seg_stats[s] = 0;
  __syncthreads();
  // segment of op i: the first s with seg_end[s] > i
  auto seg_of = [&](int i) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (s_segend[mid] > i)
        hi = mid;
      else
        lo = mid + 1;
    }
    return lo;
  };
  // ---- phase 1: validate and sort ops by (canonical edge, order)
  for (int i = threadIdx.x; i < P; i += kPrepThreads) {
    uint64_t kk = ~0ull;
    if (i < k) {
      int32_t u = p.src[i], v = p.dst[i];
      int o = p.op[i];
      if (u < 0 || v < 0 || (int64_t)u >= p.n || (int64_t)v >= p.n || (o != 1 && o != -1)) {
        atomicAdd(&s_bad, 1);
      } else {
        if (!p.directed && u > v) {
          int32_t t = u;
          u = v;
          v = t;
        }
        // u in bits 33..63, v in bits 2..32; equal edges keep batch order via idx
        kk = (((uint64_t)(uint32_t)u) << 33) | ((uint64_t)(uint32_t)v << 2);
      }
    }
    key[i] = kk;
    idx[i] = (uint16_t)i;
  }
  __syncthreads();
  if (s_bad > 0) {
    if (threadIdx.x == 0) set_header(p.hdr, s_bad, 0, 0, 0, 0, 0, 0, 0);
    return;
  }
  // sort (key, idx) pairs; equal keys keep batch order through idx
  for (int kk = 2; kk <= P; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += kPrepThreads) {
        int q = i ^ j;
        if (q > i) {
          uint64_t a = key[i], b = key[q];
          uint16_t ia = idx[i], ib = idx[q];
          bool gt = (a > b) || (a == b && ia > ib);
          bool up = (i & kk) == 0;
          if (gt == up) {
            key[i] = b;
            key[q] = a;
            idx[i] = ib;
            idx[q] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  // Per (edge, request) group: the group's last op against the state before
  // the group (the previous group's last op on the edge, else presence in A).
  // Per edge: the last op against presence in A (the batch's net change).
  for (int i = threadIdx.x; i < k; i += kPrepThreads) {
    int8_t d = 0, dc = 0;
    const uint64_t kk = key[i];
    const int sg = seg_of(idx[i]);
    const bool run_last = (i == k - 1) || key[i + 1] != kk;
    const bool grp_last = run_last || seg_of(idx[i + 1]) != sg;
    if (grp_last) {
      const int32_t u = (int32_t)(kk >> 33), v = (int32_t)((kk >> 2) & 0x7fffffffu);
      int g0 = i;
      while (g0 > 0 && key[g0 - 1] == kk && seg_of(idx[g0 - 1]) == sg) --g0;
      const bool after = p.op[idx[i]] == 1;
      bool before;
      int pres = -1;
      if (g0 > 0 && key[g0 - 1] == kk) {
        before = p.op[idx[g0 - 1]] == 1;
      } else {
        pres = csr_has(p.out, u, v) ? 1 : 0;
        before = pres != 0;
      }
      d = (int8_t)((int)after - (int)before);
      if (run_last) {
        if (pres < 0) pres = csr_has(p.out, u, v) ? 1 : 0;
        dc = (int8_t)((int)after - pres);
      }
    }
    dl[i] = d;
    dlc[i] = dc;
  }
  __syncthreads();
  // compact the units (edge order) with their segment, and the batch's units
  int n_units = 0, n_comb = 0;
  for (int base = 0; base < k; base += kPrepThreads) {
    int i = base + threadIdx.x;
    int f = (i < k) && dl[i] != 0;
    int fc = (i < k) && dlc[i] != 0;
    int tot = 0, totc = 0;
    int pos = block_scan_excl(f, wbuf, &tot);
    int posc = block_scan_excl(fc, wbuf, &totc);
    if (f || fc) {
      int32_t u = (int32_t)(key[i] >> 33), v = (int32_t)((key[i] >> 2) & 0x7fffffffu);
      if (f) {
        p.units[n_units + pos] = entry_key(u, v, dl[i] > 0);
        order[n_units + pos] = ((uint32_t)seg_of(idx[i]) << 16) | (uint32_t)(n_units + pos);
      }
      if (fc) p.units_comb[n_comb + posc] = entry_key(u, v, dlc[i] > 0);
    }
    n_units += tot;
    n_comb += totc;
  }
  __syncthreads();
  // units into (segment, edge) order: a stable sort by segment
  if (nseg > 1) {
    int P2 = 1;
    while (P2 < n_units) P2 <<= 1;
    for (int i = n_units + threadIdx.x; i < P2; i += kPrepThreads) order[i] = 0xffffffffu;
    __syncthreads();
    bitonic_u32(order, P2);
  }
  {
    constexpr int PER = kMaxBatch / kPrepThreads;
    uint64_t uk[PER];
    int us[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int t = threadIdx.x + q * kPrepThreads;
      if (t < n_units) {
        uk[q] = p.units[order[t] & 0xffffu];
        us[q] = (int)(order[t] >> 16);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int t = threadIdx.x + q * kPrepThreads;
      if (t < n_units) {
        p.units[t] = uk[q];
        p.unit_seg[t] = us[q];
      }
    }
  }
  __syncthreads();
  // ---- phase 2: entries of the batch's net change sorted by (row, col)
  uint64_t *ent = reinterpret_cast<uint64_t *>(lds);
  int ne = 0;
  for (int base = 0; base < n_comb; base += kPrepThreads) {
    int i = base + threadIdx.x;
    int cnt = 0;
    uint64_t uk = 0;
    if (i < n_comb) {
      uk = p.units_comb[i];
      int32_t u = (int32_t)(uk >> 33), v = (int32_t)((uk >> 1) & 0x7fffffffu);
      cnt = (p.directed || u == v) ? 1 : 2;
    }
    int tot = 0;
    int pos = block_scan_excl(cnt, wbuf, &tot);
    if (i < n_comb) {
      int32_t u = (int32_t)(uk >> 33), v = (int32_t)((uk >> 1) & 0x7fffffffu);
      int ins = (int)(uk & 1u);
      ent[ne + pos] = entry_key(u, v, ins);
      if (cnt == 2) ent[ne + pos + 1] = entry_key(v, u, ins);
    }
    ne += tot;
  }
  __syncthreads();
  int n_rows_out = emit_sorted_entries(ent, ne, false, p.net, p.rows_out, p.rowpos_out, wbuf);
  // ---- phase 3: same entries sorted by (col, row)
  for (int i = threadIdx.x; i < ne; i += kPrepThreads) {
    NetEntry en = p.net[i];
    ent[i] = entry_key(en.col, en.row, en.delta > 0);
  }
  __syncthreads();
  int n_rows_in = emit_sorted_entries(ent, ne, true, p.net_t, p.rows_in, p.rowpos_in, wbuf);
  // ---- phase 4: greedy chunking of the units (one wave, sequential)
  __shared__ int s_nchunks, s_maxs, s_s1tot, s_s2tot;
  // the wave's window of 64 units and the per-request counts live in LDS: a
  // window in VGPRs, or a read-modify-write of the counts in global memory,
  // makes every step wait for the vector-memory counter, which the entry
  // stores keep busy
  __shared__ uint64_t s_wuk[64];
  __shared__ int s_wsg[64];
  __shared__ int s_segc[2 * kMaxRequests];
  for (int i = threadIdx.x; i < 2 * nseg; i += kPrepThreads) s_segc[i] = 0;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int32_t s1v = -1, s2v = -1;  // lane-held members of S1 and S2
    int s1 = 0, s2 = 0, cur_units = 0, e_start = 0, e_cnt = 0, cur_seg = 0;
    int nchunks = 0, maxs = 0, s1_total = 0, s2_total = 0;
    auto close = [&](void) {
      // sort the lane-held lists by rank and write them out
      int r1 = 0, r2 = 0;
      for (int q = 0; q < 64; ++q) {
        int32_t a = __shfl(s1v, q, 64), b = __shfl(s2v, q, 64);
        if (q < s1 && a < s1v) ++r1;
        if (q < s2 && b < s2v) ++r2;
      }
      if (lane < s1) p.chunk_s1[s1_total + r1] = s1v;
      if (lane < s2) p.chunk_s2[s2_total + r2] = s2v;
      if (lane == 0) {
        ChunkDesc c{};
        c.s1_off = s1_total;
        c.s1 = s1;
        c.s2_off = s2_total;
        c.s2 = s2;
        c.e_off = e_start;
        c.ne = e_cnt;
        p.chunks[nchunks] = c;
        s_segc[2 * cur_seg + 1] += 1;
      }
      maxs = max(maxs, max(s1, s2));
      s1_total += s1;
      s2_total += s2;
      ++nchunks;
      e_start += e_cnt;
      e_cnt = 0;
      s1 = s2 = 0;
      s1v = s2v = -1;
      cur_units = 0;
    };
    // the units arrive 64 at a time (one per lane, through LDS) and are read
    // one by one (a global load per unit would put its latency on every step)
    int acc_seg = -1, acc_cnt = 0;  // lane 0: the current segment's entry count
    for (int t = 0; t < n_units; ++t) {
      if ((t & 63) == 0) {
        const int q = t + lane;
        s_wuk[lane] = (q < n_units) ? p.units[q] : 0ull;
        s_wsg[lane] = (q < n_units) ? p.unit_seg[q] : 0;
        __builtin_amdgcn_wave_barrier();  // LDS operations of one wave complete in order
      }
      const int at = t & 63;
      const uint64_t ukv = s_wuk[at];
      const uint32_t ulo = __builtin_amdgcn_readfirstlane((uint32_t)ukv);
      const uint32_t uhi = __builtin_amdgcn_readfirstlane((uint32_t)(ukv >> 32));
      const uint64_t uk = ((uint64_t)uhi << 32) | ulo;
      const int sg = __builtin_amdgcn_readfirstlane(s_wsg[at]);
      int32_t u = (int32_t)(uk >> 33), v = (int32_t)((uk >> 1) & 0x7fffffffu);
      int ins = (int)(uk & 1u);
      bool pair = !p.directed && u != v;
      // rows {u} (+{v}), cols {v} (+{u})
      int32_t r0 = u, r1x = pair ? v : -1, c0 = v, c1x = pair ? u : -1;
      auto count_new = [&](int32_t a, int32_t b, int32_t mine, int cnt) {
        int newc = 0;
        bool ina = __ballot(lane < cnt && mine == a) != 0ull;
        if (!ina) ++newc;
        if (b >= 0 && b != a) {
          bool inb = __ballot(lane < cnt && mine == b) != 0ull;
          if (!inb) ++newc;
        }
        return newc;
      };
      int n1 = count_new(r0, r1x, s1v, s1), n2 = count_new(c0, c1x, s2v, s2);
      int ns1 = s1 + n1, ns2 = s2 + n2;
      if (cur_units > 0 &&
          (sg != cur_seg || !(min(ns1, ns2) <= p.r && max(ns1, ns2) <= p.r_max)))
        close();
      cur_seg = sg;
      // add members
      auto add = [&](int32_t a, int32_t &mine, int &cnt) {
        bool in = __ballot(lane < cnt && mine == a) != 0ull;
        if (!in) {
          if (lane == cnt) mine = a;
          ++cnt;
        }
      };
      add(r0, s1v, s1);
      if (r1x >= 0) add(r1x, s1v, s1);
      add(c0, s2v, s2);
      if (c1x >= 0) add(c1x, s2v, s2);
      // entries of the unit
      if (lane == 0) {
        NetEntry en;
        en.row = u;
        en.col = v;
        en.delta = ins ? 1 : -1;
        en.pad = 0;
        p.chunk_ent[e_start + e_cnt] = en;
        if (pair) {
          en.row = v;
          en.col = u;
          p.chunk_ent[e_start + e_cnt + 1] = en;
        }
        // entries per segment, flushed when the segment changes (units come
        // in segment order)
        if (sg != acc_seg) {
          if (acc_seg >= 0) s_segc[2 * acc_seg] += acc_cnt;
          acc_seg = sg;
          acc_cnt = 0;
        }
        acc_cnt += pair ? 2 : 1;
      }
      e_cnt += pair ? 2 : 1;
      ++cur_units;
    }
    if (cur_units > 0) close();
    if (lane == 0 && acc_seg >= 0) s_segc[2 * acc_seg] += acc_cnt;
    if (lane == 0) {
      s_nchunks = nchunks;
      s_maxs = maxs;
      s_s1tot = s1_total;
      s_s2tot = s2_total;
    }
  }
  __syncthreads();
  // ---- phase 5: chunks whose S1 meets the previous chunk's S1, or whose S2
  // meets its S2 (both lists sorted): Step 1 of such a chunk reads rows that
  // the previous chunk's Step 3 writes, so the host orders the two
  __shared__ unsigned long long s_meets[kMaxBatch / 64];
  for (int i = threadIdx.x; i < kMaxBatch / 64; i += kPrepThreads) s_meets[i] = 0ull;
  __syncthreads();
  // one wave per chunk j; lane l looks up entry l of chunk j's lists (at most
  // 64 each) in chunk j - 1's sorted lists
  for (int i = threadIdx.x; i < 2 * nseg; i += kPrepThreads) p.seg_stats[i] = s_segc[i];
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    auto has = [](const int32_t *a, int na, int32_t x) {
      const int64_t q = lower_bound(a, (int64_t)na, x);
      return q < na && a[q] == x;
    };
    for (int j = 1 + wv; j < s_nchunks; j += kPrepThreads / 64) {
      const ChunkDesc a = p.chunks[j - 1], b = p.chunks[j];
      const bool m1 = lane < b.s1 && has(p.chunk_s1 + a.s1_off, a.s1, p.chunk_s1[b.s1_off + lane]);
      const bool m2 = lane < b.s2 && has(p.chunk_s2 + a.s2_off, a.s2, p.chunk_s2[b.s2_off + lane]);
      if (__ballot(m1 || m2) != 0ull && lane == 0) atomicOr(&s_meets[j >> 6], 1ull << (j & 63));
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kMaxBatch / 64; i += kPrepThreads) p.hdr->meets_prev[i] = s_meets[i];
  if (threadIdx.x == 0)
    set_header(p.hdr, 0, ne, s_nchunks, n_rows_out, n_rows_in, s_maxs, s_s1tot, s_s2tot);
}

hipError_t launch_batch_prepare(damf_ctx *c, int k, int nseg) {
  PrepParams p;
  p.src = c->ws.ops_src;
  p.dst = c->ws.ops_dst;
  p.op = c->ws.ops_op;
  p.k = k;
  p.n = c->n;
  p.directed = c->cfg.directed;
  p.r = c->cfg.max_core_rank;
  p.r_max = c->cfg.max_side;
  p.out = c->out;
  p.seg_end = c->ws.seg_end;
  p.nseg = nseg;
  p.units = c->ws.units;
  p.unit_seg = c->ws.unit_seg;
  p.units_comb = c->ws.units_comb;
  p.seg_stats = c->ws.seg_stats;
  p.net = c->ws.net;
  p.net_t = c->ws.net_t;
  p.rows_out = c->ws.rows_out;
  p.rowpos_out = c->ws.rowpos_out;
  p.rows_in = c->ws.rows_in;
  p.rowpos_in = c->ws.rowpos_in;
  p.chunks = c->ws.chunks;
  p.chunk_s1 = c->ws.chunk_s1;
  p.chunk_s2 = c->ws.chunk_s2;
  p.chunk_ent = c->ws.chunk_ent;
  p.hdr = c->ws.hdr;
  batch_prepare_kernel<<<1, kPrepThreads, 0, c->stream>>>(p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CSR row edits: one workgroup per changed row.  Old elements move to
// i - p + 2 ins(p) where p counts the row's edits below them; inserted
// elements go to lb - q + 2 ins(q) (lb = old elements below, q = edits below).

constexpr int kEditThreads = 256;
constexpr int kEditStage = 8192;

// A row that keeps fitting its reservation is edited in place: it is staged
// (LDS up to kEditStage entries, else a slice of the global staging pool) and
// written back.  A row that outgrows its reservation, or finds the staging
// pool full, moves to fresh pool space (the old space is reclaimed by the
// next compaction).
__global__ __launch_bounds__(kEditThreads) void csr_edit_kernel(Csr g, const NetEntry *ent,
                                                                const int32_t *rows,
                                                                const int32_t *rowpos,
                                                                int transposed,
                                                                int32_t *overflow,
                                                                int32_t *gstage,
                                                                int64_t *gstage_top,
                                                                int64_t gstage_cap) {
  __shared__ int32_t stage[kEditStage];
  __shared__ int64_t s_newstart, s_gstage;
  __shared__ int32_t s_newcap;
  const int j = blockIdx.x;
  const int32_t R = rows[j];
  const int e0 = rowpos[j], nr = rowpos[j + 1] - e0;
  const NetEntry *E = ent + e0;
  const int32_t L = g.len[R], C = g.cap[R];
  const int64_t S = g.start[R];
  const int base_ins = E[0].pad;
  const int tot_ins = E[nr - 1].pad + (E[nr - 1].delta > 0) - base_ins;
  const int32_t newL = L + tot_ins - (nr - tot_ins);
  auto val = [&](int q) { return transposed ? E[q].row : E[q].col; };
  const bool fits = newL <= C;
  const bool lds = fits && (L <= kEditStage);
  if (threadIdx.x == 0) {
    s_gstage = -1;
    bool move = !fits;
    if (fits && !lds) {
      const int64_t at = (int64_t)atomicAdd((unsigned long long *)gstage_top,
                                            (unsigned long long)L);
      if (at + L <= gstage_cap)
        s_gstage = at;
      else
        move = true;
    }
    if (!move) {
      s_newstart = S;
      s_newcap = C;
    } else {
      int32_t nc = newL + (newL >> 1) + 8;
      int64_t at = atomicAdd((unsigned long long *)g.top, (unsigned long long)nc);
      if (at + nc > g.pool_cap) {
        atomicAdd(overflow, 1);
        s_newcap = -1;
      } else {
        s_newstart = at;
        s_newcap = nc;
      }
    }
  }
  __syncthreads();
  const int32_t *old = g.col + S;
  const int64_t gs = s_gstage;
  if (lds) {
    for (int i = threadIdx.x; i < L; i += kEditThreads) stage[i] = old[i];
  } else if (gs >= 0) {
    for (int i = threadIdx.x; i < L; i += kEditThreads) gstage[gs + i] = old[i];
  }
  __syncthreads();
  if (s_newcap < 0) return;
  const int32_t *src = lds ? stage : (gs >= 0 ? gstage + gs : old);
  int32_t *dstrow = g.col + s_newstart;
  for (int i = threadIdx.x; i < L; i += kEditThreads) {
    int32_t x = src[i];
    int lo = 0, hi = nr;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (val(mid) < x)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < nr && val(lo) == x) continue;  // deleted
    int insb = (lo < nr) ? (E[lo].pad - base_ins) : tot_ins;
    dstrow[i - lo + 2 * insb] = x;
  }
  for (int q = threadIdx.x; q < nr; q += kEditThreads) {
    if (E[q].delta < 0) continue;
    int32_t x = val(q);
    int lo = 0, hi = L;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (src[mid] < x)
        lo = mid + 1;
      else
        hi = mid;
    }
    int insb = E[q].pad - base_ins;
    dstrow[lo - q + 2 * insb] = x;
  }
  if (threadIdx.x == 0) {
    g.len[R] = newL;
    g.start[R] = s_newstart;
    g.cap[R] = s_newcap;
  }
}

// Pool space the edit of these rows may take: every row that outgrows its
// reservation moves to newL + newL/2 + 8 fresh entries.
__global__ void csr_need_kernel(Csr g, const NetEntry *ent, const int32_t *rows,
                                const int32_t *rowpos, int nrows, int64_t *need) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  int64_t v = 0;
  if (j < nrows) {
    const int32_t R = rows[j];
    const int e0 = rowpos[j], nr = rowpos[j + 1] - e0;
    const NetEntry *E = ent + e0;
    const int tot_ins = E[nr - 1].pad + (E[nr - 1].delta > 0) - E[0].pad;
    const int32_t newL = g.len[R] + tot_ins - (nr - tot_ins);
    if (newL > g.cap[R]) v = newL + (newL >> 1) + 8;
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd((unsigned long long *)need, (unsigned long long)v);
}

hipError_t launch_csr_need(damf_ctx *c, const Csr &g, const NetEntry *net, const int32_t *rows,
                           const int32_t *rowpos, int nrows, int64_t *need) {
  DAMF_HIP(hipMemsetAsync(need, 0, sizeof(int64_t), c->stream));
  if (nrows <= 0) return hipSuccess;
  csr_need_kernel<<<ceil_div(nrows, 256), 256, 0, c->stream>>>(g, net, rows, rowpos, nrows, need);
  return hipGetLastError();
}

hipError_t launch_csr_edit(damf_ctx *c, Csr &g, const NetEntry *net, const int32_t *rows,
                           const int32_t *rowpos, int nrows, bool transposed) {
  if (nrows <= 0) return hipSuccess;
  DAMF_HIP(hipMemsetAsync(c->ws.edit_stage_top, 0, sizeof(int64_t), c->stream));
  csr_edit_kernel<<<nrows, kEditThreads, 0, c->stream>>>(
      g, net, rows, rowpos, transposed ? 1 : 0, &c->ws.hdr->pool_overflow, c->ws.edit_stage,
      c->ws.edit_stage_top, kEditStagePool);
  return hipGetLastError();
}

// Rebuilds the pool compactly: every row gets a fresh reservation
// (len + len/4 + 4) at its prefix-sum position, the space left by moved rows
// is dropped, and the pool is sized as at build time for the current edges
// with at least min_free free entries.
hipError_t csr_compact(damf_ctx *c, Csr &g, double slack, int64_t min_free) {
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  int64_t *nstart = nullptr, *tmp_sums = nullptr, *total = nullptr;
  int32_t *ncol = nullptr;
  DAMF_HIP(hipMalloc(&nstart, n * sizeof(int64_t)));
  DAMF_HIP(hipMalloc(&tmp_sums, (ceil_div(n, 1024) + 1) * sizeof(int64_t)));
  DAMF_HIP(hipMalloc(&total, 2 * sizeof(int64_t)));
  DAMF_HIP(hipMemsetAsync(total + 1, 0, sizeof(int64_t), s));
  sum_len_kernel<<<stride_grid(n, 256), 256, 0, s>>>(n, g.len, total + 1);
  DAMF_HIP(exclusive_scan(CapOf{g.len}, n, nstart, tmp_sums, total, s));
  int64_t h[2] = {0, 0};
  DAMF_HIP(hipMemcpyAsync(h, total, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  const int64_t pool_used = h[0], nnz = h[1];
  const int64_t cap = std::max(pool_capacity(pool_used, nnz, slack), pool_used + min_free);
  DAMF_HIP(hipMalloc(&ncol, cap * sizeof(int32_t)));
  copy_rows_kernel<<<stride_grid(n, 4), 256, 0, s>>>(n, g.start, g.col, nstart, g.len, ncol);
  set_caps_kernel<<<stride_grid(n, 256), 256, 0, s>>>(n, g.len, g.cap);
  DAMF_HIP(hipGetLastError());
  DAMF_HIP(hipMemcpyAsync(g.start, nstart, n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  DAMF_HIP(hipMemcpyAsync(g.top, &h[0], sizeof(int64_t), hipMemcpyHostToDevice, s));
  DAMF_HIP(hipStreamSynchronize(s));
  (void)hipFree(g.col);
  g.col = ncol;
  g.pool_cap = cap;
  (void)hipFree(nstart);
  (void)hipFree(tmp_sums);
  (void)hipFree(total);
  return hipSuccess;
}

}  // namespace damf
