// state.hip -- small kernels on the embedding state: node queries
// (Sec. 4.6: X[u] = X_b[u] P_X at O(d^2) per node), identity projections,
// residual norms.
#include <hip/hip_runtime.h>

#include "common.h"
#include "damf_internal.h"

namespace damf {

// out[q][c] = sum_k M_b[node_q][k] P[k][c] * sqrt(sigma_c), FP64 accumulate.
// One wave per queried row; lanes own columns c = lane + 64 j.
__global__ __launch_bounds__(256) void query_kernel(const float *Mb, const double *P,
                                                    const double *sigma, int d, int64_t q,
                                                    const int32_t *nodes, float *out,
                                                    bool split) {
  __shared__ double row[4][kMaxD];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + w;
  if (i >= q) return;
  const int64_t node = nodes ? nodes[i] : i;
  for (int k = lane; k < d; k += 64) row[w][k] = (double)basis_ld(Mb, node * d + k, split);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int c = lane; c < d; c += 64) {
    double acc = 0.0;
    for (int k = 0; k < d; ++k) acc = fma(row[w][k], P[k * d + c], acc);
    out[i * d + c] = (float)(acc * sqrt(sigma[c]));
  }
}

hipError_t launch_query(damf_ctx *c, int which, int64_t q, const int32_t *d_nodes,
                        float *d_out) {
  const float *Mb = (which == DAMF_X) ? c->Ub : (which == DAMF_Y) ? c->Vb : c->Zb;
  const double *P = (which == DAMF_Y) ? c->P + (size_t)c->d * c->d : c->P;
  if (q <= 0) return hipSuccess;
  query_kernel<<<ceil_div(q, 4), 256, 0, c->stream>>>(Mb, P, c->sigma, c->d, q, d_nodes,
                                                       d_out, c->split && which != DAMF_Z);
  return hipGetLastError();
}

}  // namespace damf
