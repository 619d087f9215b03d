// rsvd.hip -- initial factorisation (Appendix A, Algorithm 3): randomized
// rank-d t-SVD of A with oversampling p and q power iterations, as cited by
// the paper (Halko, Martinsson, Tropp) for its O(n d^2 + m d) cost:
//
//   Omega[i, j] = +/-1 from SplitMix64,  Y = A Omega,  Q = qr(Y)
//   q times:  Q = qr(A^T Q),  Q = qr(A Q)
//   B^T = A^T Q = Q2 R2,   svd(R2^T) = Ut S Vt^T,
//   U = Q Ut[:, :d],  V = Q2 Vt[:, :d],  Sigma = S[:d]
//
// Kernels: sketch generation, CSR SpMM of width l = d + p (spmm.hip), tall-skinny
// Householder QR (recursive TSQR over blocks of 512 rows), an FP64 one-sided
// Jacobi SVD of the l x l factor in one workgroup, and the n x l by l x d
// rotation GEMM on MFMA (FP32 in, FP32 accumulate).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "damf_internal.h"
#include "jacobi.h"

namespace damf {

namespace {

// ---------------------------------------------------------------- sketch

__device__ __forceinline__ uint64_t splitmix64_out(uint64_t state) {
  // output of SplitMix64 whose state before the call is `state`
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void sketch_kernel(float *Om, int64_t n, int l, int ld, uint64_t seed) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * l;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / l;
    const int j = (int)(e - i * l);
    const uint64_t ctr = (seed << 40) ^ ((uint64_t)i * (uint64_t)l + (uint64_t)j);
    Om[i * ld + j] = (splitmix64_out(ctr) >> 63) ? -1.f : 1.f;
  }
}

// ---------------------------------------------------------------- TSQR
// Block of TB = 512 rows; the l <= 192 columns are spread over the 16 waves
// (column c lives in wave c % 16, slot c / 16); lane holds rows lane + 64 r.

constexpr int TB = 512;
constexpr int TNT = 1024;
constexpr int TW = 16;
constexpr int TCOLS = 12;  // ceil(192 / 16)
constexpr int TRPL = TB / 64;

// Householder reflector of x (rows >= j of one column held by a wave):
// beta = -sign(x_j) ||x||, v = (x - beta e_j) / (x_j - beta), tau = (beta - x_j) / beta.
// Writes v (v_j = 1, zeros above) to vbuf and tau to *tau_out; returns beta.
__device__ float house(float (&x)[TRPL], int j, int rows, float *vbuf, float *tau_out) {
  const int lane = threadIdx.x & 63;
  float s2 = 0.f, xj = 0.f;
#pragma unroll
  for (int r = 0; r < TRPL; ++r) {
    const int i = r * 64 + lane;
    if (i > j && i < rows) s2 = fmaf(x[r], x[r], s2);
    if (i == j) xj = x[r];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s2 += __shfl_xor(s2, off, 64);
    xj += __shfl_xor(xj, off, 64);
  }
  float beta, tau, scale;
  if (s2 == 0.f) {
    beta = xj;
    tau = 0.f;
    scale = 0.f;
  } else {
    const float nrm = sqrtf(xj * xj + s2);
    beta = (xj >= 0.f) ? -nrm : nrm;
    tau = (beta - xj) / beta;
    scale = 1.f / (xj - beta);
  }
#pragma unroll
  for (int r = 0; r < TRPL; ++r) {
    const int i = r * 64 + lane;
    float v = 0.f;
    if (i == j) v = 1.f;
    else if (i > j && i < rows) v = x[r] * scale;
    vbuf[i] = v;
  }
  if (lane == 0) *tau_out = tau;
  return beta;
}

// Factor one block: V (reflectors) overwrites the block in place, tau[l] per
// block, R (l x l, upper) written to S rows [blk * l, (blk + 1) * l).
__global__ __launch_bounds__(TNT) void tsqr_factor_kernel(float *A, int64_t m, int l, int ld,
                                                          float *tau_all, float *S) {
  __shared__ float vbuf[2][TB];
  __shared__ float taus[2];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = (int64_t)blockIdx.x * TB;
  const int rows = (int)min<int64_t>(TB, m - r0);
  float x[TCOLS][TRPL];
#pragma unroll
  for (int s = 0; s < TCOLS; ++s) {
    const int c = s * TW + w;
#pragma unroll
    for (int r = 0; r < TRPL; ++r) {
      const int i = r * 64 + lane;
      x[s][r] = (c < l && i < rows) ? A[(r0 + i) * ld + c] : 0.f;
    }
  }
  for (int j = 0; j < l; ++j) {
    const int par = j & 1;
    const int owner = j % TW, slot = j / TW;
    if (w == owner) {
#pragma unroll
      for (int s = 0; s < TCOLS; ++s) {
        if (s == slot) {
          const float beta = house(x[s], j, TB, vbuf[par], &taus[par]);
          // the column becomes (beta at row j, v below): keep v below j, R above
#pragma unroll
          for (int r = 0; r < TRPL; ++r) {
            const int i = r * 64 + lane;
            if (i == j) x[s][r] = beta;
            else if (i > j) x[s][r] = vbuf[par][i];
          }
        }
      }
    }
    __syncthreads();
    const float tau = taus[par];
    if (tau != 0.f) {
#pragma unroll
      for (int s = 0; s < TCOLS; ++s) {
        const int c = s * TW + w;
        if (c > j && c < l) {
          float p = 0.f;
#pragma unroll
          for (int r = 0; r < TRPL; ++r) p = fmaf(vbuf[par][r * 64 + lane], x[s][r], p);
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) p += __shfl_xor(p, off, 64);
          const float tw = tau * p;
#pragma unroll
          for (int r = 0; r < TRPL; ++r) x[s][r] = fmaf(-tw, vbuf[par][r * 64 + lane], x[s][r]);
        }
      }
    }
    if (threadIdx.x == 0) tau_all[(int64_t)blockIdx.x * l + j] = tau;
  }
  // write back: reflectors below the diagonal, R to S
#pragma unroll
  for (int s = 0; s < TCOLS; ++s) {
    const int c = s * TW + w;
    if (c < l) {
#pragma unroll
      for (int r = 0; r < TRPL; ++r) {
        const int i = r * 64 + lane;
        if (i < rows) A[(r0 + i) * ld + c] = x[s][r];
        if (i < l) S[((int64_t)blockIdx.x * l + i) * l + c] = (i <= c) ? x[s][r] : 0.f;
      }
    }
  }
}

// Form the explicit Q of one block: X = [C; 0] with C the block's l x l slab
// of the next level's Q (or I at the top), then X <- H_0 ... H_{l-1} X.
// Overwrites the block (which held the reflectors) with Q.
__global__ __launch_bounds__(TNT) void tsqr_formq_kernel(float *A, int64_t m, int l, int ld,
                                                         const float *tau_all, const float *QS) {
  __shared__ float vb[2][TB];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = (int64_t)blockIdx.x * TB;
  const int rows = (int)min<int64_t>(TB, m - r0);
  float x[TCOLS][TRPL];
#pragma unroll
  for (int s = 0; s < TCOLS; ++s) {
    const int c = s * TW + w;
#pragma unroll
    for (int r = 0; r < TRPL; ++r) {
      const int i = r * 64 + lane;
      float v = 0.f;
      if (c < l && i < l) v = QS ? QS[((int64_t)blockIdx.x * l + i) * l + c] : (i == c ? 1.f : 0.f);
      x[s][r] = v;
    }
  }
  for (int j = l - 1; j >= 0; --j) {
    const int par = j & 1;
    for (int i = threadIdx.x; i < TB; i += TNT) {
      float v = 0.f;
      if (i == j) v = 1.f;
      else if (i > j && i < rows) v = A[(r0 + i) * ld + j];
      vb[par][i] = v;
    }
    __syncthreads();
    const float tau = tau_all[(int64_t)blockIdx.x * l + j];
    if (tau != 0.f) {
#pragma unroll
      for (int s = 0; s < TCOLS; ++s) {
        const int c = s * TW + w;
        if (c < l) {
          float p = 0.f;
#pragma unroll
          for (int r = 0; r < TRPL; ++r) p = fmaf(vb[par][r * 64 + lane], x[s][r], p);
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) p += __shfl_xor(p, off, 64);
          const float tw = tau * p;
#pragma unroll
          for (int r = 0; r < TRPL; ++r) x[s][r] = fmaf(-tw, vb[par][r * 64 + lane], x[s][r]);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < TCOLS; ++s) {
    const int c = s * TW + w;
    if (c < l) {
#pragma unroll
      for (int r = 0; r < TRPL; ++r) {
        const int i = r * 64 + lane;
        if (i < rows) A[(r0 + i) * ld + c] = x[s][r];
      }
    }
  }
}

// ---------------------------------------------------------------- small SVD

// Orthonormal completion, by one wave, of the columns c of M (l x d,
// row-major, l <= 192) whose singular value sv[c] is <= cut: unit vectors
// e_q, q = 0, 1, ..., are orthogonalised (two Gram-Schmidt passes) against
// the kept columns and the completed ones before c, and the first with at
// least a quarter of its norm left is taken.
__device__ void complete_columns(double *M, int l, int d, const double *sv, double cut) {
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < d; ++c) {
    if (sv[c] > cut) continue;
    for (int q = 0; q < l; ++q) {
      double v[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) v[r] = (r * 64 + lane == q) ? 1.0 : 0.0;
      for (int pass = 0; pass < 2; ++pass) {
        for (int o = 0; o < d; ++o) {
          if (o == c || (sv[o] <= cut && o > c)) continue;
          double dot = 0.0;
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const int i = r * 64 + lane;
            if (i < l) dot = fma(M[i * d + o], v[r], dot);
          }
          dot = wave_sum(dot);
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const int i = r * 64 + lane;
            if (i < l) v[r] = fma(-dot, M[i * d + o], v[r]);
          }
        }
      }
      double nn = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r)
        if (r * 64 + lane < l) nn = fma(v[r], v[r], nn);
      nn = wave_sum(nn);
      if (nn > 0.25) {
        const double inv = 1.0 / sqrt(nn);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const int i = r * 64 + lane;
          if (i < l) M[i * d + c] = v[r] * inv;
        }
        break;
      }
    }
  }
}
// FP64 one-sided Jacobi SVD of M (l x l, row-major FP32 upper-triangular R
// given; the kernel factors M = R^T).  Outputs the top d left vectors E
// (l x d), singular values and right vectors H = M^T E Theta^-1 (l x d),
// all float64, row-major.
__global__ __launch_bounds__(1024) void small_svd_kernel(const float *Rtop, int l, int d,
                                                         double *E, double *theta, double *H) {
  constexpr int RPL = 3, NW = 16;
  using SH = JacobiShape<RPL, NW>;
  constexpr int NP = SH::NP, CPW = SH::CPW;
  __shared__ double lds[SH::LDS];
  __shared__ double sv[256];
  __shared__ int sid[256], rank_of[256];
  __shared__ int flag;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  JacobiRegs<RPL, NW> J;
  // M = R^T: M[i][j] = R[j][i]
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = jacobi_slot_col<RPL, NW>(w, c);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = r * 64 + lane;
      J.a[c][r] = (i < l && j < l) ? (double)Rtop[j * l + i] : 0.0;
    }
  }
  jacobi_sweeps<RPL, NW>(J, lds, &flag, 40, 1e-12);
  const double *nrm = lds + 4 * NW * SH::SLOT;
  // a NaN or infinite norm gets the key -0.5: after every finite value and
  // before the -1 padding, so the sort is a total order and every real
  // column ranks below NP (theta < 0 then reports the failure)
  for (int j = threadIdx.x; j < 256; j += 1024) {
    const double v = (j < NP) ? sqrt(nrm[j]) : -1.0;
    sv[j] = (j >= NP || v <= DBL_MAX) ? v : -0.5;
    sid[j] = j;
  }
  __syncthreads();
  for (int kk = 2; kk <= 256; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      if (threadIdx.x < 256) {
        int i = threadIdx.x, q = i ^ jj;
        if (q > i) {
          double a = sv[i], b = sv[q];
          int ia = sid[i], ib = sid[q];
          bool before = (a > b) || (a == b && ia < ib);
          bool up = (i & kk) == 0;
          if (before != up) {
            sv[i] = b;
            sv[q] = a;
            sid[i] = ib;
            sid[q] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x < NP) rank_of[sid[threadIdx.x]] = threadIdx.x;
  if (threadIdx.x < d) theta[threadIdx.x] = sv[threadIdx.x];
  __syncthreads();
  const double cut = 1e-12 * sv[0];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = jacobi_slot_col<RPL, NW>(w, c);
    const int rk = rank_of[j];
    if (rk < d) {
      const double inv = (sv[rk] > cut) ? 1.0 / sv[rk] : 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = r * 64 + lane;
        if (i < l) E[i * d + rk] = J.a[c][r] * inv;
      }
    }
  }
  __syncthreads();
  // H[j][c] = sum_i M[i][j] E[i][c] / theta_c = sum_i R[j][i] E[i][c] / theta_c
  for (int e = threadIdx.x; e < l * d; e += 1024) {
    const int j = e / d, c = e - j * d;
    double acc = 0.0;
    for (int i = 0; i < l; ++i) acc = fma((double)Rtop[j * l + i], E[i * d + c], acc);
    H[j * d + c] = (sv[c] > cut) ? acc / sv[c] : 0.0;
  }
  __syncthreads();
  // rank(A) < d leaves columns with theta <= cut: complete E and H to
  // orthonormal columns so that U = Q E and V = Q2 H stay orthonormal
  if (threadIdx.x < 64 && sv[d - 1] <= cut) {
    complete_columns(E, l, d, sv, cut);
    complete_columns(H, l, d, sv, cut);
  }
}

// ---------------------------------------------------------------- GEMM
// C (n x d, ldc) = A (n x l, lda) * B (l x d, row-major, FP32) on MFMA
// (v_mfma_f32_16x16x4f32).  Workgroup: 64 rows x 128 cols; 4 waves, each 16
// rows x 128 cols = 8 MFMA tiles.  A and B tiles staged in LDS.
constexpr int GM = 64;
constexpr int GK = 16;

typedef float v4f __attribute__((ext_vector_type(4)));

// C (n x d) = A (n x l) B (l x d), d <= 16 TL.  C may be A itself (lda == ldc):
// each workgroup owns whole rows and has read all of them before it writes.
template <int TL>
__global__ __launch_bounds__(256) void gemm_tall_kernel(const float *A, int64_t n, int l, int lda,
                                                        const float *__restrict__ B, int d,
                                                        float *C, int ldc) {
  constexpr int BW = 16 * TL;
  __shared__ float As[GM][GK + 1];
  __shared__ float Bs[GK][BW + 4];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  // row blocks in a grid-stride loop (workgroup-uniform, so barriers align)
  for (int64_t row0 = (int64_t)blockIdx.x * GM; row0 < n; row0 += (int64_t)gridDim.x * GM) {
    v4f acc[TL];
#pragma unroll
    for (int t = 0; t < TL; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < l; k0 += GK) {
      for (int e = threadIdx.x; e < GM * GK; e += 256) {
        const int i = e / GK, k = e - i * GK;
        const int64_t r = row0 + i;
        As[i][k] = (r < n && k0 + k < l) ? A[r * lda + k0 + k] : 0.f;
      }
      for (int e = threadIdx.x; e < GK * BW; e += 256) {
        const int k = e / BW, j = e - k * BW;
        Bs[k][j] = (k0 + k < l && j < d) ? B[(k0 + k) * d + j] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < GK; kk += 4) {
        const float a = As[w * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int t = 0; t < TL; ++t) {
          const float b = Bs[kk + (lane >> 4)][t * 16 + (lane & 15)];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < TL; ++t) {
      const int j = t * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = row0 + w * 16 + (lane >> 4) * 4 + q;
        if (r < n && j < d) C[r * ldc + j] = acc[t][q];
      }
    }
  }
}

// The same product with B resident in LDS, for d <= 16 TL and l <= 192: one
// workgroup of NWV waves per CU (B takes up to 111 KB) strides over blocks
// of 16 NWV rows, so B is read from L2 once per workgroup instead of once
// per 64 rows.  A moves through a double-buffered LDS tile GK2 wide, the
// next tile loaded into registers while the current one is multiplied, one
// barrier per k step.  Each wave owns 16 rows of a block and all 16 TL
// columns.  Launched with 16 waves and GK2 = 16 (4 waves per SIMD, 148 KB
// of LDS at TL = 9); 8 waves with GK2 = 32 ran 6% slower.
constexpr int kTallLmax = 192;
template <int TL, int NWV, int GK2>
__global__ __launch_bounds__(64 * NWV) void gemm_tall_res_kernel(const float *A, int64_t n, int l, int lda,
                                                            const float *__restrict__ B, int d,
                                                            float *C, int ldc) {
  constexpr int BW = 16 * TL;
  constexpr int GM2 = 16 * NWV;  // rows per block
  constexpr int NTH = 64 * NWV;
  __shared__ float Bs[kTallLmax][BW + 4];
  __shared__ float As[2][GM2][GK2 + 1];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < kTallLmax * BW; e += NTH) {
    const int k = e / BW, j = e - k * BW;
    Bs[k][j] = (k < l && j < d) ? B[(int64_t)k * d + j] : 0.f;
  }
  constexpr int PER = GM2 * GK2 / NTH;  // A values per thread per tile
  const int nk = (l + GK2 - 1) / GK2;
  float pre[PER];
  auto fetch = [&](int64_t r0, int k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * NTH;
      const int i = e / GK2, k = e - i * GK2;
      const int64_t r = r0 + i;
      pre[q] = (r < n && k0 + k < l) ? A[r * lda + k0 + k] : 0.f;
    }
  };
  const int64_t step = (int64_t)gridDim.x * GM2;
  int buf = 0;
  fetch((int64_t)blockIdx.x * GM2, 0);
  for (int64_t row0 = (int64_t)blockIdx.x * GM2; row0 < n; row0 += step) {
    v4f acc[TL];
#pragma unroll
    for (int t = 0; t < TL; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * NTH;
        As[buf][e / GK2][e - (e / GK2) * GK2] = pre[q];
      }
      // B written (first pass); the tile in As[buf] complete; every wave is
      // past its reads of As[buf] from two k steps back
      __syncthreads();
      if (kt + 1 < nk)
        fetch(row0, (kt + 1) * GK2);
      else if (row0 + step < n)
        fetch(row0 + step, 0);
      const int k0 = kt * GK2;
#pragma unroll
      for (int kk = 0; kk < GK2; kk += 4) {
        if (k0 + kk >= l) break;
        const float a = As[buf][w * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int t = 0; t < TL; ++t) {
          const float b = Bs[k0 + kk + (lane >> 4)][t * 16 + (lane & 15)];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
        }
      }
      buf ^= 1;
    }
    // the whole block's rows were read by this workgroup before these stores
#pragma unroll
    for (int t = 0; t < TL; ++t) {
      const int j = t * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = row0 + w * 16 + (lane >> 4) * 4 + q;
        if (r < n && j < d) C[r * ldc + j] = acc[t][q];
      }
    }
  }
}

// ---------------------------------------------------------------- CholeskyQR2
// Tall-skinny QR of Y (m x l, l <= 192) as two CholeskyQR passes: the Gram
// G = Y^T Y in FP64 (one read of Y), G = R^T R by Cholesky in FP64, then
// Y <- Y R^-1 on FP32 MFMA in place (one read and write); the second pass
// restores the orthogonality the first loses to FP32 rounding, and the R
// factor is R2 R1.  A first Gram whose pivots fall below 1e-10 of its largest
// diagonal (Y numerically rank deficient, or cond(Y) above ~1e5) sends the
// QR to the Householder TSQR above instead.

constexpr int LM = kMaxCore;     // widest sketch, d + p <= 192
constexpr int kCqrParts = 256;   // workgroups of a Gram pass
constexpr double kCqrPivot = 1e-10;

// Partial Grams on FP64 MFMA (v_mfma_f64_16x16x4 f64): workgroup b sums
// its share of the rows into part[b] (LM x LM, upper-triangle 16 x 16 tiles
// only; the reduction mirrors them).  The tiles I <= J are dealt to the 8
// waves in turn, so every SIMD carries about the same number; each MFMA
// takes four rows of Y, converted to FP64 from a 64-row LDS tile, and the
// next 64 rows are loaded into registers while the current ones are used.
typedef double v4f64 __attribute__((ext_vector_type(4)));
constexpr int kGramSlots = (12 * 13 / 2 + 7) / 8;  // tiles per wave at l = 192
__global__ __launch_bounds__(512) void cqr_gram_kernel(const float *Y, int64_t m, int l, int ld,
                                                       double *part) {
  __shared__ float tile[64][LM + 4];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int nt = (l + 15) >> 4;           // 16-wide column tiles
  const int ntiles = nt * (nt + 1) / 2;   // tiles with I <= J
  int ti[kGramSlots], tj[kGramSlots];
#pragma unroll
  for (int q = 0; q < kGramSlots; ++q) {
    int u = w + 8 * q, I = 0;
#pragma unroll
    for (int t = 0; t < 12; ++t) {  // row I of the triangle holds nt - I tiles
      const bool past = I < nt && u >= nt - I;
      u -= past ? nt - I : 0;
      I += past ? 1 : 0;
    }
    // slots past the last tile (I == nt) read tile nt - 1 and are not used
    ti[q] = min(I, nt - 1);
    tj[q] = min(I + u, nt - 1);
  }
  const int nslot = (ntiles - w + 7) / 8;  // slots q with w + 8 q < ntiles
  v4f64 acc[kGramSlots];
#pragma unroll
  for (int q = 0; q < kGramSlots; ++q) acc[q] = v4f64{0.0, 0.0, 0.0, 0.0};
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = min<int64_t>(m, r0 + per);
  // tile loads: thread t moves columns t % 64 + 64 j (j < 3) of rows
  // t / 64 + 8 i (i < 8)
  const int fc = threadIdx.x & 63, fr = threadIdx.x >> 6;
  bool col_in[LM / 64];
#pragma unroll
  for (int j = 0; j < LM / 64; ++j) col_in[j] = fc + 64 * j < l;
  float pre[8][LM / 64];
  auto fetch = [&](int64_t base) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t r = base + fr + 8 * i;
      const float *row = Y + r * ld + fc;
#pragma unroll
      for (int j = 0; j < LM / 64; ++j) pre[i][j] = (r < r1 && col_in[j]) ? row[64 * j] : 0.f;
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t base = r0; base < r1; base += 64) {
    __syncthreads();  // every wave is done with the previous rows
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < LM / 64; ++j) tile[fr + 8 * i][fc + 64 * j] = pre[i][j];
    __syncthreads();
    if (base + 64 < r1) fetch(base + 64);
#pragma unroll 1
    for (int k = 0; k < 64; k += 4) {
      const int rr = k + (lane >> 4);
      float a[kGramSlots], b[kGramSlots];  // all reads first, one wait
#pragma unroll
      for (int q = 0; q < kGramSlots; ++q) {
        a[q] = tile[rr][16 * ti[q] + (lane & 15)];
        b[q] = tile[rr][16 * tj[q] + (lane & 15)];
      }
#pragma unroll
      for (int q = 0; q < kGramSlots; ++q)
        if (q < nslot)
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[q], (double)b[q], acc[q], 0, 0, 0);
    }
  }
  // output layout of the FP64 16 x 16 x 4 MFMA: register v of lane group g
  // (lanes 16 g .. 16 g + 15) holds row 4 v + g, column lane % 16
  double *out = part + (size_t)blockIdx.x * LM * LM;
#pragma unroll
  for (int q = 0; q < kGramSlots; ++q) {
    if (q < nslot) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(16 * ti[q] + 4 * v + (lane >> 4)) * LM + 16 * tj[q] + (lane & 15)] = acc[q][v];
    }
  }
}

// G[i][j] = sum over the parts (i, j < l), row stride LM; the parts hold the
// upper triangle (i <= j).
__global__ void cqr_reduce_kernel(const double *part, int nparts, int l, double *G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= l * l) return;
  const int i = e / l, j = e - i * l;
  const int src = (i <= j) ? i * LM + j : j * LM + i;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(size_t)b * LM * LM + src];
  G[i * LM + j] = s;
}

// One workgroup: G = R^T R (right-looking, upper R in G's upper triangle,
// FP64), then Rinv = R^-1 (upper) written as FP32 l x l row-major for the
// MFMA product, R kept in FP64 (stride LM).  *bad = 1 on a pivot below
// kCqrPivot times the largest diagonal entry (or not finite).
__global__ __launch_bounds__(1024) void cqr_chol_kernel(double *G, int l, double *R, float *Rinv,
                                                        int *bad) {
  __shared__ double dmax;
  __shared__ int s_bad;
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int i = 0; i < l; ++i) mx = fmax(mx, G[i * LM + i]);
    dmax = mx;
    s_bad = 0;
  }
  __syncthreads();
  for (int j = 0; j < l; ++j) {
    const double piv = G[j * LM + j];
    if (!(piv > kCqrPivot * dmax)) {
      if (threadIdx.x == 0) s_bad = 1;
      break;  // uniform: every thread read the same pivot
    }
    const double rjj = sqrt(piv), inv = 1.0 / rjj;
    __syncthreads();
    for (int c = j + threadIdx.x; c < l; c += 1024) G[j * LM + c] = (c == j) ? rjj : G[j * LM + c] * inv;
    __syncthreads();
    // trailing update of the upper triangle: G[i][c] -= R[j][i] R[j][c], j < i <= c
    const int t = l - j - 1;
    for (int e = threadIdx.x; e < t * t; e += 1024) {
      const int i = j + 1 + e / t, c = j + 1 + e % t;
      if (c >= i) G[i * LM + c] = fma(-G[j * LM + i], G[j * LM + c], G[i * LM + c]);
    }
    __syncthreads();
  }
  __syncthreads();
  if (s_bad) {
    if (threadIdx.x == 0) *bad = 1;
    return;
  }
  // R (upper, zeros below) and its inverse, one column per thread
  for (int e = threadIdx.x; e < l * l; e += 1024) {
    const int i = e / l, c = e - i * l;
    R[i * LM + c] = (c >= i) ? G[i * LM + c] : 0.0;
  }
  __syncthreads();
  // X = R^-1 by columns, one thread per column c, in G's space (row c of G
  // holds column c of X): X[c][c] = 1 / R[c][c],
  // X[i][c] = -(sum_{k=i+1..c} R[i][k] X[k][c]) / R[i][i] for i < c
  for (int c = threadIdx.x; c < l; c += 1024) {
    double *x = G + c * LM;
    for (int i = 0; i < l; ++i) x[i] = 0.0;
    x[c] = 1.0 / R[c * LM + c];
    for (int i = c - 1; i >= 0; --i) {
      double sacc = 0.0;
      for (int k = i + 1; k <= c; ++k) sacc = fma(R[i * LM + k], x[k], sacc);
      x[i] = -sacc / R[i * LM + i];
    }
    for (int i = 0; i < l; ++i) Rinv[i * l + c] = (float)x[i];
  }
  if (threadIdx.x == 0) *bad = 0;
}

// Rtop (FP32, l x l row-major) = R2 R1 (both upper, FP64, stride LM).
__global__ void cqr_rprod_kernel(const double *R2, const double *R1, int l, float *Rtop) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= l * l) return;
  const int i = e / l, c = e - i * l;
  double s = 0.0;
  for (int k = i; k <= c; ++k) s = fma(R2[i * LM + k], R1[k * LM + c], s);
  Rtop[e] = (c >= i) ? (float)s : 0.f;
}

__global__ void encode_kernel(float *M, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    M[i] = __uint_as_float(split_encode(M[i]));
}

__global__ void to_float_kernel(const double *x, float *y, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = (float)x[i];
}

// ---------------------------------------------------------------- driver

struct Tsqr {
  std::vector<float *> S;    // stacked R per level
  std::vector<float *> tau;  // per level
  std::vector<int64_t> m;    // rows per level
};

// In-place QR of A (m x l): A <- Q.  Rtop receives the final R (l x l).
hipError_t tsqr(float *A, int64_t m, int l, int ld, float *Rtop, hipStream_t s) {
  // levels: level 0 is A itself
  std::vector<float *> mats{A};
  std::vector<int64_t> rows{m};
  std::vector<int> lds{ld};
  std::vector<float *> taus;
  hipError_t err = hipSuccess;
  // each level has at most ceil(m / TB) * l <= 0.375 m + l rows, so the stack
  // of R factors shrinks until it fits one block
  while (true) {
    if (mats.size() > 64) {
      err = hipErrorInvalidValue;
      break;
    }
    const int64_t mm = rows.back();
    const int64_t nb = (mm + TB - 1) / TB;
    float *tau = nullptr, *S = nullptr;
    if ((err = hipMalloc(&tau, nb * l * sizeof(float))) != hipSuccess) break;
    if ((err = hipMalloc(&S, nb * l * (int64_t)l * sizeof(float))) != hipSuccess) break;
    taus.push_back(tau);
    static_assert(TB == 512 && TNT == 1024, "geom_tsqr assumes 512-row blocks of 1024 threads");
    tsqr_factor_kernel<<<geom_tsqr(mm).blocks, TNT, 0, s>>>(mats.back(), mm, l, lds.back(), tau, S);
    if ((err = hipGetLastError()) != hipSuccess) break;
    if (nb == 1) {
      // S holds the final R
      err = hipMemcpyAsync(Rtop, S, (size_t)l * l * sizeof(float), hipMemcpyDeviceToDevice, s);
      (void)hipStreamSynchronize(s);
      (void)hipFree(S);
      break;
    }
    mats.push_back(S);
    rows.push_back(nb * l);
    lds.push_back(l);
  }
  if (err == hipSuccess) {
    // form Q top-down: level L-1 from I, then each lower level from the next
    const int levels = (int)mats.size();
    for (int lev = levels - 1; lev >= 0; --lev) {
      const int64_t mm = rows[lev];
      const int64_t nb = (mm + TB - 1) / TB;
      const float *QS = (lev == levels - 1) ? nullptr : mats[lev + 1];
      tsqr_formq_kernel<<<geom_tsqr(mm).blocks, TNT, 0, s>>>(mats[lev], mm, l, lds[lev], taus[lev], QS);
      if ((err = hipGetLastError()) != hipSuccess) break;
    }
  }
  (void)hipStreamSynchronize(s);
  for (size_t i = 1; i < mats.size(); ++i) (void)hipFree(mats[i]);
  for (float *t : taus) (void)hipFree(t);
  return err;
}

}  // namespace

hipError_t gemm_tall(const float *A, int64_t n, int l, int lda, const float *B, int d, float *C,
                     int ldc, hipStream_t s) {
  if (l < 1 || l > kTallLmax || n < 1) return hipErrorInvalidValue;
  // one workgroup per CU, B resident; at most as many as there are row blocks
  constexpr int NWV = 16, GK2 = 16;
  static_assert(64 * NWV == 1024 && 16 * NWV == 256, "geom_gemm_tall_res assumes 16 waves");
  const Grid g = geom_gemm_tall_res(n);
  const Grid g12 = geom_gemm_tall(n);
  if (d <= 128)
    gemm_tall_res_kernel<8, NWV, GK2><<<g.blocks, g.threads, 0, s>>>(A, n, l, lda, B, d, C, ldc);
  else if (d <= 144)  // d + p = 138 at d = 128: nine column tiles, not twelve
    gemm_tall_res_kernel<9, NWV, GK2><<<g.blocks, g.threads, 0, s>>>(A, n, l, lda, B, d, C, ldc);
  else if (d <= 192)
    gemm_tall_kernel<12><<<g12.blocks, g12.threads, 0, s>>>(A, n, l, lda, B, d, C, ldc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

namespace {

// CholeskyQR2 of Y in place (Rtop = R2 R1); the Householder TSQR when the
// first Gram is not clearly positive definite.
hipError_t tall_qr(float *Y, int64_t m, int l, int ld, float *Rtop, hipStream_t s,
                   int64_t *fallbacks) {
  if (l > LM) return hipErrorInvalidValue;
  const int nparts = (int)std::min<int64_t>(kCqrParts, (m + 63) / 64);
  double *part = nullptr, *G = nullptr, *R1 = nullptr, *R2 = nullptr;
  float *Rinv = nullptr;
  int *bad = nullptr;
  int hbad = 0;
  hipError_t err = hipSuccess;
  auto pass = [&](double *R) -> hipError_t {
    cqr_gram_kernel<<<nparts, 512, 0, s>>>(Y, m, l, ld, part);
    cqr_reduce_kernel<<<ceil_div((int64_t)l * l, 256), 256, 0, s>>>(part, nparts, l, G);
    cqr_chol_kernel<<<1, 1024, 0, s>>>(G, l, R, Rinv, bad);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || hbad) return e;
    return gemm_tall(Y, m, l, ld, Rinv, l, Y, ld, s);
  };
  if ((err = hipMalloc(&part, (size_t)nparts * LM * LM * sizeof(double))) == hipSuccess &&
      (err = hipMalloc(&G, (size_t)LM * LM * sizeof(double))) == hipSuccess &&
      (err = hipMalloc(&R1, (size_t)LM * LM * sizeof(double))) == hipSuccess &&
      (err = hipMalloc(&R2, (size_t)LM * LM * sizeof(double))) == hipSuccess &&
      (err = hipMalloc(&Rinv, (size_t)l * l * sizeof(float))) == hipSuccess &&
      (err = hipMalloc(&bad, sizeof(int))) == hipSuccess) {
    err = pass(R1);
    if (err == hipSuccess && hbad) {
      ++*fallbacks;
      err = tsqr(Y, m, l, ld, Rtop, s);  // Y untouched by the failed pass
    } else if (err == hipSuccess) {
      err = pass(R2);
      if (err == hipSuccess && hbad) err = hipErrorInvalidValue;  // Q1 not finite
      if (err == hipSuccess) {
        cqr_rprod_kernel<<<ceil_div((int64_t)l * l, 256), 256, 0, s>>>(R2, R1, l, Rtop);
        err = hipGetLastError();
      }
    }
  }
  (void)hipStreamSynchronize(s);
  for (void *q : {(void *)part, (void *)G, (void *)R1, (void *)R2, (void *)Rinv, (void *)bad})
    if (q) (void)hipFree(q);
  return err;
}

}  // namespace

hipError_t rsvd_init(damf_ctx *c) {
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  const int d = c->d;
  const int l = d + c->cfg.oversample;
  const int ld = l;
  float *Y = nullptr, *T = nullptr, *Rt = nullptr, *Ef = nullptr, *Hf = nullptr;
  double *E = nullptr, *H = nullptr, *th = nullptr;
  DAMF_HIP(hipMalloc(&Y, (size_t)n * ld * sizeof(float)));
  DAMF_HIP(hipMalloc(&T, (size_t)n * ld * sizeof(float)));
  DAMF_HIP(hipMalloc(&Rt, (size_t)l * l * sizeof(float)));
  DAMF_HIP(hipMalloc(&E, (size_t)l * d * sizeof(double)));
  DAMF_HIP(hipMalloc(&H, (size_t)l * d * sizeof(double)));
  DAMF_HIP(hipMalloc(&th, (size_t)kMaxCore * sizeof(double)));
  DAMF_HIP(hipMalloc(&Ef, (size_t)l * d * sizeof(float)));
  DAMF_HIP(hipMalloc(&Hf, (size_t)l * d * sizeof(float)));
  sketch_kernel<<<stride_grid(n * l, 256), 256, 0, s>>>(T, n, l, ld, c->cfg.seed);
  DAMF_HIP(hipGetLastError());
  SpmmPlan pout, pin;
  DAMF_HIP(spmm_plan_build(c, c->out, ld, &pout));
  DAMF_HIP(spmm_plan_build(c, c->in, ld, &pin));
  DAMF_HIP(csr_spmm(c->out, pout, T, Y, n, l, ld, s));  // Y = A Omega
  DAMF_HIP(tall_qr(Y, n, l, ld, Rt, s, &c->init_info.qr_fallbacks));
  for (int it = 0; it < c->cfg.power_iters; ++it) {
    DAMF_HIP(csr_spmm(c->in, pin, Y, T, n, l, ld, s));  // A^T Q
    DAMF_HIP(tall_qr(T, n, l, ld, Rt, s, &c->init_info.qr_fallbacks));
    DAMF_HIP(csr_spmm(c->out, pout, T, Y, n, l, ld, s));  // A Q
    DAMF_HIP(tall_qr(Y, n, l, ld, Rt, s, &c->init_info.qr_fallbacks));
  }
  DAMF_HIP(csr_spmm(c->in, pin, Y, T, n, l, ld, s));  // B^T = A^T Q
  DAMF_HIP(hipStreamSynchronize(s));
  spmm_plan_free(pout);
  spmm_plan_free(pin);
  DAMF_HIP(tall_qr(T, n, l, ld, Rt, s, &c->init_info.qr_fallbacks));     // T = Q2, Rt = R2
  small_svd_kernel<<<1, 1024, 0, s>>>(Rt, l, d, E, th, H);
  DAMF_HIP(hipGetLastError());
  to_float_kernel<<<ceil_div((int64_t)l * d, 256), 256, 0, s>>>(E, Ef, (int64_t)l * d);
  to_float_kernel<<<ceil_div((int64_t)l * d, 256), 256, 0, s>>>(H, Hf, (int64_t)l * d);
  DAMF_HIP(gemm_tall(Y, n, l, ld, Ef, d, c->Ub, d, s));  // U = Q Ut_d
  DAMF_HIP(gemm_tall(T, n, l, ld, Hf, d, c->Vb, d, s));  // V = Q2 Vt_d
  if (c->split) {  // precision form: store the bases as BF16 pairs
    encode_kernel<<<stride_grid((int64_t)n * d, 256), 256, 0, s>>>(c->Ub, (int64_t)n * d);
    encode_kernel<<<stride_grid((int64_t)n * d, 256), 256, 0, s>>>(c->Vb, (int64_t)n * d);
    DAMF_HIP(hipGetLastError());
  }
  // projections = I, Sigma
  std::vector<double> P(2 * (size_t)d * d, 0.0);
  for (int sd = 0; sd < 2; ++sd)
    for (int i = 0; i < d; ++i) P[sd * d * d + i * d + i] = 1.0;
  DAMF_HIP(hipMemcpyAsync(c->P, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice, s));
  DAMF_HIP(hipMemsetAsync(c->sigma, 0, kMaxCore * sizeof(double), s));
  DAMF_HIP(hipMemcpyAsync(c->sigma, th, d * sizeof(double), hipMemcpyDeviceToDevice, s));
  std::vector<double> th_host(d);
  DAMF_HIP(hipMemcpyAsync(th_host.data(), th, d * sizeof(double), hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  for (double t : th_host)  // NaN or Inf anywhere upstream ends as theta < 0 or non-finite
    if (!(t >= 0.0 && t <= DBL_MAX)) c->nonfinite = true;
  (void)hipFree(Y);
  (void)hipFree(T);
  (void)hipFree(Rt);
  (void)hipFree(E);
  (void)hipFree(H);
  (void)hipFree(th);
  (void)hipFree(Ef);
  (void)hipFree(Hf);
  return hipSuccess;
}

}  // namespace damf
