// reorth.hip -- flush of the lazy projections and FP64 re-orthogonalisation.
//
// The lazy base space (Sec. 4.1, the lazy update equation) keeps
// U = U_b P_U and V = V_b P_V; every chunk multiplies its rotation F into P
// (Step 3, Sec. 4.5).  A flush applies the projections to the bases:
//     U_b <- U_b P_U,  Z_b <- Z_b P_U,  R <- R P_U,  V_b <- V_b P_V,  P <- I.
// Z_b and R follow U_b because PPR acts on the left, so PPR(U_b P) =
// PPR(U_b) P and the push invariant PPR(U_b) = Z_b + Pi R is kept.
//
// Re-orthogonalisation restores U^T U = V^T V = I, which rounding in the FP32
// bases erodes over many chunks, without changing the product U Sigma V^T:
//     G_U = U^T U = P_U^T (U_b^T U_b) P_U = R_U^T R_U    (FP64 Gram, Cholesky)
//     R_U Sigma R_V^T = Ut S Vt^T                         (FP64 Jacobi SVD)
//     U <- U R_U^-1 Ut,  V <- V R_V^-1 Vt,  Sigma <- S,  P <- I.
// (CholeskyQR of U and V, then the t-SVD of the d x d core.)  The whole
// change of U_b is the single d x d matrix P_U R_U^-1 Ut, so the bases are
// read once for the Grams and rewritten once by the MFMA rotation.
#include <hip/hip_runtime.h>

#include "common.h"
#include "damf_internal.h"
#include "jacobi.h"

namespace damf {

namespace {

constexpr int DM = kMaxD;
constexpr int kGramParts = 256;     // workgroups of the Gram pass (one per CU)
constexpr double kMinPivot = 0.25;  // G must be near I: pivots of R_U^T R_U

// Partial Grams in FP64: workgroup b sums M[r]^T M[r] over its share of the
// rows into part[b] (d x d, stride DM).  Thread t owns the 8 x 8 block
// (t / 16, t % 16) of the 128 x 128 result.
__global__ __launch_bounds__(256) void gram_partial_kernel(const float *M, int64_t n, int d,
                                                           double *part, bool split) {
  __shared__ float tile[64][DM + 4];
  const int bi = threadIdx.x >> 4, bj = threadIdx.x & 15;
  double acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
  const int64_t rows_per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min<int64_t>(n, r0 + rows_per);
  for (int64_t base = r0; base < r1; base += 64) {
    for (int e = threadIdx.x; e < 64 * DM; e += 256) {
      const int rr = e / DM, c = e - rr * DM;
      const int64_t r = base + rr;
      tile[rr][c] = (r < r1 && c < d) ? basis_ld(M, r * d + c, split) : 0.f;
    }
    __syncthreads();
    for (int rr = 0; rr < 64; ++rr) {
      double a[8], b[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a[q] = (double)tile[rr][bi * 8 + q];
        b[q] = (double)tile[rr][bj * 8 + q];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  double *out = part + (size_t)blockIdx.x * DM * DM;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) out[(bi * 8 + i) * DM + bj * 8 + j] = acc[i][j];
}

__global__ void gram_reduce_kernel(const double *part, int nparts, double *G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= DM * DM) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(size_t)b * DM * DM + e];
  G[e] = s;
}

// Workgroup `side` (0 = U, 1 = V): G = P^T Gb P, then G = R^T R (Cholesky,
// R upper triangular, written to Rout, stride DM).  A pivot below kMinPivot
// means the basis is far from orthonormal (not rounding drift): *bad is set
// and the caller leaves the state alone.
__global__ __launch_bounds__(1024) void gram_chol_kernel(const double *Gb, const double *P, int d,
                                                         double *T1, double *Rout, int *bad) {
  __shared__ double A[DM * DM];  // 128 KB
  const int side = blockIdx.x;
  const double *G = Gb + (size_t)side * DM * DM;
  const double *Ps = P + (size_t)side * d * d;
  double *T = T1 + (size_t)side * DM * DM;
  double *R = Rout + (size_t)side * DM * DM;
  // T = Gb P, then A = P^T T
  for (int e = threadIdx.x; e < d * d; e += 1024) {
    const int i = e / d, j = e - (e / d) * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) s = fma(G[i * DM + k], Ps[k * d + j], s);
    T[i * DM + j] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < d * d; e += 1024) {
    const int i = e / d, j = e - (e / d) * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) s = fma(Ps[k * d + i], T[k * DM + j], s);
    A[i * d + j] = s;
  }
  __syncthreads();
  // right-looking Cholesky A = L L^T in the lower triangle
  for (int j = 0; j < d; ++j) {
    const double piv = A[j * d + j];
    if (piv < kMinPivot && threadIdx.x == 0) atomicOr(bad, 1);
    const double ljj = sqrt(fmax(piv, kMinPivot));
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < d; i += 1024) A[i * d + j] /= ljj;
    __syncthreads();
    if (threadIdx.x == 0) A[j * d + j] = ljj;
    const int m = d - j - 1;
    for (int e = threadIdx.x; e < m * m; e += 1024) {
      const int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) A[i * d + l] = fma(-A[i * d + j], A[l * d + j], A[i * d + l]);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < d * d; e += 1024) {
    const int i = e / d, j = e - (e / d) * d;
    R[i * DM + j] = (j >= i) ? A[j * d + i] : 0.0;
  }
}

// Core t-SVD: C = R_U diag(Sigma) R_V^T (d x d) by FP64 one-sided Jacobi;
// C = Ut diag(S) Vt^T with S descending.  Columns whose S is zero (rank(A)
// below d) are completed to orthonormal bases so U and V stay orthonormal.
// Writes Ut, Vt (d x d, stride DM) and S (d).
__global__ __launch_bounds__(1024) void core_svd_kernel(const double *Rf, const double *sigma,
                                                        int d, double *Cg, double *Ut,
                                                        double *Vt, double *S) {
  constexpr int RPL = 2, NW = 16;  // NP = 128 >= d
  using SH = JacobiShape<RPL, NW>;
  constexpr int NP = SH::NP, CPW = SH::CPW;
  __shared__ double lds[SH::LDS];
  __shared__ double sv[NP];
  __shared__ int sid[NP], rank_of[NP];
  __shared__ double red[NP];
  __shared__ int flag;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double *RU = Rf, *RV = Rf + DM * DM;
  // C[i][j] = sum_k RU[i][k] sigma_k RV[j][k]  (both upper triangular: k >= max(i, j))
  for (int e = threadIdx.x; e < d * d; e += 1024) {
    const int i = e / d, j = e - (e / d) * d;
    double s = 0.0;
    for (int k = max(i, j); k < d; ++k) s = fma(RU[i * DM + k] * sigma[k], RV[j * DM + k], s);
    Cg[i * DM + j] = s;
  }
  __syncthreads();
  JacobiRegs<RPL, NW> J;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = jacobi_slot_col<RPL, NW>(w, c);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = r * 64 + lane;
      J.a[c][r] = (i < d && j < d) ? Cg[i * DM + j] : 0.0;
    }
  }
  jacobi_sweeps<RPL, NW>(J, lds, &flag, 40, 1e-13);
  const double *nrm = lds + 4 * NW * SH::SLOT;
  for (int j = threadIdx.x; j < NP; j += 1024) {
    sv[j] = sqrt(nrm[j]);
    sid[j] = j;
  }
  __syncthreads();
  for (int kk = 2; kk <= NP; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      if (threadIdx.x < NP) {
        const int i = threadIdx.x, q = i ^ jj;
        if (q > i) {
          const double a = sv[i], b = sv[q];
          const int ia = sid[i], ib = sid[q];
          const bool before = (a > b) || (a == b && ia < ib);
          const bool up = (i & kk) == 0;
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
  __syncthreads();
  const double cut = 1e-12 * sv[0];
  int live = 0;  // columns with S above the cut (a prefix: S is sorted)
  for (int j = 0; j < d; ++j) live += (sv[j] > cut) ? 1 : 0;
  if (threadIdx.x < d) S[threadIdx.x] = (sv[threadIdx.x] > cut) ? sv[threadIdx.x] : 0.0;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = jacobi_slot_col<RPL, NW>(w, c);
    const int rk = rank_of[j];
    if (rk < live) {
      const double inv = 1.0 / sv[rk];
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = r * 64 + lane;
        if (i < d) Ut[i * DM + rk] = J.a[c][r] * inv;
      }
    }
  }
  __syncthreads();
  // Vt[j][c] = sum_i C[i][j] Ut[i][c] / S_c
  for (int e = threadIdx.x; e < d * live; e += 1024) {
    const int j = e / live, c = e - (e / live) * live;
    double acc = 0.0;
    for (int i = 0; i < d; ++i) acc = fma(Cg[i * DM + j], Ut[i * DM + c], acc);
    Vt[j * DM + c] = acc / sv[c];
  }
  __syncthreads();
  // complete columns live .. d-1 of Ut and Vt: for column c, take the unit
  // vector e_p least covered by the columns so far, orthogonalise it twice
  // (classical Gram-Schmidt) and normalise
  for (int side = 0; side < 2; ++side) {
    double *Q = side ? Vt : Ut;
    for (int c = live; c < d; ++c) {
      if (threadIdx.x < d) {
        const int p = threadIdx.x;
        double cov = 0.0;
        for (int k = 0; k < c; ++k) cov = fma(Q[p * DM + k], Q[p * DM + k], cov);
        red[p] = cov;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int best = 0;
        for (int p = 1; p < d; ++p)
          if (red[p] < red[best]) best = p;
        flag = best;
      }
      __syncthreads();
      const int p = flag;
      if (threadIdx.x < d) Q[threadIdx.x * DM + c] = (threadIdx.x == p) ? 1.0 : 0.0;
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        // coefficients a_k = Q[:, k] . q, then q -= sum_k a_k Q[:, k]
        if (threadIdx.x < c) {
          const int k = threadIdx.x;
          double a = 0.0;
          for (int i = 0; i < d; ++i) a = fma(Q[i * DM + k], Q[i * DM + c], a);
          red[k] = a;
        }
        __syncthreads();
        double qi = 0.0;
        if (threadIdx.x < d) {
          const int i = threadIdx.x;
          qi = Q[i * DM + c];
          for (int k = 0; k < c; ++k) qi = fma(-red[k], Q[i * DM + k], qi);
        }
        __syncthreads();
        if (threadIdx.x < d) Q[threadIdx.x * DM + c] = qi;
        __syncthreads();
      }
      if (threadIdx.x < d) red[threadIdx.x] = Q[threadIdx.x * DM + c] * Q[threadIdx.x * DM + c];
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < d; ++i) s += red[i];
        red[NP - 1] = 1.0 / sqrt(s);
      }
      __syncthreads();
      const double inv = red[NP - 1];
      __syncthreads();
      if (threadIdx.x < d) Q[threadIdx.x * DM + c] *= inv;
      __syncthreads();
    }
  }
}

// Workgroup `side`: X = R^-1 Q (triangular solve, column per thread), then
// Rot = P X in FP32 for the MFMA rotation of the bases.
__global__ __launch_bounds__(128) void rotation_kernel(const double *Rf, const double *Qf,
                                                       const double *P, int d, double *X,
                                                       float *Rot) {
  const int side = blockIdx.x;
  const double *R = Rf + (size_t)side * DM * DM;
  const double *Q = Qf + (size_t)side * DM * DM;
  const double *Ps = P + (size_t)side * d * d;
  double *Xs = X + (size_t)side * DM * DM;
  float *Ro = Rot + (size_t)side * d * d;
  const int c = threadIdx.x;
  if (c < d) {
    for (int i = d - 1; i >= 0; --i) {
      double v = Q[i * DM + c];
      for (int k = i + 1; k < d; ++k) v = fma(-R[i * DM + k], Xs[k * DM + c], v);
      Xs[i * DM + c] = v / R[i * DM + i];
    }
  }
  __syncthreads();
  if (c < d) {
    for (int i = 0; i < d; ++i) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s = fma(Ps[i * d + k], Xs[k * DM + c], s);
      Ro[i * d + c] = (float)s;
    }
  }
}

__global__ void p_to_float_kernel(const double *P, float *Pf, int count) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) Pf[e] = (float)P[e];
}

// P <- I for both sides and, when S is given, Sigma <- S.
__global__ void reset_projection_kernel(double *P, int d, double *sigma, const double *S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < 2 * d * d) {
    const int r = e % (d * d);
    P[e] = (r / d == r % d) ? 1.0 : 0.0;
  }
  if (S && e < d) sigma[e] = S[e];
}

// Precision form: M <- M B in place for a basis of BF16 pairs (n x d,
// d <= 128) and FP32 B (d x d), on BF16 MFMA (v_mfma_f32_16x16x16 bf16):
// with M = Mh + Ml and B = Bh + Bl, M B ~ Mh Bh + Mh Bl + Ml Bh accumulated
// in FP32, then stored again as pairs.  The product reads and writes each
// row once (2 x 4d bytes for 6d flops per element), so it is bound by HBM.
// Workgroups of NW waves stride over blocks of 64 whole rows.  The waves
// split the 128 output columns; each keeps the B fragments (hi and lo) of
// its columns in registers for the whole launch, so LDS holds only the row
// block (33 KB) and several workgroups share a CU.  Rows are loaded and
// stored whole through that LDS tile, 16 B per lane when d is a multiple of
// 4, and the next block is loaded into registers while the current one is
// multiplied.  With NW = 4 the kernel takes 208 VGPRs (2 waves per SIMD);
// NW = 8 still takes 178, so it is launched with 4.
typedef short v4s16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));
template <bool V4, int NW>
__global__ __launch_bounds__(64 * NW) void gemm_split_kernel(float *M, int64_t n, int d,
                                                             const float *B) {
  __shared__ __align__(16) uint32_t As[64][DM + 4];  // row block as pairs; then the result
  constexpr int KT = DM / 16;
  constexpr int NT = DM / 16 / NW;   // 16-wide output tiles per wave
  constexpr int CPW = 16 * NT;       // output columns per wave
  constexpr int NTH = 64 * NW;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int dp = (d + 15) & ~15;  // k and output columns padded to the 16-wide MFMA
  const int nkt = dp >> 4;
  bool tile_on[NT];
  v4s16 bh[KT][NT], bl[KT][NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    const int col = CPW * w + 16 * c + (lane & 15);
    tile_on[c] = CPW * w + 16 * c < dp;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * kt + 4 * (lane >> 4) + j;
        const uint32_t b = (k < d && col < d) ? split_encode(B[k * d + col]) : 0u;
        bh[kt][c][j] = (short)(b >> 16);
        bl[kt][c][j] = (short)(b & 0xffffu);
      }
  }
  // row-block transfers: V4 moves 16 B per lane (d % 4 == 0), else 4 B
  constexpr int CW = V4 ? 4 : 1;            // words per transfer
  constexpr int PER = 64 * DM / NTH / CW;   // transfers per thread per block
  constexpr int RW = DM / CW;               // transfers per row
  uint4 pre4[V4 ? PER : 1];
  uint32_t pre1[V4 ? 1 : PER];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * NTH;
      const int i = e / RW, k = (e - i * RW) * CW;
      const int64_t r = r0 + i;
      const bool in = r < n && k < d;
      if constexpr (V4) {
        pre4[q] = in ? *reinterpret_cast<const uint4 *>(M + r * d + k) : uint4{0u, 0u, 0u, 0u};
      } else {
        pre1[q] = in ? __float_as_uint(M[r * d + k]) : 0u;
      }
    }
  };
  const int64_t step = (int64_t)gridDim.x * 64;
  fetch((int64_t)blockIdx.x * 64);
  for (int64_t row0 = (int64_t)blockIdx.x * 64; row0 < n; row0 += step) {
    __syncthreads();  // the previous block's results have been read out of As
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * NTH;
      const int i = e / RW, k = (e - i * RW) * CW;
      if constexpr (V4) {
        *reinterpret_cast<uint4 *>(&As[i][k]) = pre4[q];
      } else {
        As[i][k] = pre1[q];
      }
    }
    __syncthreads();
    if (row0 + step < n) fetch(row0 + step);
    v4f32 acc[4][NT];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int c = 0; c < NT; ++c) acc[rt][c] = v4f32{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      if (kt >= nkt) break;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const uint4 a = *reinterpret_cast<const uint4 *>(
            &As[16 * rt + (lane & 15)][16 * kt + 4 * (lane >> 4)]);
        const uint32_t av[4] = {a.x, a.y, a.z, a.w};
        v4s16 ah, al;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          ah[j] = (short)(av[j] >> 16);
          al[j] = (short)(av[j] & 0xffffu);
        }
#pragma unroll
        for (int c = 0; c < NT; ++c) {
          if (!tile_on[c]) continue;
          acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh[kt][c], acc[rt][c], 0, 0, 0);
          acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl[kt][c], acc[rt][c], 0, 0, 0);
          acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh[kt][c], acc[rt][c], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // every wave has read the row block
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        if (!tile_on[c]) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          As[16 * rt + 4 * (lane >> 4) + q][CPW * w + 16 * c + (lane & 15)] =
              split_encode(acc[rt][c][q]);
      }
    __syncthreads();
    // every row of the block was read before the first store, so in place is safe
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * NTH;
      const int i = e / RW, k = (e - i * RW) * CW;
      const int64_t r = row0 + i;
      if (r < n && k < d) {
        if constexpr (V4) {
          *reinterpret_cast<uint4 *>(M + r * d + k) = *reinterpret_cast<const uint4 *>(&As[i][k]);
        } else {
          M[r * d + k] = __uint_as_float(As[i][k]);
        }
      }
    }
  }
}

template <class T>
struct DevBuf {
  T *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t count) { return hipMalloc(&p, count * sizeof(T)); }
};

// Rotates every basis in place: U_b, Z_b, R by RotU; V_b by RotV.
hipError_t rotate_bases(damf_ctx *c, const float *RotU, const float *RotV) {
  hipStream_t s = c->stream;
  const int d = c->d;
  const int64_t n = c->n;
  auto basis = [&](float *M, const float *Rot) -> hipError_t {
    if (c->split) {
      // row blocks of 64, at least 16 per workgroup; 16-B row transfers need
      // d % 4 == 0 and a 16-B aligned basis
      const unsigned g = geom_gemm_split(n).blocks;
      if (d % 4 == 0 && reinterpret_cast<uintptr_t>(M) % 16 == 0)
        gemm_split_kernel<true, 4><<<g, 256, 0, s>>>(M, n, d, Rot);
      else
        gemm_split_kernel<false, 4><<<g, 256, 0, s>>>(M, n, d, Rot);
      return hipGetLastError();
    }
    return gemm_tall(M, n, d, d, Rot, d, M, d, s);
  };
  DAMF_HIP(basis(c->Ub, RotU));
  DAMF_HIP(basis(c->Vb, RotV));
  if (c->ppr_on) {  // Z_b and R are FP32 in both forms
    DAMF_HIP(gemm_tall(c->Zb, n, d, d, RotU, d, c->Zb, d, s));
    DAMF_HIP(gemm_tall(c->R, n, d, d, RotU, d, c->R, d, s));
  }
  return hipSuccess;
}

}  // namespace

hipError_t flush_projections(damf_ctx *c) {
  hipStream_t s = c->stream;
  const int d = c->d;
  DevBuf<float> Pf;
  DAMF_HIP(Pf.alloc(2 * (size_t)d * d));
  p_to_float_kernel<<<ceil_div(2 * d * d, 256), 256, 0, s>>>(c->P, Pf.p, 2 * d * d);
  DAMF_HIP(hipGetLastError());
  DAMF_HIP(rotate_bases(c, Pf.p, Pf.p + (size_t)d * d));
  reset_projection_kernel<<<ceil_div(2 * d * d, 256), 256, 0, s>>>(c->P, d, nullptr, nullptr);
  DAMF_HIP(hipGetLastError());
  return hipStreamSynchronize(s);
}

hipError_t reorthogonalize(damf_ctx *c, int *numeric_bad) {
  hipStream_t s = c->stream;
  const int d = c->d;
  const int64_t n = c->n;
  *numeric_bad = 0;
  DevBuf<double> part, G, T1, Rf, Cg, Qf, X, S;
  DevBuf<float> Rot;
  DevBuf<int> bad;
  DAMF_HIP(part.alloc((size_t)kGramParts * DM * DM));
  DAMF_HIP(G.alloc(2 * (size_t)DM * DM));
  DAMF_HIP(T1.alloc(2 * (size_t)DM * DM));
  DAMF_HIP(Rf.alloc(2 * (size_t)DM * DM));
  DAMF_HIP(Cg.alloc((size_t)DM * DM));
  DAMF_HIP(Qf.alloc(2 * (size_t)DM * DM));
  DAMF_HIP(X.alloc(2 * (size_t)DM * DM));
  DAMF_HIP(S.alloc(DM));
  DAMF_HIP(Rot.alloc(2 * (size_t)d * d));
  DAMF_HIP(bad.alloc(1));
  DAMF_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  for (int side = 0; side < 2; ++side) {
    gram_partial_kernel<<<kGramParts, 256, 0, s>>>(side ? c->Vb : c->Ub, n, d, part.p, c->split);
    gram_reduce_kernel<<<ceil_div(DM * DM, 256), 256, 0, s>>>(part.p, kGramParts,
                                                              G.p + (size_t)side * DM * DM);
    DAMF_HIP(hipGetLastError());
  }
  gram_chol_kernel<<<2, 1024, 0, s>>>(G.p, c->P, d, T1.p, Rf.p, bad.p);
  DAMF_HIP(hipGetLastError());
  int hbad = 0;
  DAMF_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  DAMF_HIP(hipStreamSynchronize(s));
  if (hbad) {  // nothing has been modified yet
    *numeric_bad = 1;
    return hipSuccess;
  }
  core_svd_kernel<<<1, 1024, 0, s>>>(Rf.p, c->sigma, d, Cg.p, Qf.p, Qf.p + (size_t)DM * DM, S.p);
  rotation_kernel<<<2, 128, 0, s>>>(Rf.p, Qf.p, c->P, d, X.p, Rot.p);
  DAMF_HIP(hipGetLastError());
  DAMF_HIP(rotate_bases(c, Rot.p, Rot.p + (size_t)d * d));
  reset_projection_kernel<<<ceil_div(2 * d * d, 256), 256, 0, s>>>(c->P, d, c->sigma, S.p);
  DAMF_HIP(hipGetLastError());
  return hipStreamSynchronize(s);
}

}  // namespace damf
