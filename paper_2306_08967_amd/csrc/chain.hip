// chain.hip -- Steps 1-3 of the update (Sec. 4.5; Theorem 2; Algorithm 1,
// UpdateEmbeddingE) for every chunk of a batch.
//
// Chunks depend on each other through Sigma and the projections, so they run
// one after another; each step of a chunk is a kernel of one or two 512-thread
// workgroups that keep the small dense state in LDS / L2 and the core matrix
// in VGPRs.  For a chunk with rows S1, columns S2 and dA = I[:,S1] D I[:,S2]^T
// the kernels compute, in the U-form (U = U_b P_U, V = V_b P_V):
//
//   Step 1  W_B = U^T B, W_C = V^T C  (gather of the touched rows, Lemma 2)
//           residual Grams G = B^T B - W^T W (Proposition 1 for k columns),
//           factored by pivoted Cholesky with drop threshold tau:
//           (I - U U^T) B ~ Q_B R_B,  Q_B = (I - U U^T) B T_B
//   Step 2  K = [[Sigma, 0], [0, 0]] + [W_B; R_B][W_C; R_C]^T, FP64 one-sided
//           Jacobi SVD K = E Theta H^T, keep the top d
//   Step 3  F_U = E[:d] - W_B T_B E[d:],  dU = B T_B E[d:]   (same for V)
//           P_U <- P_U F_U and U_b[S1] += dU P_U^-1 (the lazy base-space
//           update of Sec. 4.1), Sigma <- Theta[:d]
//
// The PPR residual R receives the same base-coordinate signal change as U_b
// (Step 4 input, Algorithm 2).
#include <hip/hip_runtime.h>

#include <cfloat>
#include <utility>

#include "common.h"
#include "damf_internal.h"
#include "jacobi_wave.h"

namespace damf {

namespace {

constexpr int NPMAX = 192;   // max padded core size
constexpr int DMAX = 128;
constexpr int KMAX = 64;
constexpr int LDS_DOUBLES = 19456;  // 152 KB (with 4 KB of ints, under the CU's 160 KB)
// Core-SVD Jacobi tolerance: a pair is rotated while |a_i . a_j| exceeds it
// relative to ||a_i|| ||a_j||, and sweeps stop once every rotation of a sweep
// was below its square root, leaving the columns orthogonal to about 1e-9 --
// well under the rounding of the FP32 bases the result is stored into (6e-8).
// The precision form stores about 16 significant bits (2^-17 relative), so
// its default is 1e-8: C1's product error against the FP64 oracle stays at
// 5.9e-6 either way, and a batch takes about 10% fewer sweeps.
// damf_config.jacobi_tol overrides both.
constexpr double kJacobiTol = 1e-9;
// The lazy scatter solves with the new projection P and stores U_b's rows in
// FP32, so its rounding reaches U = U_b P amplified by up to cond(P).  A pivot
// ratio max |u_ii| / min |u_ii| of P's LU above the chunk limit marks P as too
// ill-conditioned for that, and the chunk is applied explicitly instead
// (api.hip).  The limit is the flush limit, at least kMinExplicitCond; with
// flushing off it is kSingularCond (only numerically singular P).
constexpr double kSingularCond = 1e10;
constexpr double kMinExplicitCond = 1e3;
constexpr double kJacobiTolSplit = 1e-8;

// global scratch layout (doubles)
constexpr size_t OFF_EG = 0;                              // E, col-major, stride NPMAX
constexpr size_t OFF_HG = OFF_EG + NPMAX * DMAX;          // H, row-major [j][c], stride DMAX
constexpr size_t OFF_UP = OFF_HG + NPMAX * DMAX;          // U rows of S1, [i][c]
constexpr size_t OFF_VP = OFF_UP + KMAX * DMAX;
constexpr size_t OFF_WB = OFF_VP + KMAX * DMAX;           // W_B^T [t][c]
constexpr size_t OFF_WC = OFF_WB + KMAX * DMAX;
constexpr size_t OFF_LB = OFF_WC + KMAX * DMAX;           // pivoted Cholesky factor [i][j]
constexpr size_t OFF_LC = OFF_LB + KMAX * KMAX;
constexpr size_t OFF_RB = OFF_LC + KMAX * KMAX;           // R_B [i][t]
constexpr size_t OFF_RC = OFF_RB + KMAX * KMAX;
constexpr size_t OFF_FU = OFF_RC + KMAX * KMAX;           // F_U [i][c]
constexpr size_t OFF_FV = OFF_FU + DMAX * DMAX;
constexpr size_t OFF_DU = OFF_FV + DMAX * DMAX;           // dU rows [i][c]
constexpr size_t OFF_DV = OFF_DU + KMAX * DMAX;
constexpr size_t OFF_YB = OFF_DV + KMAX * DMAX;           // Y = T E_bot [t][c]
constexpr size_t OFF_YC = OFF_YB + KMAX * DMAX;
constexpr size_t OFF_DU2 = OFF_YC + KMAX * DMAX;          // dU, dV of odd chunks
constexpr size_t OFF_DV2 = OFF_DU2 + KMAX * DMAX;
constexpr size_t OFF_TH = OFF_DV2 + KMAX * DMAX;          // theta (NPMAX)
constexpr size_t OFF_META = OFF_TH + NPMAX + 64;         // ints: rho_B, rho_C, perm_B, perm_C
constexpr size_t SCRATCH_DOUBLES = OFF_META + (2 + 2 * KMAX) / 2 + 8;
// Row corrections of chunk ch (side 0: dU on S1, side 1: dV on S2), by chunk
// parity: the solve-and-scatter of chunk ch runs while chunk ch + 1 computes.
__host__ __device__ constexpr size_t off_dl(int side, int ch) {
  return (ch & 1) ? (side ? OFF_DV2 : OFF_DU2) : (side ? OFF_DV : OFF_DU);
}

struct ChainParams {
  int d;
  int64_t n;
  const ChunkDesc *chunks;
  int n_chunks;
  const int32_t *S1, *S2;
  const NetEntry *ent;
  float *Ub, *Vb, *R;
  double *P, *Pnext;  // [P_U | P_V], 2 d x d row-major
  double *sigma;
  double *scr;
  double tau;
  double jtol;  // relative tolerance of the core's Jacobi
  double explicit_cond;  // pivot ratio of the new P above which a chunk goes explicit
  ChainStats *stats;
  bool split;  // U_b, V_b as BF16 pairs
};

struct ChunkState {
  int s1, s2, k, mode;  // mode 1: s1 <= s2 (B = I[:,S1]), mode 0: B = I[:,S1] D
  int rhoB, rhoC;
  const int32_t *S1, *S2;
  const NetEntry *ent;
  int ne;
};

__device__ __forceinline__ int tid() { return threadIdx.x; }
constexpr int NT = kChainThreads;
constexpr int NW = NT / 64;   // waves
constexpr int NG = NT / 128;  // groups of 128 threads (one column each)

// ---------------------------------------------------------------- Step 1

// C = A B for one 512-thread workgroup on FP64 MFMA (v_mfma_f64_16x16x4f64),
// M, N <= 128, any K.  The 16 x 16 output tiles t = I TN + J (TN = ceil(N /
// 16)) are dealt to the 8 waves (wave w: t = w, w + 8, ...; at most 8 each,
// one v4f64 accumulator per tile).  K is staged through LDS KC = 16 values at
// a time, A as [i][k] (odd row stride, conflict-free fragment reads) and B as
// [k][j]; the next stage is fetched into registers while the current one is
// used (A with consecutive threads along k, B along j: both coalesced for
// row-major operands).  aload(i, k), bload(k, c) fetch the operands; cstore(i,
// c, v) writes the result.  Uses wg_mma_lds() doubles of LDS; starts and ends
// with the caller's LDS free.
typedef double v4f64 __attribute__((ext_vector_type(4)));
constexpr int kMmaKC = 16, kMmaAS = kMmaKC + 1, kMmaBS = 128 + 2;
constexpr int wg_mma_lds() { return 128 * kMmaAS + kMmaKC * kMmaBS; }
// NQ tiles per wave: tile slot q of wave w is t = w + 8 q, clamped to the last
// tile (a clamped slot repeats that tile's MFMAs and is not stored), so the
// inner loop has no branches.
template <int NQ, class AL, class BL, class CS>
__device__ __forceinline__ void wg_mma_n(int M, int N, int K, int TN, int T, AL aload, BL bload,
                                         CS cstore, double *lds) {
  constexpr int KC = kMmaKC, AS = kMmaAS, BS = kMmaBS;
  constexpr int PF = KC * 128 / NT;  // operand values per thread per stage
  static_assert(NT == 512 && PF * NT == KC * 128 && wg_mma_lds() <= LDS_DOUBLES, "wg_mma shape");
  double *As = lds, *Bs = lds + 128 * AS;
  const int lane = tid() & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid() >> 6);
  v4f64 acc[NQ];
  int ia[NQ], ib[NQ];  // fragment offsets of the wave's tiles
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    acc[q] = v4f64{0.0, 0.0, 0.0, 0.0};
    const int t = min(w + 8 * q, T - 1), I = t / TN, J = t - I * TN;
    ia[q] = (16 * I + (lane & 15)) * AS + (lane >> 4);
    ib[q] = (lane >> 4) * BS + 16 * J + (lane & 15);
  }
  double pa[PF], pb[PF];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid() + q * NT;
      const int i = e / KC, kk = e % KC, kb = e >> 7, c = e & 127;
      pa[q] = (i < M && k0 + kk < K) ? aload(i, k0 + kk) : 0.0;
      pb[q] = (c < N && k0 + kb < K) ? bload(k0 + kb, c) : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();  // the previous stage's fragments are read
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid() + q * NT;
      As[(e / KC) * AS + e % KC] = pa[q];
      Bs[(e >> 7) * BS + (e & 127)] = pb[q];
    }
    __syncthreads();
    if (k0 + KC < K) fetch(k0 + KC);
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      double a[NQ], b[NQ];  // all of the step's fragments first, then the MFMAs
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        a[q] = As[ia[q] + ks];
        b[q] = Bs[ib[q] + ks * BS];
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc[q], 0, 0, 0);
    }
  }
  // output layout: register v of lane group g (lanes 16 g .. 16 g + 15) holds
  // row 4 v + g of the tile, column lane % 16
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = w + 8 * q;
    if (t < T) {
      const int I = t / TN, J = t - I * TN;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * I + 4 * v + (lane >> 4), c = 16 * J + (lane & 15);
        if (i < M && c < N) cstore(i, c, acc[q][v]);
      }
    }
  }
  __syncthreads();
}
template <class AL, class BL, class CS>
__device__ __forceinline__ void wg_mma(int M, int N, int K, AL aload, BL bload, CS cstore, double *lds) {
  const int TN = __builtin_amdgcn_readfirstlane((N + 15) >> 4);
  const int T = __builtin_amdgcn_readfirstlane(((M + 15) >> 4) * TN);
  if (T > 32)
    wg_mma_n<8>(M, N, K, TN, T, aload, bload, cstore, lds);
  else if (T > 16)
    wg_mma_n<4>(M, N, K, TN, T, aload, bload, cstore, lds);
  else if (T > 8)
    wg_mma_n<2>(M, N, K, TN, T, aload, bload, cstore, lds);
  else if (T > 0)
    wg_mma_n<1>(M, N, K, TN, T, aload, bload, cstore, lds);
}

// MP[i][c] = sum_q Mb[rows[i]][q] * Pm[q][c]  (rows of U or V in the current basis)
__device__ __forceinline__ void gather_project(const float *Mb, const int32_t *rows, int s, const double *Pm,
                               int d, double *lds, double *MP, bool split) {
  wg_mma(
      s, d, d, [&](int i, int q) { return (double)basis_ld(Mb, (int64_t)rows[i] * d + q, split); },
      [&](int q, int c) { return Pm[q * d + c]; }, [&](int i, int c, double v) { MP[i * d + c] = v; },
      lds);
}

// Dense D (s1 x s2) into LDS from the chunk entries.
__device__ __forceinline__ void build_D(const ChunkState &cs, double *D) {
  for (int e = tid(); e < cs.s1 * cs.s2; e += NT) D[e] = 0.0;
  __syncthreads();
  for (int e = tid(); e < cs.ne; e += NT) {
    NetEntry en = cs.ent[e];
    int i = (int)lower_bound(cs.S1, (int64_t)cs.s1, en.row);
    int j = (int)lower_bound(cs.S2, (int64_t)cs.s2, en.col);
    D[i * cs.s2 + j] = (double)en.delta;
  }
  __syncthreads();
}

// W^T (k x d) for one side into Wg (global): side 0 (B): mode 1: W_B^T = UP;
// mode 0: W_B^T = D^T UP.  side 1 (C): mode 1: W_C^T = D VP; mode 0: W_C^T =
// VP.  D (LDS, s1 x s2) stays readable; stage is wg_mma's LDS.
__device__ __forceinline__ void build_Wt(const ChunkState &cs, int side, int d, const double *D,
                                      const double *MP, double *Wg, double *stage) {
  const int k = cs.k, s2 = cs.s2;
  const bool copy = side ? (cs.mode == 0) : (cs.mode != 0);
  if (copy) {
    for (int e = tid(); e < k * d; e += NT) Wg[e] = MP[e];
    __syncthreads();
  } else if (side == 0) {
    wg_mma(
        k, d, cs.s1, [&](int t, int i) { return D[i * s2 + t]; },
        [&](int i, int c) { return MP[i * d + c]; }, [&](int t, int c, double v) { Wg[t * d + c] = v; },
        stage);
  } else {
    wg_mma(
        k, d, s2, [&](int t, int j) { return D[t * s2 + j]; },
        [&](int j, int c) { return MP[j * d + c]; }, [&](int t, int c, double v) { Wg[t * d + c] = v; },
        stage);
  }
}

// G = B^T B - W^T W (side B) or C^T C - W^T W (side C), k x k in LDS (row
// stride KMAX), as one product [B^T | W] [B | -W]^T (B^T B = D^T D, C^T C =
// D D^T, or I); also returns max(1, max diag of B^T B) through *bmax.
__device__ __forceinline__ void build_gram(const ChunkState &cs, int side, int d, const double *D,
                                        const double *Wg, double *G, double *bmax_out, double *stage) {
  const int k = cs.k, s2 = cs.s2;
  __shared__ double s_bmax;
  const bool ident = (side == 0) ? (cs.mode != 0) : (cs.mode == 0);
  const int sB = ident ? 0 : ((side == 0) ? cs.s1 : s2);
  // column a of B (side B: D[:, a]) or row a of C^T (side C: D[a, :])
  auto bel = [&](int a, int x) { return (side == 0) ? D[x * s2 + a] : D[a * s2 + x]; };
  if (tid() == 0) s_bmax = 1.0;
  __syncthreads();
  for (int a = tid(); a < k && sB > 0; a += NT) {
    double v = 0.0;
    for (int x = 0; x < sB; ++x) v = fma(bel(a, x), bel(a, x), v);
    if (v > 1.0) atomicMax((unsigned long long *)&s_bmax, __double_as_longlong(v));
  }
  wg_mma(
      k, k, sB + d, [&](int a, int x) { return (x < sB) ? bel(a, x) : Wg[a * d + x - sB]; },
      [&](int x, int b) { return (x < sB) ? bel(b, x) : -Wg[b * d + x - sB]; },
      [&](int a, int b, double v) { G[a * KMAX + b] = (ident && a == b) ? 1.0 + v : v; }, stage);
  *bmax_out = s_bmax;
  __syncthreads();
}

// (value, index) of the larger value, ties to the lower index: a total
// order, so a butterfly leaves every lane with the same winner.
__device__ __forceinline__ void argmax_take(double &v, int &i, double ov, int oi) {
  // non-short-circuit operators: a select, not a branch, per stage
  const bool take = (ov > v) | ((ov == v) & (oi < i));
  v = take ? ov : v;
  i = take ? oi : i;
}
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double &v, int &i) {
  argmax_take(v, i, dpp_d<CTRL>(v), __builtin_amdgcn_mov_dpp(i, CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ void argmax_wave(double &v, int &i) {
  argmax_dpp<0xB1>(v, i);   // quad_perm [1,0,3,2]
  argmax_dpp<0x4E>(v, i);   // quad_perm [2,3,0,1]
  argmax_dpp<0x141>(v, i);  // row_half_mirror
  argmax_dpp<0x140>(v, i);  // row_mirror
  {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    const auto ii = __builtin_amdgcn_permlane16_swap(i, i, false, false);
    double va = __hiloint2double(hi[0], lo[0]), vb = __hiloint2double(hi[1], lo[1]);
    int ia = ii[0], ib = ii[1];
    argmax_take(va, ia, vb, ib);
    v = va;
    i = ia;
  }
  {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    const auto ii = __builtin_amdgcn_permlane32_swap(i, i, false, false);
    double va = __hiloint2double(hi[0], lo[0]), vb = __hiloint2double(hi[1], lo[1]);
    int ia = ii[0], ib = ii[1];
    argmax_take(va, ia, vb, ib);
    v = va;
    i = ia;
  }
}
// Pivoted Cholesky of the k x k PSD matrix G (LDS, row stride KMAX, k <= 64)
// by the whole workgroup: thread (row i = tid % 64, column group cg = tid /
// 64) keeps the Schur complement's entries (i, 8 cg .. 8 cg + 7) in VGPRs,
// and every wave keeps its diagonal (lane i: row i).  Each step every wave
// picks the largest remaining diagonal v (the same wave argmax on the same
// values, so the same pivot everywhere) and stops when it is <= thr; the wave
// holding the pivot's column writes that column u of the Schur complement to
// LDS; after one barrier every thread applies the rank-1 update u u^T / v to
// its eight entries and its diagonal copy, and the owner stores column j of L
// (u / sqrt(v)) into G.  The column buffer alternates between two halves of
// lc by step parity, so a wave that runs ahead never overwrites a column
// another wave still reads; lc holds 2 KMAX doubles of LDS.  Rows are never
// moved: on return G[i][j] (j < rho) holds L in the original row order (row
// i's entry for the j-th pivot; 0 for steps after row i was itself the
// pivot), perm[j] the j-th pivot for j < rho and the other rows in increasing
// order after it.  Returns rho.
__device__ __forceinline__ double sel8(double g0, double g1, double g2, double g3, double g4, double g5,
                                       double g6, double g7, int u) {
  // a select tree on the bits of a wave-uniform u (no runtime-indexed array,
  // which would live in scratch memory)
  const double a0 = (u & 1) ? g1 : g0, a1 = (u & 1) ? g3 : g2;
  const double a2 = (u & 1) ? g5 : g4, a3 = (u & 1) ? g7 : g6;
  const double b0 = (u & 2) ? a1 : a0, b1 = (u & 2) ? a3 : a2;
  return (u & 4) ? b1 : b0;
}
__device__ __forceinline__ int pivoted_cholesky(double *G, int k, double thr, int *perm, double *lc) {
  static_assert(KMAX == 64 && NT == 512, "one row per lane, eight column groups");
  const int i = tid() & 63;
  const int cg = __builtin_amdgcn_readfirstlane(tid() >> 6);
  const bool row = i < k;
  double g[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int c = 8 * cg + u;
    g[u] = (row && c < k) ? G[i * KMAX + c] : 0.0;
  }
  double dg = row ? G[i * KMAX + i] : 0.0;
  __syncthreads();  // every thread has read G before column 0 of L overwrites it
  uint64_t done = 0;  // rows already used as pivots (uniform)
  int rho = k;
  for (int j = 0; j < k; ++j) {
    double v = (row && !((done >> i) & 1)) ? dg : -1.0;
    int p = i;
    argmax_wave(v, p);
    p = __builtin_amdgcn_readfirstlane(p);
    if (!(v > thr)) {  // the same decision in every wave
      rho = j;
      break;
    }
    double *col = lc + (j & 1) * KMAX;
    const bool owner = cg == (p >> 3);
    const bool live = row && !((done >> i) & 1);
    if (owner) {
      const double gp = sel8(g[0], g[1], g[2], g[3], g[4], g[5], g[6], g[7], p & 7);
      col[i] = live ? gp : 0.0;  // the pivot's own entry is v
      if (i == 0) perm[j] = p;
    }
    const double inv = rcp_nr(v);
    __syncthreads();
    done |= 1ull << p;
    const double ui = col[i];
    const double si = ui * inv;
    const double2 *u2 = reinterpret_cast<const double2 *>(col + 8 * cg);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 x = u2[q];
      g[2 * q] = fma(-si, x.x, g[2 * q]);
      g[2 * q + 1] = fma(-si, x.y, g[2 * q + 1]);
    }
    dg = fma(-si, ui, dg);
    if (owner && row) G[i * KMAX + j] = ui * rsqrt_nr(v);  // column j of L
  }
  // the remaining rows after the pivots, in increasing order
  if (cg == 0 && row && !((done >> i) & 1)) {
    const uint64_t below = (i == 0) ? 0ull : (~done & ((1ull << i) - 1));
    perm[rho + __builtin_popcountll(below)] = i;
  }
  __syncthreads();
  return rho;
}

// L (k x k, pivoted order) and R (rho x k): with Lo = G in original row
// order, L[a][b] = Lo[perm[a]][b] (b < rho) and R[i][perm[j]] = L[j][i] (j >= i),
// i.e. R = L^T Pi^T.
__device__ __forceinline__ void store_factor(const double *G, int k, int rho, const int *perm, double *Lg,
                             double *Rg) {
  for (int e = tid(); e < KMAX * KMAX; e += NT) {
    const int i = e >> 6, j = e & 63;
    if (i < k && j < k) Lg[i * k + j] = (j < rho) ? G[perm[i] * KMAX + j] : 0.0;
    if (i < rho && j < k) Rg[i * k + perm[j]] = (j >= i) ? G[perm[j] * KMAX + i] : 0.0;
  }
}

// ---------------------------------------------------------------- Step 2

template <int RPL>
__device__ __noinline__ int core_svd(const ChunkState &cs, int d, const double *sigma, double *scr,
                         double *lds, int *ilds, int *sweeps_out, uint64_t *ticks, double jtol) {
  constexpr int NP = 64 * RPL;
  using S = JW<NP>;
  static_assert(S::LDS <= LDS_DOUBLES && NT == 64 * S::NW, "Jacobi layout does not fit the workgroup");
  const int lane = tid() & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid() >> 6);
  const int k = cs.k;
  const int NB = d + cs.rhoB, NC = d + cs.rhoC;
  const double *WBt = scr + OFF_WB, *WCt = scr + OFF_WC;
  const double *RB = scr + OFF_RB, *RC = scr + OFF_RC;
  double *EG = scr + OFF_EG, *HG = scr + OFF_HG, *TH = scr + OFF_TH;
  // K = diag(Sigma, 0) + L_m R_m^T with L_m = [W_B; R_B], R_m = [W_C; R_C]
  // (NP x k each); wave w holds columns jw_col(w, c), lane l rows l + 64 r.
  // Both factors are staged in LDS as [t][i] in chunks of KC values of t;
  // a wave reads its columns' R_m entries as broadcasts.
  constexpr int KC = 32;
  static_assert(2 * KC * NP <= LDS_DOUBLES, "K build staging does not fit");
  double *Lm = lds, *Rm = lds + KC * NP;
  JWRegs<S> J;
#pragma unroll
  for (int c = 0; c < S::C; ++c) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) J.a[c][r] = 0.0;
  }
  for (int t0 = 0; t0 < k; t0 += KC) {
    const int tn = min(KC, k - t0);
    __syncthreads();
    for (int e = tid(); e < tn * NP; e += NT) {
      const int t = t0 + e / NP, i = e % NP;
      double lv = 0.0, rv = 0.0;
      if (i < d) {
        lv = WBt[t * d + i];
        rv = WCt[t * d + i];
      } else {
        if (i < NB) lv = RB[(i - d) * k + t];
        if (i < NC) rv = RC[(i - d) * k + t];
      }
      Lm[e] = lv;
      Rm[e] = rv;
    }
    __syncthreads();
    for (int t = 0; t < tn; ++t) {
      double lm[RPL];
#pragma unroll
      for (int r = 0; r < RPL; ++r) lm[r] = Lm[t * NP + r * 64 + lane];
#pragma unroll
      for (int c = 0; c < S::C; ++c) {
        const double rm = Rm[t * NP + jw_col<S>(w, c)];
#pragma unroll
        for (int r = 0; r < RPL; ++r) J.a[c][r] = fma(lm[r], rm, J.a[c][r]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < S::C; ++c) {
    const int j = jw_col<S>(w, c);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = r * 64 + lane;
      if (i >= NB || j >= NC) J.a[c][r] = 0.0;
      if (i == j && i < d) J.a[c][r] += sigma[i];
    }
  }
  __syncthreads();
  int *flag = ilds;
  int *skipped = ilds + 2;  // steps without a rotation, counted by jw_sweeps
  if (tid() == 0) *skipped = 0;
  __syncthreads();
  uint64_t tj0 = wall_clock64();
  const int sweeps = jw_sweeps<S>(J, lds, flag, 40, jtol);
  if (tid() == 0) ticks[1] += wall_clock64() - tj0;
  *sweeps_out = sweeps;
  // ---- singular values, descending order
  double *sv = lds;                        // NP values
  int *sid = ilds + 8;                     // NP column ids -> sorted order
  int *rank_of = ilds + 8 + 256;           // column id -> rank

  __syncthreads();
  // a NaN or infinite value gets the key -0.5: it sorts after every finite
  // value and before the -1 padding, so the sort stays a total order and
  // every real column keeps a rank below NP
  for (int j = tid(); j < NP; j += NT) {
    const double v = sqrt(jw_norm2<S>(lds, j));
    sv[j] = (v <= DBL_MAX) ? v : -0.5;
    sid[j] = j;
  }
  __syncthreads();
  // bitonic sort descending by value (ties by id), NP entries padded to 256
  for (int i = NP + tid(); i < 256; i += NT) {
    sv[i] = -1.0;
    sid[i] = 1 << 20;
  }
  __syncthreads();
  for (int kk = 2; kk <= 256; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      if (tid() < 256) {
        int i = tid(), q = i ^ jj;
        if (q > i) {
          double a = sv[i], b = sv[q];
          int ia = sid[i], ib = sid[q];
          bool before = (a > b) || (a == b && ia < ib);  // a should precede b
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
  const int nonfinite = sv[NP - 1] < 0.0;  // some column norm was NaN or infinite
  if (tid() < NP) rank_of[sid[tid()]] = tid();
  if (tid() < NPMAX) TH[tid()] = (tid() < NP) ? sv[tid()] : 0.0;
  __syncthreads();
  const double smax = sv[0];
  const double cut = 1e-10 * smax;
  // E columns (top d), zero rows beyond NB
#pragma unroll
  for (int c = 0; c < S::C; ++c) {
    const int j = jw_col<S>(w, c);
    const int rk = rank_of[j];
    if (rk < d) {
      const double sv_ = sv[rk];
      const double inv = (sv_ > cut) ? 1.0 / sv_ : 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = r * 64 + lane;
        EG[rk * NPMAX + i] = (i < NB) ? J.a[c][r] * inv : 0.0;
      }
    }
  }
  __syncthreads();
  // ---- H = K^T E Theta^-1 for the top d, from K = D + L_m R_m^T (D =
  // diag(Sigma, 0)): K^T E = D E + R_m (L_m^T E), two products on FP64 MFMA
  // (2 k NB d + 2 NC k d flops instead of 2 NC NB d for K^T E itself).
  {
    double *T1 = lds + 6000;            // L_m^T E, k x d (row stride DMAX)
    double *rth = lds + 6000 + KMAX * DMAX;  // 1 / theta_c, 0 below the cut
    static_assert(wg_mma_lds() <= 6000 && 6000 + KMAX * DMAX + DMAX <= LDS_DOUBLES, "H staging");
    for (int c = tid(); c < d; c += NT) rth[c] = (TH[c] > cut) ? 1.0 / TH[c] : 0.0;
    wg_mma(
        k, d, NB, [&](int t, int i) { return (i < d) ? WBt[t * d + i] : RB[(i - d) * k + t]; },
        [&](int i, int c) { return EG[c * NPMAX + i]; }, [&](int t, int c, double v) { T1[t * DMAX + c] = v; },
        lds);
    for (int j0 = 0; j0 < NC; j0 += 128) {
      wg_mma(
          min(128, NC - j0), d, k,
          [&](int jj, int t) {
            const int j = j0 + jj;
            return (j < d) ? WCt[t * d + j] : RC[(j - d) * k + t];
          },
          [&](int t, int c) { return T1[t * DMAX + c]; },
          [&](int jj, int c, double v) {
            const int j = j0 + jj;
            const double de = (j < d) ? sigma[j] * EG[c * NPMAX + j] : 0.0;
            HG[j * DMAX + c] = (v + de) * rth[c];
          },
          lds);
    }
    for (int e = tid(); e < (NP - NC) * d; e += NT) {
      const int j = NC + e / d, c = e - (e / d) * d;
      HG[j * DMAX + c] = 0.0;
    }
  }
  __syncthreads();
  return nonfinite;
}

// H = K^T E Theta^-1 carries the Jacobi's residual non-orthogonality of E
// amplified by sigma_1 / theta_c: with |e_c . e_j| <= jtol, h_c . h_j can reach
// jtol sigma_j / theta_c, which is O(1) for a theta_c at the rounding floor of
// a kept zero singular value.  Columns c < d with cut < theta_c <= hrel
// sigma_1 (ascending rank, so every larger column is final first) are
// re-orthogonalised against the columns before them (classical Gram-Schmidt,
// twice, all waves) and normalised: that moves K^T e_c - theta_c h_c by about
// jtol sigma_1, far below the FP32 bases' rounding.  A column left with less
// than half its length lies in the span of the earlier ones; it is zeroed and
// marked in `redo` for complete_basis.  Returns the number of columns treated.
__device__ __noinline__ int orthonormalize_small_h(int d, int NC, double hrel, double *scr, double *lds,
                                                   int *redo) {
  const double *TH = scr + OFF_TH;
  double *HG = scr + OFF_HG;
  const double cut = 1e-10 * TH[0], hcut = hrel * TH[0];
  const int lane = tid() & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid() >> 6);
  double *dots = lds;  // d
  __shared__ double s_nn;
  int treated = 0;
  for (int c = 0; c < d; ++c) {
    if (tid() == 0) redo[c] = 0;
    if (!(TH[c] <= hcut) || TH[c] <= cut) continue;
    ++treated;
    for (int pass = 0; pass < 2; ++pass) {
      for (int o = w; o < c; o += NW) {
        double sdot = 0.0;
        for (int j = lane; j < NC; j += 64) sdot = fma(HG[j * DMAX + o], HG[j * DMAX + c], sdot);
        sdot = wave_sum(sdot);
        if (lane == 0) dots[o] = sdot;
      }
      __syncthreads();
      for (int j = tid(); j < NC; j += NT) {
        double v = HG[j * DMAX + c];
        for (int o = 0; o < c; ++o) v = fma(-dots[o], HG[j * DMAX + o], v);
        HG[j * DMAX + c] = v;
      }
      __syncthreads();
    }
    if (w == 0) {
      double nn = 0.0;
      for (int j = lane; j < NC; j += 64) nn = fma(HG[j * DMAX + c], HG[j * DMAX + c], nn);
      nn = wave_sum(nn);
      if (lane == 0) s_nn = nn;
    }
    __syncthreads();
    const double nn = s_nn;
    const bool keep = nn > 0.25;
    const double sc = keep ? 1.0 / sqrt(nn) : 0.0;
    for (int j = tid(); j < NC; j += NT) HG[j * DMAX + c] *= sc;
    if (tid() == 0 && !keep) redo[c] = 1;
    __syncthreads();
  }
  return treated;
}

// Orthonormal completion of columns c < d whose singular value is <= cut:
// E (NB rows, col-major stride NPMAX) and H (NC rows, row-major stride DMAX);
// also the H columns that orthonormalize_small_h marked in `redo`.
__device__ __noinline__ void complete_basis(int d, int NB, int NC, double *scr, const int *redo) {
  const double *TH = scr + OFF_TH;
  double *EG = scr + OFF_EG, *HG = scr + OFF_HG;
  const double cut = 1e-10 * TH[0];
  if (tid() >= 64) return;
  const int lane = tid() & 63;
  for (int c = 0; c < d; ++c) {
    const bool zero = TH[c] <= cut, hredo = redo != nullptr && redo[c] != 0;
    if (!zero && !hredo) continue;
    for (int side = zero ? 0 : 1; side < 2; ++side) {
      const int N = side ? NC : NB;
      auto at = [&](int i, int cc) -> double & {
        return side ? HG[i * DMAX + cc] : EG[cc * NPMAX + i];
      };
      for (int cand = 0; cand < N; ++cand) {
        double v[3];
        for (int r = 0; r < 3; ++r) {
          int i = r * 64 + lane;
          v[r] = (i == cand) ? 1.0 : 0.0;
        }
        for (int pass = 0; pass < 2; ++pass) {
          for (int o = 0; o < d; ++o) {
            if (o == c || (TH[o] <= cut && o > c)) continue;
            double dot = 0.0;
            for (int r = 0; r < 3; ++r) {
              int i = r * 64 + lane;
              if (i < N) dot += at(i, o) * v[r];
            }
            dot = wave_sum(dot);
            for (int r = 0; r < 3; ++r) {
              int i = r * 64 + lane;
              if (i < N) v[r] -= dot * at(i, o);
            }
          }
        }
        double nn = 0.0;
        for (int r = 0; r < 3; ++r) {
          int i = r * 64 + lane;
          if (i < N) nn += v[r] * v[r];
        }
        nn = wave_sum(nn);
        if (nn > 0.25) {
          double inv = 1.0 / sqrt(nn);
          for (int r = 0; r < 3; ++r) {
            int i = r * 64 + lane;
            if (i < N) at(i, c) = v[r] * inv;
          }
          break;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- Step 3

template <int I>
__device__ __forceinline__ void solve_Y_step(double (&x)[KMAX / 4], int q, int rho, const double *L, int k,
                                             const double *rinv) {
  if (I >= rho) return;  // uniform
  constexpr int r = I & 3, mi = I >> 2;
  // row I is final: scale it in its owner lane, then hand it to the quad
  const bool own = q == r;
  x[mi] = own ? x[mi] * rinv[I] : x[mi];
  const double xi = dpp_d<r | (r << 2) | (r << 4) | (r << 6)>(x[mi]);  // quad_perm [r,r,r,r]
  const double keep = x[mi];
  // rows j < I of the quad's column: x_j -= L[I][j] x_I (L[I][j] = 0 for
  // j > I, so those rows are unchanged; the owner's row I is put back)
#pragma unroll
  for (int m = 0; m < KMAX / 4; ++m) {
    if (4 * m <= I) x[m] = fma(-L[I * k + 4 * m + q], xi, x[m]);
  }
  x[mi] = own ? keep : x[mi];
}

template <int... I>
__device__ __forceinline__ void solve_Y_steps(double (&x)[KMAX / 4], int q, int rho, const double *L, int k,
                                              const double *rinv, std::integer_sequence<int, I...>) {
  (solve_Y_step<KMAX - 1 - I>(x, q, rho, L, k, rinv), ...);
}

// Y = T E_bot (k x d): solve L1^T X = E_bot (rho x d) by back substitution
// with the pivoted Cholesky factor (k x k, lower triangular in pivot order)
// and scatter the rows by perm; side 0 uses E (rows d.. of EG), side 1 H
// (rows d.. of HG).  Four lanes per column hold its rows j = 4 m + q
// in registers; after row I is final (the right-looking form) its owner lane
// hands it to the quad by DPP and every lane subtracts L[I][j] x_I from its
// rows, so the only LDS traffic is the factor's rows (broadcast reads that
// do not depend on the solve) and a step's latency is a DPP move and an FMA.
__device__ __forceinline__ void solve_Y(int side, int d, int k, int rho, const int *perm, const double *Lg,
                        double *scr, double *lds) {
  static_assert(NT == 4 * DMAX && KMAX == 64, "four lanes per column, 16 rows each");
  double *Y = scr + (side ? OFF_YC : OFF_YB);
  const double *EG = scr + OFF_EG, *HG = scr + OFF_HG;
  double *L = lds;                    // k x k
  double *rinv = lds + KMAX * KMAX;   // rho
  for (int e = tid(); e < k * k; e += NT) L[e] = Lg[e];
  for (int i = tid(); i < rho; i += NT) rinv[i] = 1.0 / Lg[i * k + i];
  const int c = tid() >> 2, q = tid() & 3;
  const bool col = c < d;
  double x[KMAX / 4];
#pragma unroll
  for (int m = 0; m < KMAX / 4; ++m) {
    const int i = 4 * m + q;
    x[m] = (col && i < rho) ? (side ? HG[(d + i) * DMAX + c] : EG[c * NPMAX + d + i]) : 0.0;
  }
  __syncthreads();
  solve_Y_steps(x, q, rho, L, k, rinv, std::make_integer_sequence<int, KMAX>{});
  // rows of Y: the solved rows at their pivots' positions, zeros for the
  // dropped directions (perm is a permutation of 0 .. k - 1)
  if (col) {
#pragma unroll
    for (int m = 0; m < KMAX / 4; ++m) {
      const int i = 4 * m + q;
      if (i < k) Y[perm[i] * d + c] = (i < rho) ? x[m] : 0.0;
    }
  }
  __syncthreads();
}

// F = E_top - W Y (d x d) and the row corrections, as workgroup GEMMs.
__device__ __forceinline__ void build_F_and_delta(const ChunkState &cs, int side, int d, double *scr,
                                  double *lds, int ch) {
  const int k = cs.k, s2 = cs.s2;
  const double *Y = scr + (side ? OFF_YC : OFF_YB);
  const double *Wt = scr + (side ? OFF_WC : OFF_WB);
  const double *EG = scr + OFF_EG, *HG = scr + OFF_HG;
  double *F = scr + (side ? OFF_FV : OFF_FU);
  double *Dl = scr + off_dl(side, ch);
  wg_mma(
      d, d, k, [&](int i, int t) { return Wt[t * d + i]; }, [&](int t, int c) { return Y[t * d + c]; },
      [&](int i, int c, double v) {
        F[i * d + c] = (side ? HG[i * DMAX + c] : EG[c * NPMAX + i]) - v;
      },
      lds);
  // row corrections: side B: mode 1 -> Y (s1 rows); mode 0 -> D Y (s1 x d)
  //                  side C: mode 1 -> D^T Y (s2 rows); mode 0 -> Y
  const bool direct = side ? (cs.mode == 0) : (cs.mode != 0);
  if (direct) {
    for (int e = tid(); e < k * d; e += NT) Dl[e] = Y[e];
    __syncthreads();
    return;
  }
  double *D = lds;  // s1 x s2
  double *stage = lds + KMAX * KMAX;
  static_assert(KMAX * KMAX + wg_mma_lds() <= LDS_DOUBLES, "Step 3 staging does not fit");
  for (int e = tid(); e < cs.s1 * s2; e += NT) D[e] = 0.0;
  __syncthreads();
  for (int e = tid(); e < cs.ne; e += NT) {
    NetEntry en = cs.ent[e];
    int i = (int)lower_bound(cs.S1, (int64_t)cs.s1, en.row);
    int j = (int)lower_bound(cs.S2, (int64_t)s2, en.col);
    D[i * s2 + j] = (double)en.delta;
  }
  __syncthreads();
  if (side == 0)
    wg_mma(
        cs.s1, d, k, [&](int i, int t) { return D[i * s2 + t]; }, [&](int t, int c) { return Y[t * d + c]; },
        [&](int i, int c, double v) { Dl[i * d + c] = v; }, stage);
  else
    wg_mma(
        s2, d, k, [&](int i, int t) { return D[t * s2 + i]; }, [&](int t, int c) { return Y[t * d + c]; },
        [&](int i, int c, double v) { Dl[i * d + c] = v; }, stage);
}

// Pn = Po F (d x d).
__device__ __forceinline__ void mul_PF(int d, const double *Po, const double *F, double *Pn, double *lds) {
  wg_mma(
      d, d, d, [&](int i, int q) { return Po[i * d + q]; }, [&](int q, int c) { return F[q * d + c]; },
      [&](int i, int c, double v) { Pn[i * d + c] = v; }, lds);
}

// Partial-pivoting LU of the panel A[j0.., j0 .. j0 + jb) (jb <= 16), by one
// wave with the panel in VGPRs: lane l holds rows l and l + 64.  Pivot search
// by a wave argmax (DPP and lane swaps); the two rows to swap are passed
// through LDS (rb, 2 x 16 doubles) and read back by every lane, then the
// scaling and rank-1 updates run lane by lane.  Records piv[j]; sets *bad on a
// zero pivot column.
__device__ __forceinline__ void lu_panel(double *A, int d, int j0, int jb, int *piv, int *bad,
                                         double *rb) {
  constexpr int LUB = 16;
  const int lane = tid() & 63;
  double pr[2][LUB];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = lane + 64 * h;
#pragma unroll
    for (int t = 0; t < LUB; ++t) pr[h][t] = (i >= j0 && i < d && t < jb) ? A[i * d + j0 + t] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < LUB; ++t) {
    if (t < jb) {
      const int j = j0 + t;
      double v = (lane >= j && lane < d) ? fabs(pr[0][t]) : -1.0;
      int idx = lane;
      argmax_take(v, idx, (lane + 64 >= j && lane + 64 < d) ? fabs(pr[1][t]) : -1.0, lane + 64);
      argmax_wave(v, idx);
      idx = __builtin_amdgcn_readfirstlane(idx);
      if (lane == 0) {
        piv[j] = idx;
        if (!(v > 0.0)) *bad = 1;
      }
      // the pivot row (and row j when they differ) through LDS (rb: 2 x LUB
      // doubles; LDS operations of one wave complete in order).  j, idx and
      // their halves are wave-uniform, so only the swap's two lanes select.
      const int jh = j >> 6, jl = j & 63, ph = idx >> 6, pl = idx & 63;
      const bool swap = idx != j;
      if (lane == pl) {
        if (ph == 0) {
#pragma unroll
          for (int c = 0; c < LUB; ++c) rb[LUB + c] = pr[0][c];
        } else {
#pragma unroll
          for (int c = 0; c < LUB; ++c) rb[LUB + c] = pr[1][c];
        }
      }
      if (swap && lane == jl) {
        if (jh == 0) {
#pragma unroll
          for (int c = 0; c < LUB; ++c) rb[c] = pr[0][c];
        } else {
#pragma unroll
          for (int c = 0; c < LUB; ++c) rb[c] = pr[1][c];
        }
      }
      __builtin_amdgcn_wave_barrier();
      double rowp[LUB];
#pragma unroll
      for (int c = 0; c < LUB; ++c) rowp[c] = rb[LUB + c];
      if (swap) {
        double rowj[LUB];
#pragma unroll
        for (int c = 0; c < LUB; ++c) rowj[c] = rb[c];
        if (jh == 0) {
#pragma unroll
          for (int c = 0; c < LUB; ++c) pr[0][c] = (lane == jl) ? rowp[c] : pr[0][c];
        } else {
#pragma unroll
          for (int c = 0; c < LUB; ++c) pr[1][c] = (lane == jl) ? rowp[c] : pr[1][c];
        }
        if (ph == 0) {
#pragma unroll
          for (int c = 0; c < LUB; ++c) pr[0][c] = (lane == pl) ? rowj[c] : pr[0][c];
        } else {
#pragma unroll
          for (int c = 0; c < LUB; ++c) pr[1][c] = (lane == pl) ? rowj[c] : pr[1][c];
        }
      }
      __builtin_amdgcn_wave_barrier();
      const double pv = rowp[t];
      const double inv = (pv != 0.0) ? 1.0 / pv : 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        const bool below = i > j && i < d;
        const double l = below ? pr[h][t] * inv : 0.0;
        pr[h][t] = below ? l : pr[h][t];
#pragma unroll
        for (int c = 0; c < LUB; ++c)
          if (c > t) pr[h][c] = fma(-l, rowp[c], pr[h][c]);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = lane + 64 * h;
    if (i >= j0 && i < d) {
#pragma unroll
      for (int t = 0; t < LUB; ++t)
        if (t < jb) A[i * d + j0 + t] = pr[h][t];
    }
  }
}

// LU with partial pivoting of Pn (d x d) in LDS, then X Pn = Dl for `rows`
// row vectors; adds X to M_b[rows] (and to R when given).  Returns 0, or 1 if
// a zero pivot was met.
__device__ __forceinline__ int lu_solve_scatter(int d, const double *Pn, const double *Dl, const int32_t *rows,
                                int nrows, float *Mb, float *Rr, double *lds, int *ilds,
                                bool split, double limit, double *cond_out) {
  double *A = lds;  // d x d
  int *piv = ilds;  // d
  int *src = ilds + DMAX;
  __shared__ int s_bad;
  __shared__ double s_cond;
  for (int e = tid(); e < d * d; e += NT) A[e] = Pn[e];
  if (tid() == 0) s_bad = 0;
  __syncthreads();
  const int lane = tid() & 63;
  // Blocked right-looking LU with partial pivoting, panels of LUB columns:
  // wave 0 factors the panel (pivot search, swaps inside the panel, scaling,
  // rank-1 updates), then all threads apply the panel's row swaps to the
  // other columns, form U12 = L11^-1 A12 and update A22 -= A21 U12.
  constexpr int LUB = 16;
  for (int j0 = 0; j0 < d; j0 += LUB) {
    const int jb = min(LUB, d - j0);
    if (tid() < 64) lu_panel(A, d, j0, jb, piv, &s_bad, lds + DMAX * DMAX);
    __syncthreads();
    // row swaps of this panel on the columns outside it, in pivot order
    for (int c = tid(); c < d; c += NT) {
      if (c >= j0 && c < j0 + jb) continue;
      for (int j = j0; j < j0 + jb; ++j) {
        const int p = piv[j];
        if (p != j) {
          const double t = A[j * d + c];
          A[j * d + c] = A[p * d + c];
          A[p * d + c] = t;
        }
      }
    }
    __syncthreads();
    // U12 = L11^-1 A12 (unit lower L11), one column per thread
    for (int c = j0 + jb + tid(); c < d; c += NT) {
      for (int i = 1; i < jb; ++i) {
        double v = A[(j0 + i) * d + c];
        for (int t = 0; t < i; ++t) v -= A[(j0 + i) * d + j0 + t] * A[(j0 + t) * d + c];
        A[(j0 + i) * d + c] = v;
      }
    }
    __syncthreads();
    // A22 -= A21 U12: thread owns column c and rows j0 + jb + g, + NG, ...,
    // four rows at a time; with even d and a full panel a row of A21 is read
    // as 16-byte pairs
    const bool pairs = (d % 2 == 0) && jb == LUB;
    {
      const int c = tid() & 127;
      const int g = tid() >> 7;
      if (c >= j0 + jb && c < d) {
        double u[LUB];
#pragma unroll
        for (int t = 0; t < LUB; ++t) u[t] = (t < jb) ? A[(j0 + t) * d + c] : 0.0;
        for (int i = j0 + jb + g; i < d; i += 4 * NG) {
          double v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int ii = i + q * NG;
            v[q] = (ii < d) ? A[ii * d + c] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int ii = i + q * NG;
            if (ii < d && pairs) {
              const double2 *ar = reinterpret_cast<const double2 *>(A + ii * d + j0);
#pragma unroll
              for (int t2 = 0; t2 < LUB / 2; ++t2) {
                const double2 x = ar[t2];
                v[q] = fma(-x.x, u[2 * t2], v[q]);
                v[q] = fma(-x.y, u[2 * t2 + 1], v[q]);
              }
            } else if (ii < d) {
#pragma unroll
              for (int t = 0; t < LUB; ++t)
                if (t < jb) v[q] = fma(-A[ii * d + j0 + t], u[t], v[q]);
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int ii = i + q * NG;
            if (ii < d) A[ii * d + c] = v[q];
          }
        }
      }
    }
    __syncthreads();
  }
  if (tid() == 0) {
    for (int c = 0; c < d; ++c) src[c] = c;
    for (int j = d - 1; j >= 0; --j) {
      int t = src[j];
      src[j] = src[piv[j]];
      src[piv[j]] = t;
    }
  }
  if (tid() < 64) {
    // condition estimate of the new P: the spread of the LU's pivots
    double mx = 0.0, mn = INFINITY;
    for (int c = tid(); c < d; c += 64) {
      const double u = fabs(A[c * d + c]);
      mx = fmax(mx, u);
      mn = fmin(mn, u);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      mx = fmax(mx, __shfl_xor(mx, off, 64));
      mn = fmin(mn, __shfl_xor(mn, off, 64));
    }
    if (tid() == 0) {
      const double cond = (mn > 0.0) ? mx / mn : INFINITY;
      s_cond = (cond == cond) ? cond : INFINITY;
      if (!(s_cond <= limit)) s_bad = 1;
    }
  }
  __syncthreads();
  if (tid() == 0) *cond_out = s_cond;
  if (s_bad) return 1;
  // Row-vector solves X Pn = Dl: wave w takes rows w, w + NW, ... (up to
  // SR of them at once, interleaved for latency); lanes own columns
  // c = lane, lane + 64.  Pivot entries are broadcast with v_readlane.
  constexpr int SR = KMAX / NW;
  const int w = __builtin_amdgcn_readfirstlane(tid() >> 6);
  double y0[SR], y1[SR];
#pragma unroll
  for (int q = 0; q < SR; ++q) {
    const int i = w + NW * q;
    y0[q] = (i < nrows && lane < d) ? Dl[i * d + lane] : 0.0;
    y1[q] = (i < nrows && lane + 64 < d) ? Dl[i * d + lane + 64] : 0.0;
  }
  // Y U = Dl, forward over columns
#pragma unroll 2
  for (int c = 0; c < d; ++c) {
    const double inv = 1.0 / A[c * d + c];
    const double u0 = (lane > c && lane < d) ? A[c * d + lane] : 0.0;
    const double u1 = (lane + 64 > c && lane + 64 < d) ? A[c * d + lane + 64] : 0.0;
#pragma unroll
    for (int q = 0; q < SR; ++q) {
      const double own = (c < 64) ? y0[q] : y1[q];
      const double yc = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(own), c & 63),
                                         __builtin_amdgcn_readlane(__double2loint(own), c & 63)) *
                        inv;
      if (lane == (c & 63)) {
        if (c < 64)
          y0[q] = yc;
        else
          y1[q] = yc;
      }
      y0[q] = fma(-yc, u0, y0[q]);
      y1[q] = fma(-yc, u1, y1[q]);
    }
  }
  // W L = Y (L unit lower), backward over columns
#pragma unroll 2
  for (int c = d - 1; c >= 0; --c) {
    const double l0 = (lane < c && lane < d) ? A[c * d + lane] : 0.0;
    const double l1 = (lane + 64 < c) ? A[c * d + lane + 64] : 0.0;
#pragma unroll
    for (int q = 0; q < SR; ++q) {
      const double own = (c < 64) ? y0[q] : y1[q];
      const double zc = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(own), c & 63),
                                         __builtin_amdgcn_readlane(__double2loint(own), c & 63));
      y0[q] = fma(-zc, l0, y0[q]);
      y1[q] = fma(-zc, l1, y1[q]);
    }
  }
  // X = W Pi (the recorded row swaps, as a gather through src), then scatter;
  // the row buffers overlay the factor, so wait until every wave is done
  __syncthreads();
  double *rowbuf = lds + w * SR * DMAX;
#pragma unroll
  for (int q = 0; q < SR; ++q) {
    if (lane < d) rowbuf[q * DMAX + lane] = y0[q];
    if (lane + 64 < d) rowbuf[q * DMAX + lane + 64] = y1[q];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
  for (int q = 0; q < SR; ++q) {
    const int i = w + NW * q;
    if (i >= nrows) continue;
    const int64_t row = rows[i];
    for (int c = lane; c < d; c += 64) {
      const double x = rowbuf[q * DMAX + src[c]];
      const int64_t at = row * d + c;
      basis_st(Mb, at, (float)((double)basis_ld(Mb, at, split) + x), split);
      if (Rr) atomicAdd(Rr + row * d + c, (float)x);  // a push may run concurrently
    }
  }
  __syncthreads();
  return 0;
}

// A chunk runs as four kernels.  front (one workgroup per side): Step 1 --
// gather/project the touched rows, the residual Gram and its pivoted Cholesky
// factor.  core (one workgroup): Step 2 -- the core SVD and Sigma <- Theta.
// back (one workgroup per side): Step 3 -- Y, F and the row corrections,
// P <- P F.  scatter (one workgroup per side, second stream): the LU solve and
// scatter into the base rows.  The two sides of front, back and scatter are
// independent and run on two CUs each.

__device__ __forceinline__ ChunkState chunk_state(const ChainParams &p, int ch, const int *meta) {
  const ChunkDesc desc = p.chunks[ch];
  ChunkState cs;
  cs.s1 = desc.s1;
  cs.s2 = desc.s2;
  cs.mode = (cs.s1 <= cs.s2) ? 1 : 0;
  cs.k = cs.mode ? cs.s1 : cs.s2;
  cs.S1 = p.S1 + desc.s1_off;
  cs.S2 = p.S2 + desc.s2_off;
  cs.ent = p.ent + desc.e_off;
  cs.ne = desc.ne;
  cs.rhoB = meta ? meta[0] : 0;
  cs.rhoC = meta ? meta[1] : 0;
  return cs;
}

// phase clocks, added to the batch statistics by the first workgroup:
// 0 gather/project, 7 Grams + pivoted Cholesky, 2 core SVD total, 1 Jacobi
// sweeps (inside 2), 3 basis completion, 4 Y/F/row corrections, 5 P <- P F,
// 6 LU + solve + scatter
struct PhaseClock {
  uint64_t t;
  __device__ PhaseClock() : t(wall_clock64()) {}
  __device__ void tick(ChainStats *st, int ph) {
    const uint64_t now = wall_clock64();
    if (ph >= 0 && tid() == 0 && blockIdx.x == 0)
      atomicAdd((unsigned long long *)&st->phase_ticks[ph], (unsigned long long)(now - t));
    t = now;
  }
};

// Step 1 of chunk ch.  With pend, the solve-and-scatter of chunk ch - 1 has
// not run yet (it waits for this kernel): the rows this chunk shares with
// chunk ch - 1 are read as they were before that chunk, and its row
// corrections are added here, since (M_b + dM P^-1) P = M_b P + dM with P
// the projection after chunk ch - 1.
__global__ __launch_bounds__(NT) void chain_front_kernel(ChainParams p, int ch, const double *Pc,
                                                         int pend) {
  __shared__ __align__(16) double lds[LDS_DOUBLES];
  __shared__ __align__(16) int ilds[1024];
  const int side = blockIdx.x;
  const int d = p.d;
  double *scr = p.scr;
  int *meta = reinterpret_cast<int *>(scr + OFF_META);
  ChunkState cs = chunk_state(p, ch, nullptr);
  const int k = cs.k;
  PhaseClock clk;
  const int32_t *rows = side ? cs.S2 : cs.S1;
  const int ns = side ? cs.s2 : cs.s1;
  double *MP = scr + (side ? OFF_VP : OFF_UP);
  gather_project(side ? p.Vb : p.Ub, rows, ns, Pc + side * d * d, d, lds, MP, p.split);
  if (pend) {
    const ChunkDesc pd = p.chunks[ch - 1];
    const int32_t *prow = side ? p.S2 + pd.s2_off : p.S1 + pd.s1_off;
    const int pn = side ? pd.s2 : pd.s1;
    const double *Dl = scr + off_dl(side, ch - 1);
    int *at = ilds;  // row i's position in chunk ch - 1's list, or -1
    for (int i = tid(); i < ns; i += NT) {
      const int a = (int)lower_bound(prow, (int64_t)pn, rows[i]);
      at[i] = (a < pn && prow[a] == rows[i]) ? a : -1;
    }
    __syncthreads();
    for (int e = tid(); e < ns * d; e += NT) {
      const int i = e / d, c = e - i * d, a = at[i];
      if (a >= 0) MP[e] += Dl[a * d + c];
    }
    __syncthreads();
  }
  clk.tick(p.stats, 0);
  double bmax = 1.0;
  double *D = lds;                              // s1 x s2 (<= 4096)
  double *stage = lds + KMAX * KMAX;            // GEMM staging (< 8192)
  static_assert(wg_mma_lds() <= KMAX * DMAX, "Step 1 GEMM staging must end before G");
  double *G = lds + KMAX * KMAX + KMAX * DMAX;  // k x k, row stride KMAX
  double *Wg = scr + (side ? OFF_WC : OFF_WB);  // W^T, k x d
  build_D(cs, D);
  build_Wt(cs, side, d, D, scr + (side ? OFF_VP : OFF_UP), Wg, stage);
  build_gram(cs, side, d, D, Wg, G, &bmax, stage);
  int *perm = ilds;
  const int rho = pivoted_cholesky(G, k, p.tau * bmax, perm, lds);
  store_factor(G, k, rho, perm, scr + (side ? OFF_LC : OFF_LB), scr + (side ? OFF_RC : OFF_RB));
  for (int i = tid(); i < k; i += NT) meta[2 + side * KMAX + i] = perm[i];
  if (tid() == 0) {
    meta[side] = rho;
    if (k > rho) atomicAdd(&p.stats->dropped, k - rho);
  }
  clk.tick(p.stats, 7);
}

__global__ __launch_bounds__(NT) void chain_core_kernel(ChainParams p, int ch) {
  __shared__ __align__(16) double lds[LDS_DOUBLES];
  __shared__ __align__(16) int ilds[1024];
  __shared__ uint64_t jt[8];
  const int d = p.d;
  double *scr = p.scr;
  const int *meta = reinterpret_cast<const int *>(scr + OFF_META);
  ChunkState cs = chunk_state(p, ch, meta);
  const int k = cs.k;
  if (tid() < 8) jt[tid()] = 0;
  __syncthreads();
  PhaseClock clk;
  const int N = d + max(cs.rhoB, cs.rhoC);
  int sw = 0, nonfinite;
  if (N <= 64)
    nonfinite = core_svd<1>(cs, d, p.sigma, scr, lds, ilds, &sw, jt, p.jtol);
  else if (N <= 128)
    nonfinite = core_svd<2>(cs, d, p.sigma, scr, lds, ilds, &sw, jt, p.jtol);
  else
    nonfinite = core_svd<3>(cs, d, p.sigma, scr, lds, ilds, &sw, jt, p.jtol);
  if (nonfinite && tid() == 0) atomicOr(&p.stats->numeric_error, kNumericCore);
  clk.tick(p.stats, 2);
  // small singular values: H's columns re-orthogonalised (the threshold bounds
  // the amplified Jacobi tolerance by 1e-5 in the worst case; the sweeps'
  // quadratic convergence leaves far less), zero ones completed
  const double hrel = fmin(0.5, p.jtol * 1e5);
  int *redo = ilds + 600;
  int small_h = 0;
  if (scr[OFF_TH + d - 1] <= hrel * scr[OFF_TH]) {
    small_h = orthonormalize_small_h(d, d + cs.rhoC, hrel, scr, lds, redo);
    __syncthreads();
    bool any_redo = false;
    for (int c = 0; c < d; ++c) any_redo = any_redo || redo[c] != 0;
    if (any_redo || scr[OFF_TH + d - 1] <= 1e-10 * scr[OFF_TH]) {
      complete_basis(d, d + cs.rhoB, d + cs.rhoC, scr, redo);
      __syncthreads();
    }
  }
  for (int c = tid(); c < d; c += NT) p.sigma[c] = scr[OFF_TH + c];
  clk.tick(p.stats, 3);
  if (tid() == 0) {
    // counted FP64 work of this chunk: Jacobi (N(N-1)/2 pairs per sweep, a
    // dot of 2N flops each and a rotation of 6N flops in the steps whose
    // shears ran, share shf), H = K^T E, F, P F, LU and solves
    const double Nn = (double)N, dd = (double)d, kk = (double)k;
    // ilds[2]: steps (over the waves) without a rotation, from core_svd; a
    // sweep has 8 waves x (16 B - 1) steps, B = NP / 16 columns per half-block
    const int np = N <= 64 ? 64 : (N <= 128 ? 128 : 192);
    const double all_steps = (double)sw * 8.0 * (np - 1.0);
    const double shf = sw > 0 ? 1.0 - ilds[2] / all_steps : 1.0;
    const double jac = sw * 0.5 * Nn * (Nn - 1.0) * (2.0 * Nn + 6.0 * Nn * shf);
    atomicAdd(&p.stats->core_flops, jac + 2.0 * Nn * Nn * dd + 2.0 * Nn * Nn * kk);
    atomicAdd(&p.stats->core_flops_model, sw * 9.0 * Nn * Nn * Nn);
    double flops = jac + 2.0 * Nn * Nn * dd;
    flops += 2.0 * (2.0 * dd * dd * kk + 2.0 * dd * dd * dd + (2.0 / 3.0) * dd * dd * dd +
                    2.0 * 2.0 * (double)max(cs.s1, cs.s2) * dd * dd);
    flops += 2.0 * (double)(cs.s1 + cs.s2) * dd * dd + 4.0 * kk * kk * dd;
    atomicAdd(&p.stats->flops, flops);
    atomicAdd(&p.stats->sweeps, sw);
    if (small_h) atomicAdd(&p.stats->small_sv_columns, small_h);
    atomicMax(&p.stats->max_core, N);
    atomicAdd((unsigned long long *)&p.stats->phase_ticks[1], (unsigned long long)jt[1]);
  }
}

__global__ __launch_bounds__(NT) void chain_back_kernel(ChainParams p, int ch, const double *Pc,
                                                        double *Pn) {
  __shared__ __align__(16) double lds[LDS_DOUBLES];
  const int side = blockIdx.x;
  const int d = p.d;
  double *scr = p.scr;
  const int *meta = reinterpret_cast<const int *>(scr + OFF_META);
  ChunkState cs = chunk_state(p, ch, meta);
  PhaseClock clk;
  solve_Y(side, d, cs.k, side ? cs.rhoC : cs.rhoB, meta + 2 + side * KMAX,
          scr + (side ? OFF_LC : OFF_LB), scr, lds);
  build_F_and_delta(cs, side, d, scr, lds, ch);
  clk.tick(p.stats, 4);
  mul_PF(d, Pc + side * d * d, scr + (side ? OFF_FV : OFF_FU), Pn + side * d * d, lds);
  clk.tick(p.stats, 5);
}

// Step 3's row update of chunk ch, M_b[rows] += dM P_new^-1 (and the same
// signal change into R), on its own stream beside the next chunk's Steps
// 1-2.  Reads only P_new of this chunk, its row corrections (parity buffer)
// and its row lists, none of which the next chunk overwrites; a next chunk
// that reads any of its rows waits for it (launch_chain).
__global__ __launch_bounds__(NT) void chain_scatter_kernel(ChainParams p, int ch, const double *Pn) {
  __shared__ __align__(16) double lds[LDS_DOUBLES];
  __shared__ __align__(16) int ilds[1024];
  const int side = blockIdx.x;
  const int d = p.d;
  ChunkState cs = chunk_state(p, ch, nullptr);
  PhaseClock clk;
  double cond = 0.0;
  const int bad = lu_solve_scatter(d, Pn + side * d * d, p.scr + off_dl(side, ch),
                                   side ? cs.S2 : cs.S1, side ? cs.s2 : cs.s1,
                                   side ? p.Vb : p.Ub, side ? nullptr : p.R, lds, ilds, p.split,
                                   p.explicit_cond, &cond);
  if (tid() == 0) {
    // largest condition estimate of the batch (non-negative doubles order
    // like their bit patterns)
    atomicMax((unsigned long long *)&p.stats->p_cond_bits,
              (unsigned long long)__double_as_longlong(cond));
    if (bad) atomicOr(&p.stats->numeric_error, kNumericSingularP);
  }
  clk.tick(p.stats, 6);
}

}  // namespace

size_t chain_scratch_doubles() { return SCRATCH_DOUBLES; }

namespace {

ChainParams chain_params(damf_ctx *c, int n_chunks) {
  ChainParams p;
  p.d = c->d;
  p.n = c->n;
  p.chunks = c->ws.chunks;
  p.n_chunks = n_chunks;
  p.S1 = c->ws.chunk_s1;
  p.S2 = c->ws.chunk_s2;
  p.ent = c->ws.chunk_ent;
  p.Ub = c->Ub;
  p.Vb = c->Vb;
  p.R = c->ppr_on ? c->R : nullptr;
  p.P = c->P;
  p.Pnext = c->Pnext;
  p.sigma = c->sigma;
  p.scr = c->ws.scratch;
  p.tau = c->cfg.tau;
  p.jtol = c->cfg.jacobi_tol > 0.0 ? c->cfg.jacobi_tol : (c->split ? kJacobiTolSplit : kJacobiTol);
  const double limit = c->cfg.flush_cond == 0.0 ? kDefaultFlushCond : c->cfg.flush_cond;
  p.explicit_cond = limit > 0.0 ? std::max(limit, kMinExplicitCond) : kSingularCond;
  p.stats = c->ws.cstats;
  p.split = c->split;
  return p;
}

__global__ void zero_stats_kernel(ChainStats *st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *st = ChainStats{};
}

__global__ void copy_doubles_kernel(double *dst, const double *src, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// The launch sequence of chunks [first, last) (see launch_chain).  With
// `graph` every device-side step is a kernel (no memset or copy nodes), so the
// sequence can be captured into a HIP graph and replayed.
hipError_t enqueue_chain(damf_ctx *c, int first, int last, int n_chunks, const uint64_t *meets,
                         bool graph) {
  hipStream_t s = c->stream;
  const ChainParams p = chain_params(c, n_chunks);
  if (graph)
    zero_stats_kernel<<<1, 64, 0, s>>>(c->ws.cstats);
  else
    DAMF_HIP(hipMemsetAsync(c->ws.cstats, 0, sizeof(ChainStats), s));
  hipStream_t t = c->scatter_stream;
  double *Pbuf[2] = {c->P, c->Pnext};
  const bool timed = c->cfg.kernel_timing != 0 && !graph;
  c->core_timed = 0;
  for (int ch = first; ch < last; ++ch) {
    const int j = ch - first;
    const bool meet = j >= 1 && ((meets[ch >> 6] >> (ch & 63)) & 1);
    const bool hold = meet && ((c->chain_hold[ch >> 6] >> (ch & 63)) & 1);
    if (hold) {
      // chunk ch - 1's solve-and-scatter first, and the front reads its rows
      chain_scatter_kernel<<<2, NT, 0, t>>>(p, ch - 1, Pbuf[j & 1]);
      DAMF_HIP(hipEventRecord(c->ev_scatter[(ch - 1) & 3], t));
      DAMF_HIP(hipStreamWaitEvent(s, c->ev_scatter[(ch - 1) & 3], 0));
    }
    // the front reads rows that chunk ch - 2's solve-and-scatter wrote; the
    // corrections of chunk ch - 1 to the rows they share it adds itself
    if (j >= 2) DAMF_HIP(hipStreamWaitEvent(s, c->ev_scatter[(ch - 2) & 3], 0));
    const bool pend = meet && !hold;
    chain_front_kernel<<<2, NT, 0, s>>>(p, ch, Pbuf[j & 1], pend ? 1 : 0);
    if (j >= 1 && !hold) {
      // chunk ch - 1's solve-and-scatter, once this front has read its rows
      DAMF_HIP(hipEventRecord(c->ev_front[ch & 3], s));
      DAMF_HIP(hipStreamWaitEvent(t, c->ev_front[ch & 3], 0));
      chain_scatter_kernel<<<2, NT, 0, t>>>(p, ch - 1, Pbuf[j & 1]);
      DAMF_HIP(hipEventRecord(c->ev_scatter[(ch - 1) & 3], t));
    }
    const bool tm = timed && j < damf_ctx::kCoreTimed;
    if (tm) DAMF_HIP(hipEventRecord(c->ev_core[2 * j], s));
    chain_core_kernel<<<1, NT, 0, s>>>(p, ch);
    if (tm) {
      DAMF_HIP(hipEventRecord(c->ev_core[2 * j + 1], s));
      c->core_timed = j + 1;
    }
    chain_back_kernel<<<2, NT, 0, s>>>(p, ch, Pbuf[j & 1], Pbuf[(j + 1) & 1]);
    DAMF_HIP(hipEventRecord(c->ev_back[ch & 3], s));
    DAMF_HIP(hipStreamWaitEvent(t, c->ev_back[ch & 3], 0));
  }
  chain_scatter_kernel<<<2, NT, 0, t>>>(p, last - 1, Pbuf[(last - first) & 1]);
  DAMF_HIP(hipEventRecord(c->ev_scatter[(last - 1) & 3], t));
  DAMF_HIP(hipStreamWaitEvent(s, c->ev_scatter[(last - 1) & 3], 0));
  DAMF_HIP(hipGetLastError());
  double *Pc = Pbuf[(last - first) & 1];
  if (Pc != c->P) {
    const int cnt = 2 * c->d * c->d;
    if (graph)
      copy_doubles_kernel<<<(cnt + 255) / 256, 256, 0, s>>>(c->P, Pc, cnt);
    else
      DAMF_HIP(hipMemcpyAsync(c->P, Pc, cnt * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_chain_graph(damf_ctx *c, int n_chunks, const uint64_t *meets, bool *used) {
  *used = false;
  if (n_chunks < 1 || n_chunks > c->cfg.graph_chunks || n_chunks > 64 || c->cfg.kernel_timing)
    return hipSuccess;
  // the captured sequence depends only on the chunk count and on which
  // chunks meet their predecessor and which of those wait for its scatter
  uint64_t bits = 0, hold = 0;
  for (int ch = 1; ch < n_chunks; ++ch) {
    bits |= ((meets[0] >> ch) & 1ull) << ch;
    hold |= ((c->chain_hold[0] >> ch) & 1ull) << ch;
  }
  const auto key = std::make_tuple(bits, hold & bits, n_chunks);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    if (c->graphs.size() >= 256) {
      for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
      c->graphs.clear();
    }
    hipStream_t s = c->stream;
    DAMF_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const hipError_t e = enqueue_chain(c, 0, n_chunks, n_chunks, meets, true);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return e;
    }
    DAMF_HIP(e2);
    hipGraphExec_t x = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    DAMF_HIP(e3);
    it = c->graphs.emplace(key, x).first;
  }
  c->core_timed = 0;
  DAMF_HIP(hipGraphLaunch(it->second, c->stream));
  *used = true;
  return hipSuccess;
}

hipError_t launch_chain(damf_ctx *c, int first, int last, int n_chunks, const uint64_t *meets) {
  if (first >= last) return hipSuccess;
  // The projections alternate between P and Pnext from chunk to chunk,
  // starting from P at chunk `first`.  The solve-and-scatter of chunk ch runs
  // on the scatter stream after chunk ch's back and chunk ch + 1's front, and
  // beside chunk ch + 1's core: that front reads the rows it shares with
  // chunk ch as they were before chunk ch and adds chunk ch's row
  // corrections itself.  The context stream waits for it before the front of
  // chunk ch + 2 (which reads rows it wrote, and whose back reuses chunk ch's
  // P buffer and row-correction parity).  The result is the same as with
  // every step in one stream, up to the rounding of the stored rows.
  return enqueue_chain(c, first, last, n_chunks, meets, false);
}

hipError_t launch_chunk_scatter(damf_ctx *c, int ch, int n_chunks, const double *Pn) {
  const ChainParams p = chain_params(c, n_chunks);
  chain_scatter_kernel<<<2, NT, 0, c->stream>>>(p, ch, Pn);
  return hipGetLastError();
}

}  // namespace damf
