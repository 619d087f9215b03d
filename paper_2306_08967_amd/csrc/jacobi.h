// jacobi.h -- FP64 one-sided (Hestenes) Jacobi SVD of a small matrix held in
// the VGPRs of one workgroup of NW waves.
//
// Step 2 of the update (Sec. 4.5, Rediagonalization; Theorem 2) needs the
// full t-SVD of a (d + k) x (d + k) core.  One-sided Jacobi applies plane
// rotations to column pairs (a_i, a_j) until all columns are mutually
// orthogonal; the column norms are then the singular values and the
// normalised columns the left singular vectors.
//
// Layout: the matrix is padded to NP = 64 * RPL rows and columns.  Each wave
// holds CPW = NP / NW columns; lane l holds rows l, l + 64, ... of each.
// Columns pair up as (top[p], bottom[p]) under the round-robin ("circle")
// schedule: after each step tops shift right, bottoms shift left and top[0]
// stays, so one sweep of NP - 1 steps meets every pair once.  Columns cross
// wave boundaries through double-buffered LDS slots (one barrier per step).
// Squared column norms live in LDS, indexed by column id; the id held by a
// slot at a given step follows from the schedule, so it costs no registers.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace damf {

template <int RPL, int NW>
struct JacobiShape {
  static constexpr int NP = 64 * RPL;
  static constexpr int CPW = NP / NW;  // columns per wave
  static constexpr int H = CPW / 2;    // pairs per wave
  static constexpr int M = NP / 2;     // pairs in total
  static constexpr int SLOT = NP;      // doubles per exchanged column
  // LDS doubles: exchange buffers (2 parities x 2 directions x NW) + norms
  static constexpr int LDS = 2 * 2 * NW * SLOT + NP;
  static_assert(CPW % 2 == 0 && H >= 2, "need at least two pairs per wave");
};

template <int RPL, int NW>
struct JacobiRegs {
  double a[JacobiShape<RPL, NW>::CPW][RPL];
};

// Column id (initial column index) held by top slot i / bottom slot i after
// `s` steps.  The NP - 1 movable positions form a circle: position q < M - 1
// is top[q + 1], position q >= M - 1 is bottom[NP - 2 - q]; every step moves
// each element one position forward.  Initially top[i] holds column i and
// bottom[i] holds column M + i.
template <int NP>
__device__ __forceinline__ int circle_id0(int q) {
  constexpr int M = NP / 2;
  return (q < M - 1) ? (q + 1) : (M + (NP - 2 - q));
}
template <int NP>
__device__ __forceinline__ int top_id(int i, int s) {
  if (i == 0) return 0;
  int q = (i - 1 - s) % (NP - 1);
  if (q < 0) q += NP - 1;
  return circle_id0<NP>(q);
}
template <int NP>
__device__ __forceinline__ int bot_id(int i, int s) {
  int q = (NP - 2 - i - s) % (NP - 1);
  if (q < 0) q += NP - 1;
  return circle_id0<NP>(q);
}

// Global column id of local slot c of wave w at a sweep boundary.
template <int RPL, int NW>
__device__ __forceinline__ int jacobi_slot_col(int w, int c) {
  using S = JacobiShape<RPL, NW>;
  return (c < S::H) ? (w * S::H + c) : (S::M + w * S::H + (c - S::H));
}

template <int RPL>
__device__ __forceinline__ double col_norm2(const double (&col)[RPL]) {
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < RPL; ++r) s = fma(col[r], col[r], s);
  return wave_sum(s);
}

// Runs sweeps until a sweep applies no rotation (or max_sweeps).  A pair is
// rotated when |a_i . a_j| > tol ||a_i|| ||a_j|| and neither column is
// numerically zero.  Returns
// the number of sweeps; on return the squared column norms are in
// lds[4 * NW * NP + id].  All NW * 64 threads must call it.
template <int RPL, int NW>
__device__ int jacobi_sweeps(JacobiRegs<RPL, NW> &J, double *lds, int *lds_flag,
                             int max_sweeps, double tol) {
  using S = JacobiShape<RPL, NW>;
  constexpr int CPW = S::CPW, H = S::H, NP = S::NP, SLOT = S::SLOT;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  double *nrm = lds + 4 * NW * SLOT;
  int sweeps = 0;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const double v = col_norm2<RPL>(J.a[c]);
    if (lane == 0) nrm[jacobi_slot_col<RPL, NW>(w, c)] = v;
  }
  __syncthreads();
  for (; sweeps < max_sweeps; ++sweeps) {
    int rot = 0;
    // columns below 1e-15 of the largest column norm are numerically zero:
    // rotating them only moves rounding noise (a core with more columns than
    // rows, or a rank-deficient one, has such columns)
    double mx = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) mx = fmax(mx, nrm[r * 64 + lane]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    const double floor2 = 1e-30 * mx;
    for (int step = 0; step < NP - 1; ++step) {
      // ---- rotate the H local pairs
      double g[H];
#pragma unroll
      for (int p = 0; p < H; ++p) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) s = fma(J.a[p][r], J.a[H + p][r], s);
        g[p] = s;
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int p = 0; p < H; ++p) g[p] += __shfl_xor(g[p], off, 64);
      }
      // lane p < H computes the rotation of pair p, then broadcasts it
      double myg = g[0];
#pragma unroll
      for (int p = 1; p < H; ++p) myg = (lane == p) ? g[p] : myg;
      double cs = 1.0, sn = 0.0;
      bool doit = false;
      if (lane < H) {
        const int it = top_id<NP>(w * H + lane, step);
        const int ib = bot_id<NP>(w * H + lane, step);
        const double al = nrm[it], be = nrm[ib];
        doit = al > floor2 && be > floor2 && fabs(myg) > tol * sqrt(al * be);
        if (doit) {
          const double zeta = (be - al) / (2.0 * myg);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          cs = 1.0 / sqrt(1.0 + t * t);
          sn = cs * t;
          nrm[it] = al - t * myg;
          nrm[ib] = be + t * myg;
        }
      }
      rot += __popcll(__ballot(doit));
#pragma unroll
      for (int p = 0; p < H; ++p) {
        const double c = __shfl(cs, p, 64), sgn = __shfl(sn, p, 64);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const double x = J.a[p][r], y = J.a[H + p][r];
          J.a[p][r] = c * x - sgn * y;
          J.a[H + p][r] = sgn * x + c * y;
        }
      }
      // ---- circle move across waves
      double *buf = lds + (step & 1) * (2 * NW * SLOT);
      double *xt = buf;                // last top of wave w -> wave w + 1
      double *xb = buf + NW * SLOT;    // first bottom of wave w -> wave w - 1
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        xt[w * SLOT + r * 64 + lane] = J.a[H - 1][r];
        xb[w * SLOT + r * 64 + lane] = J.a[H][r];
      }
      __syncthreads();
      double lastTop[RPL], firstBot[RPL];
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        lastTop[r] = J.a[H - 1][r];
        firstBot[r] = J.a[H][r];
      }
#pragma unroll
      for (int p = H - 1; p >= 2; --p) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) J.a[p][r] = J.a[p - 1][r];
      }
      if (w == 0) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) J.a[1][r] = firstBot[r];
      } else {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          J.a[1][r] = J.a[0][r];
          J.a[0][r] = xt[(w - 1) * SLOT + r * 64 + lane];
        }
      }
#pragma unroll
      for (int p = 0; p < H - 1; ++p) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) J.a[H + p][r] = J.a[H + p + 1][r];
      }
      if (w == NW - 1) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) J.a[CPW - 1][r] = lastTop[r];
      } else {
#pragma unroll
        for (int r = 0; r < RPL; ++r) J.a[CPW - 1][r] = xb[(w + 1) * SLOT + r * 64 + lane];
      }
    }
    // refresh norms exactly; stop when no wave rotated in this sweep
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double v = col_norm2<RPL>(J.a[c]);
      if (lane == 0) nrm[jacobi_slot_col<RPL, NW>(w, c)] = v;
    }
    if (threadIdx.x == 0) *lds_flag = 0;
    __syncthreads();
    if (lane == 0 && rot > 0) atomicAdd(lds_flag, rot);  // rot is wave-uniform
    __syncthreads();
    const int total = *lds_flag;
    __syncthreads();
    if (total == 0) {
      ++sweeps;
      break;
    }
  }
  return sweeps;
}

}  // namespace damf
