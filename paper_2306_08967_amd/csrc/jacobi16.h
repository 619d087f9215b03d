// jacobi16.h -- FP64 one-sided (Hestenes) Jacobi SVD with each column held
// by a 16-lane row of a wave.
//
// Used for the rank-d t-SVD of the core in Step 2 (Sec. 4.5,
// Rediagonalization; Theorem 2).  Rotating column pairs (a_i, a_j) until all
// columns are orthogonal leaves the singular values as column norms and the
// left singular vectors as normalised columns.
//
// Layout: the NP x NP matrix (NP = 64, 128, 192) is spread over G groups of
// 16 lanes (4 groups per wave).  Group g holds CPG = NP / G columns; lane s of
// the group holds rows s, s + 16, ... (NP / 16 per lane).  A dot product is a
// lane-local sum plus four DPP steps inside the 16-lane row (no LDS).  The
// group's CPG / 2 pairs are (top[p], bottom[p]); the round-robin ("circle")
// schedule shifts tops right and bottoms left across groups after every step
// (top[0] of group 0 stays), so one sweep of NP - 1 steps meets every pair
// once.  Columns cross group boundaries through LDS.  Squared column norms
// live in LDS by column id; the id a slot holds at a given step follows from
// the schedule.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace damf {

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a row, result in every lane of the row.
__device__ __forceinline__ double row_sum16(double x) {
  x += dpp_d<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_d<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_d<0x141>(x);  // row_half_mirror
  x += dpp_d<0x140>(x);  // row_mirror
  return x;
}

__device__ __forceinline__ double row_max16(double x) {
  x = fmax(x, dpp_d<0xB1>(x));
  x = fmax(x, dpp_d<0x4E>(x));
  x = fmax(x, dpp_d<0x141>(x));
  x = fmax(x, dpp_d<0x140>(x));
  return x;
}

// Value of lane P of each 16-lane row, in every lane of the row.
template <int P>
__device__ __forceinline__ double row_bcast(double x) {
  return dpp_d<0x150 + P>(x);  // row_newbcast
}

// 1 / sqrt(x) and 1 / x for normal positive x: the hardware estimates
// refined by two Newton steps each (quadratic convergence from the
// estimate's error to about one ulp).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}

template <int NP_, int G_>
struct J16 {
  static constexpr int NP = NP_;
  static constexpr int G = G_;            // groups of 16 lanes taking part
  static constexpr int RL = NP / 16;      // rows per lane
  static constexpr int CPG = NP / G;      // columns per group
  static constexpr int H = CPG / 2;       // pairs per group
  static constexpr int M = NP / 2;        // pairs in total
  static constexpr int SLOT = NP;         // doubles per exchanged column
  static constexpr int LDS = 2 * G * SLOT + NP;  // exchange (tops, bottoms) + norms
  static_assert(CPG * G == NP && H >= 2, "need >= 2 pairs per group");
};

template <class S>
struct J16Regs {
  double a[S::CPG][S::RL];
};

template <int NP>
__device__ __forceinline__ int circ_id0(int q) {
  constexpr int M = NP / 2;
  return (q < M - 1) ? (q + 1) : (M + (NP - 2 - q));
}
// column id held by global top slot i / bottom slot i after s steps
template <int NP>
__device__ __forceinline__ int j16_top_id(int i, int s) {
  if (i == 0) return 0;
  int q = (i - 1 - s) % (NP - 1);
  if (q < 0) q += NP - 1;
  return circ_id0<NP>(q);
}
template <int NP>
__device__ __forceinline__ int j16_bot_id(int i, int s) {
  int q = (NP - 2 - i - s) % (NP - 1);
  if (q < 0) q += NP - 1;
  return circ_id0<NP>(q);
}

// column id of local slot c of group g at a sweep boundary
template <class S>
__device__ __forceinline__ int j16_col(int g, int c) {
  return (c < S::H) ? (g * S::H + c) : (S::M + g * S::H + (c - S::H));
}

template <class S>
__device__ __forceinline__ double j16_norm2(const double (&col)[S::RL]) {
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < S::RL; ++r) s = fma(col[r], col[r], s);
  return row_sum16(s);
}

// Sweeps until one applies no rotation or all its rotations were below
// sqrt(tol) (or max_sweeps); returns the sweep count.  lds_flag points to 4
// ints of LDS.  A pair is rotated when |a_i . a_j| > tol ||a_i|| ||a_j|| and
// neither column is numerically zero (norm^2 below 1e-30 of the largest).
// Every thread of the workgroup calls it; groups >= G only join barriers.
// On return the squared norms are in lds[2 * G * NP + id].
template <class S>
__device__ int jacobi16_sweeps(J16Regs<S> &J, double *lds, int *lds_flag, int max_sweeps,
                               double tol) {
  constexpr int NP = S::NP, G = S::G, RL = S::RL, CPG = S::CPG, H = S::H, SLOT = S::SLOT;
  const int lane = threadIdx.x & 63;
  const int sl = lane & 15;
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 4 + (lane >> 4);
  const bool active = grp < G;
  double *xt = lds;               // last top of group g -> group g + 1
  double *xb = lds + G * SLOT;    // first bottom of group g -> group g - 1
  double *nrm = lds + 2 * G * SLOT;
  if (active) {
#pragma unroll
    for (int c = 0; c < CPG; ++c) {
      const double v = j16_norm2<S>(J.a[c]);
      if (sl == 0) nrm[j16_col<S>(grp, c)] = v;
    }
  }
  __syncthreads();
  int sweeps = 0;
  const double tol2 = tol * tol, conv2 = tol;  // (sqrt(tol))^2
  int big = 0;  // some pair had |a_i . a_j| >= sqrt(tol) ||a_i|| ||a_j|| this sweep
  for (; sweeps < max_sweeps; ++sweeps) {
    int rot = 0;
    big = 0;
    double mx = 0.0;
    for (int j = sl; j < NP; j += 16) mx = fmax(mx, nrm[j]);
    mx = row_max16(mx);
    const double floor2 = 1e-30 * mx;
    for (int step = 0; step < NP - 1; ++step) {
      if (active) {
        double g[H];
#pragma unroll
        for (int p = 0; p < H; ++p) {
          double s = 0.0;
#pragma unroll
          for (int r = 0; r < RL; ++r) s = fma(J.a[p][r], J.a[H + p][r], s);
          g[p] = row_sum16(s);
        }
        // lane p < H of the group computes pair p's rotation
        double myg = g[0];
#pragma unroll
        for (int p = 1; p < H; ++p) myg = (sl == p) ? g[p] : myg;
        const int pp = (sl < H) ? sl : 0;
        const int it = j16_top_id<NP>(grp * H + pp, step);
        const int ib = j16_bot_id<NP>(grp * H + pp, step);
        const double al = nrm[it], be = nrm[ib];
        const bool live = (sl < H) && al > floor2 && be > floor2;
        const double g2 = myg * myg, ab = al * be;
        const bool doit = live && g2 > tol2 * ab;
        big |= (live && g2 >= conv2 * ab) ? 1 : 0;
        // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (be - al) / (2 g),
        // as sign(be - al) 2g / (|be - al| + sqrt((be - al)^2 + 4 g^2))
        const double dd = be - al, gg = doit ? 2.0 * myg : 0.0;
        const double q2 = fma(dd, dd, gg * gg);
        const double den = fabs(dd) + q2 * rsqrt_nr(q2);
        const double t = doit ? (dd >= 0.0 ? gg : -gg) * rcp_nr(den) : 0.0;
        const double cs = rsqrt_nr(fma(t, t, 1.0));
        const double sn = cs * t;
        if (doit) {
          nrm[it] = fma(-t, myg, al);
          nrm[ib] = fma(t, myg, be);
        }
        rot += doit ? 1 : 0;
#pragma unroll
        for (int p = 0; p < H; ++p) {
          double c, s;
          if (p == 0) {
            c = row_bcast<0>(cs);
            s = row_bcast<0>(sn);
          } else if (p == 1) {
            c = row_bcast<1>(cs);
            s = row_bcast<1>(sn);
          } else if (p == 2) {
            c = row_bcast<2>(cs);
            s = row_bcast<2>(sn);
          } else {
            c = row_bcast<3>(cs);
            s = row_bcast<3>(sn);
          }
#pragma unroll
          for (int r = 0; r < RL; ++r) {
            const double x = J.a[p][r], y = J.a[H + p][r];
            J.a[p][r] = c * x - s * y;
            J.a[H + p][r] = s * x + c * y;
          }
        }
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          xt[grp * SLOT + r * 16 + sl] = J.a[H - 1][r];
          xb[grp * SLOT + r * 16 + sl] = J.a[H][r];
        }
      }
      __syncthreads();
      if (active) {
#pragma unroll
        for (int p = H - 1; p >= 2; --p) {
#pragma unroll
          for (int r = 0; r < RL; ++r) J.a[p][r] = J.a[p - 1][r];
        }
        if (grp == 0) {
#pragma unroll
          for (int r = 0; r < RL; ++r) J.a[1][r] = xb[r * 16 + sl];  // own first bottom
        } else {
#pragma unroll
          for (int r = 0; r < RL; ++r) {
            J.a[1][r] = J.a[0][r];
            J.a[0][r] = xt[(grp - 1) * SLOT + r * 16 + sl];
          }
        }
#pragma unroll
        for (int p = 0; p < H - 1; ++p) {
#pragma unroll
          for (int r = 0; r < RL; ++r) J.a[H + p][r] = J.a[H + p + 1][r];
        }
        if (grp == G - 1) {
#pragma unroll
          for (int r = 0; r < RL; ++r) J.a[CPG - 1][r] = xt[grp * SLOT + r * 16 + sl];  // own last top
        } else {
#pragma unroll
          for (int r = 0; r < RL; ++r) J.a[CPG - 1][r] = xb[(grp + 1) * SLOT + r * 16 + sl];
        }
      }
      __syncthreads();
    }
    // exact norms; stop when no group rotated in this sweep
    if (active) {
#pragma unroll
      for (int c = 0; c < CPG; ++c) {
        const double v = j16_norm2<S>(J.a[c]);
        if (sl == 0) nrm[j16_col<S>(grp, c)] = v;
      }
    }
    // Stop when no pair rotated, or when every rotation of this sweep was
    // below sqrt(tol): Jacobi converges quadratically, so the off-diagonal
    // left after such a sweep is O(tol) and another sweep would find nothing.
    if (threadIdx.x == 0) {
      lds_flag[0] = 0;
      lds_flag[1] = 0;
    }
    __syncthreads();
    if (rot > 0) atomicAdd(lds_flag, rot);
    if (big) atomicOr(lds_flag + 1, 1);
    __syncthreads();
    const int total = lds_flag[0], any_big = lds_flag[1];
    __syncthreads();
    if (total == 0 || !any_big) {
      ++sweeps;
      break;
    }
  }
  return sweeps;
}

}  // namespace damf
