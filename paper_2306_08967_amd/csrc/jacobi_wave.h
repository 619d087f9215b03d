// jacobi_wave.h -- FP64 one-sided (Hestenes) Jacobi SVD with column blocks
// owned by waves and rows spread over the lanes.
//
// Used for the rank-d t-SVD of the core in Step 2 (Sec. 4.5,
// Rediagonalization; Theorem 2).  Rotating column pairs (a_i, a_j) until all
// columns are orthogonal leaves the singular values as column norms and the
// left singular vectors as normalised columns.
//
// Layout: the NP x NP matrix (NP = 64, 128, 192) is cut into 16 half-blocks of
// B = NP / 16 columns.  Each of the 8 waves of the workgroup holds two of them
// (a "top" and a "bottom" half-block, 2B columns) in VGPRs; lane l holds rows
// l, l + 64, l + 128 of every column.  A sweep has 15 rounds: the half-blocks
// follow the round-robin ("circle") schedule over the waves, so every pair of
// half-blocks shares a wave in exactly one round.  In a round a wave rotates the
// B x B cross pairs of its two half-blocks (B steps of B disjoint pairs, the
// bottom block turned by one column per step); in round 0 it instead runs a
// circle over all its 2B columns, which also covers the pairs inside each
// half-block.  Each step needs only wave-level communication: the B dot
// products are reduced across the 64 lanes by lane swaps (reduce-scatter) and
// DPP, the pair's rotation is computed by the lane that ends up with its dot
// product, and read back by every lane from LDS.  Half-blocks move between
// waves through LDS only between rounds (4 workgroup barriers per round).
// Squared column norms (with the column scales below, as pairs, and the
// scales' reciprocals) live in LDS by column id; a wave touches only those of
// the columns it holds.
//
// Rotations are applied in scaled form: column i is held as x_i with a scale
// d_i (a_i = d_i x_i, scales in LDS by id).  The rotation (c, s = c t) of the
// pair (a_i' = c a_i - s a_j, a_j' = s a_i + c a_j) becomes two in-place shears,
// x_j <- x_j + t (d_i / d_j) x_i, then x_i <- x_i - c^2 t (d_j / d_i) x_j with the
// new x_j, and d_j <- c d_j, d_i <- d_i / c: two FMAs per row and no copies.  A
// scale changes by at most sqrt 2 per rotation (|t| <= 1) and the scales are
// folded back into the columns after every sweep.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "common.h"
#include "wave_ops.h"

namespace damf {

template <int NP_, int NW_ = 8>
struct JW {
  static constexpr int NP = NP_;
  static constexpr int NW = NW_;           // waves
  static constexpr int B = NP / (2 * NW);  // columns per half-block
  static constexpr int C = 2 * B;          // columns per wave
  static constexpr int RPL = NP / 64;      // rows per lane
  // reduction of B values: the first lane-swap stage leaves H per lane, the
  // second QF full slots (one pair per 16-lane row each) and, for odd H, one
  // leftover slot (rows 0 and 2)
  static constexpr int H = B / 2;
  static constexpr int QF = H / 2, QL = H % 2, QS = QF + QL;
  static constexpr int XU = B;  // cross steps per loop iteration: all of a round
  static constexpr int SLOT = B * NP;      // doubles per half-block in the exchange buffer
  static constexpr int NS_OFF = NW * SLOT;      // per column id: JNs
  static constexpr int BC_OFF = NS_OFF + 4 * NP;  // per wave: B rotation factor pairs
  static constexpr int LDS = BC_OFF + NW * 2 * B;  // exchange, norms, scales, factors
  static_assert(NP % 64 == 0 && NP <= 192 && B % 2 == 0 && B * 2 * NW == NP,
                "NP must be 64, 128 or 192 and split into 2 NW half-blocks of even width");
};

// Per column id: the squared norm of a_i = d_i x_i, the scale d_i and 1 / d_i.
struct __align__(16) JNs {
  double n2, d, rd, pad;
};

// squared norm of column id after jw_sweeps
template <class S>
__device__ __forceinline__ double jw_norm2(const double *lds, int id) {
  return lds[S::NS_OFF + 4 * id];
}

template <class S>
struct JWRegs {
  double a[S::C][S::RPL];
};

// column id held by slot c of wave w at a sweep boundary
template <class S>
__device__ __forceinline__ int jw_col(int w, int c) {
  return (c < S::B) ? (w * S::B + c) : ((S::NW + w) * S::B + (c - S::B));
}

// Lanes l < 32 get x[l] + x[l + 32]; lanes l >= 32 get y[l - 32] + y[l].
__device__ __forceinline__ double xsum32(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
// 16-lane rows 0, 1, 2, 3 get x0 + x1, y0 + y1, x2 + x3, y2 + y3 (row sums lane by lane).
__device__ __forceinline__ double xsum16(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double wave_max_d(double x) {
  x = row_max16(x);
  {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(x), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(x), false, false);
    x = fmax(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
  }
  {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(x), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(x), false, false);
    x = fmax(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
  }
  return x;
}

// Index of the pair whose wave total lands in slot q of 16-lane row `row`;
// slot q is held by the four lanes 4 q .. 4 q + 3 of the row, and the first
// of them ("plane" lane) computes the pair's rotation.
template <class S>
__device__ __forceinline__ int jw_pair(int row, int q) {
  return q + (row & 1) * S::QF + (row >> 1) * S::H;
}
__device__ __forceinline__ int jw_slot(int lane) { return (lane >> 2) & 3; }
template <class S>
__device__ __forceinline__ bool jw_plane(int lane) {
  return (lane & 3) == 0 && jw_slot(lane) < S::QF;
}

// v[p] (p < B): per-lane partial sums.  Returns, in the four lanes of slot q
// of 16-lane row R, the wave total of v[jw_pair(R, q)] (q < QF; lanes of
// slots QF .. 3 return zero or partial sums).  Lane swaps across the halves
// and quarters of the wave (permlane32 / permlane16 swaps), then a reduce-
// scatter inside each row: lanes l and l ^ 8 keep two slots each (DPP
// row_ror:8), lanes l and 7 - l of each half-row one each (row_half_mirror),
// and a quad sum.
template <class S>
__device__ __forceinline__ double jw_reduce(const double (&v)[S::B]) {
  constexpr int H = S::H, QF = S::QF;
  static_assert(S::QL == 0 && QF >= 1 && QF <= 4, "even half count, at most four slots a row");
  double h[H];
#pragma unroll
  for (int p = 0; p < H; ++p) h[p] = xsum32(v[p], v[p + H]);
  double q[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] = (i < QF) ? xsum16(h[i], h[i + QF]) : 0.0;
  const int lane = threadIdx.x & 63;
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
  // slots 0, 1 stay in the lanes without bit 3, slots 2, 3 in the others; a
  // slot at or past QF holds nothing, so what its lanes keep or send is free
  // (no select)
  const double s0 = (QF > 2 && !b3) ? q[2] : q[0], s1 = (QF > 3 && !b3) ? q[3] : q[1];
  double k0 = (QF > 2 && b3) ? q[2] : q[0], k1 = (QF > 3 && b3) ? q[3] : q[1];
  k0 += dpp_d<0x128>(s0);  // row_ror:8, lane l ^ 8
  k1 += dpp_d<0x128>(s1);
  // the even slot stays in the lanes without bit 2 (row_half_mirror pairs
  // lane l with 7 - l, which has bit 2 flipped)
  const double sb = (QF > 1 && !b2) ? k1 : k0;
  double kb = (QF > 1 && b2) ? k1 : k0;
  kb += dpp_d<0x141>(sb);
  kb += dpp_d<0xB1>(kb);  // quad_perm [1,0,3,2]
  kb += dpp_d<0x4E>(kb);  // quad_perm [2,3,0,1]
  return kb;
}

// Exact squared norms of the wave's 2B columns into ns[].x by column id (the
// wave holds its sweep-boundary half-blocks w and NW + w).
template <class S>
__device__ __forceinline__ void jw_norms(const JWRegs<S> &J, JNs *ns, int w) {
  constexpr int B = S::B, RPL = S::RPL;
  const int lane = threadIdx.x & 63, row = lane >> 4;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    double v[B];
#pragma unroll
    for (int p = 0; p < B; ++p) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) s = fma(J.a[half * B + p][r], J.a[half * B + p][r], s);
      v[p] = s;
    }
    const double mine = jw_reduce<S>(v);
    if (jw_plane<S>(lane)) ns[jw_col<S>(w, half * B + jw_pair<S>(row, jw_slot(lane)))].n2 = mine;
  }
}

// Pair maps: pair p of a step rotates slots PM::a(p) and PM::b(p).
// Cross: top slot p with bottom slot (p + SH) mod B.  Intra: the pairs of a circle inside
// each half-block (top half-block pairs first, then the bottom one).
template <class S, int SH = 0>
struct JWCross {
  static constexpr int a(int p) { return p; }
  static constexpr int b(int p) { return S::B + (p + SH) % S::B; }
};
template <class S>
struct JWIntra {
  static constexpr int H = S::B / 2;
  static constexpr int a(int p) { return (p < H) ? p : S::B + (p - H); }
  static constexpr int b(int p) { return (p < H) ? H + p : S::B + H + (p - H); }
};

// One step: rotate the B disjoint pairs (slot PM::a(p), slot PM::b(p)).
// ids(p, it, ib) gives the column ids the two slots of pair p hold.  bc: the
// wave's B (t1, t2) slots in LDS; the lane that computes a pair's rotation
// writes it there and every lane reads all B back (broadcast reads; LDS
// operations of one wave complete in order).
template <class S, class PM, class IdF>
__device__ __forceinline__ void jw_step(JWRegs<S> &J, JNs *ns, double2 *bc,
                                        double floor2, double tol2, double conv2, IdF ids, int &rot,
                                        int &big, int &skip) {
  constexpr int B = S::B, RPL = S::RPL;
  const int lane = threadIdx.x & 63, row = lane >> 4;
  double v[B];
#pragma unroll
  for (int p = 0; p < B; ++p) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) s = fma(J.a[PM::a(p)][r], J.a[PM::b(p)][r], s);
    v[p] = s;
  }
  // the plane lane of slot q of row R computes the rotation of pair jw_pair(R, q)
  const double myg = jw_reduce<S>(v);
  const bool plane = jw_plane<S>(lane);
  int pair = plane ? jw_pair<S>(row, jw_slot(lane)) : 0;
  // an opaque copy per step: the pair's column ids are then formed here
  // (a few integer ops) instead of being kept live across the unrolled round
  asm volatile("" : "+v"(pair));
  int it, ib;
  ids(pair, it, ib);
  const double al = ns[it].n2, be = ns[ib].n2;
  const double di = ns[it].d, dj = ns[ib].d;
  const double rdi = ns[it].rd, rdj = ns[ib].rd;
  const double gt = myg * (di * dj);  // a_i . a_j
  const bool live = plane && al > floor2 && be > floor2;
  const double g2 = gt * gt, ab = al * be;
  const bool doit = live && g2 > tol2 * ab;
  rot += doit ? 1 : 0;
  // a step in which no pair rotates would only add zeros (t = 0): skip its
  // rotation parameters and shears; finite results are unchanged bit for bit
  const bool none = __builtin_amdgcn_ballot_w64(doit) == 0;  // uniform over the wave
  skip += none ? 1 : 0;
  if (none) return;
  // a pair above sqrt(tol) is above tol too (tol < 1), so only steps that
  // rotate can set big
  big |= (live && g2 >= conv2 * ab) ? 1 : 0;
  // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (be - al) / (2 g),
  // as sign(be - al) 2g / (|be - al| + sqrt((be - al)^2 + 4 g^2)); a pair
  // that does not rotate gets t = 0 (its den may be 0)
  const double dd = be - al, gg = 2.0 * gt;
  // t itself needs no more than about 1e-14 (any angle near the optimal one
  // shrinks the pair's inner product quadratically); c = (1 + t^2)^-1/2 is
  // formed from this t with one Newton step as well, which keeps each
  // rotation orthogonal to about 1e-14 (the columns' exact norms are taken
  // again after every sweep; a second step changed none of the C2 accuracy
  // figures)
  const double q2 = fma(dd, dd, gg * gg);
  const double den = fabs(dd) + q2 * rsqrt_nr1(q2);
  const double t = doit ? gg * __builtin_copysign(rcp_nr1(den), dd) : 0.0;
  const double q1 = fma(t, t, 1.0);
  const double cs = rsqrt_nr1(q1);
  // two in-place shears: x_j += t (d_i / d_j) x_i, then x_i -= c^2 t (d_j / d_i) x_j
  // (the new x_j), with d_j <- c d_j and d_i <- d_i / c (1 / c = (1 + t^2) c);
  // the scales' reciprocals are carried along, so no division is needed
  const double t2 = t * (di * rdj), t1 = ((cs * cs) * t) * (dj * rdi);
  if (doit) {
    const double ic = q1 * cs;
    ns[it].n2 = fma(-t, gt, al);
    ns[it].d = di * ic;
    ns[it].rd = rdi * cs;
    ns[ib].n2 = fma(t, gt, be);
    ns[ib].d = cs * dj;
    ns[ib].rd = rdj * ic;
  }
  if (plane) bc[pair] = make_double2(t1, t2);
  __builtin_amdgcn_wave_barrier();
  // the factor pairs are requested in two halves, each in one LDS round trip
  // (the compiler otherwise reuses a few registers and waits once per pair of
  // pairs; all B at once would spill), then consumed in order
  constexpr int BH = B / 2;
  double2 u[B];
#pragma unroll
  for (int p = 0; p < BH; ++p) u[p] = bc[p];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int p = 0; p < B; ++p) {
    if (p == BH) {
#pragma unroll
      for (int q = BH; q < B; ++q) u[q] = bc[q];
      __builtin_amdgcn_sched_barrier(0);
    }
    const double u1 = u[p].x, u2 = u[p].y;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      J.a[PM::b(p)][r] = fma(u2, J.a[PM::a(p)][r], J.a[PM::b(p)][r]);
      J.a[PM::a(p)][r] = fma(-u1, J.a[PM::b(p)][r], J.a[PM::a(p)][r]);
    }
  }
}

// circle move inside each half-block (B slots: B/2 tops, then B/2 bottoms):
// top p <- top p-1 (p >= 2), top 1 <- bottom 0, bottom p <- bottom p+1,
// last bottom <- last top
template <class S>
__device__ __forceinline__ void jw_intra_move(JWRegs<S> &J) {
  constexpr int B = S::B, H = B / 2, RPL = S::RPL;
  if (B == 2) return;  // a circle of two columns has one step and no move
#pragma unroll
  for (int o = 0; o < 2 * B; o += B) {
    double b0[RPL], tl[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      b0[r] = J.a[o + H][r];
      tl[r] = J.a[o + H - 1][r];
    }
#pragma unroll
    for (int p = H - 1; p >= 2; --p) {
#pragma unroll
      for (int r = 0; r < RPL; ++r) J.a[o + p][r] = J.a[o + p - 1][r];
    }
    if (H >= 2) {
#pragma unroll
      for (int r = 0; r < RPL; ++r) J.a[o + 1][r] = b0[r];
    }
#pragma unroll
    for (int p = 0; p < H - 1; ++p) {
#pragma unroll
      for (int r = 0; r < RPL; ++r) J.a[o + H + p][r] = J.a[o + H + p + 1][r];
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) J.a[o + B - 1][r] = tl[r];
  }
}

// turn the bottom half-block by K columns: bottom p <- bottom p+K (mod B)
template <class S, int K>
__device__ __forceinline__ void jw_cross_move(JWRegs<S> &J) {
  constexpr int B = S::B, RPL = S::RPL;
  if (K % B == 0) return;
  double keep[K][RPL];
#pragma unroll
  for (int q = 0; q < K; ++q) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) keep[q][r] = J.a[B + q][r];
  }
#pragma unroll
  for (int p = 0; p < B - K; ++p) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) J.a[B + p][r] = J.a[B + p + K][r];
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) J.a[2 * B - K + q][r] = keep[q][r];
  }
}

template <class S>
__device__ __forceinline__ void jw_put(const JWRegs<S> &J, double *xb, int slot, int c0, int lane) {
#pragma unroll
  for (int j = 0; j < S::B; ++j) {
#pragma unroll
    for (int r = 0; r < S::RPL; ++r) xb[slot * S::SLOT + j * S::NP + r * 64 + lane] = J.a[c0 + j][r];
  }
}
template <class S>
__device__ __forceinline__ void jw_get(JWRegs<S> &J, const double *xb, int slot, int c0, int lane) {
#pragma unroll
  for (int j = 0; j < S::B; ++j) {
#pragma unroll
    for (int r = 0; r < S::RPL; ++r) J.a[c0 + j][r] = xb[slot * S::SLOT + j * S::NP + r * 64 + lane];
  }
}

// Move the half-blocks to the next round of the circle over waves:
// new top[w] = old top[w-1] (w >= 2), new top[1] = old bottom[0], top[0] stays;
// new bottom[w] = old bottom[w+1] (w < NW-1), new bottom[NW-1] = old top[NW-1].
// Bottoms go through slot w - 1 (wave 0's through slot L), tops of waves
// 1 .. L-1 through slot w.  Two barriers suffice: a slot is next written by
// the wave that last read it, except slot 0 (read by wave 0, written by wave
// 1) and slot L (read by wave 1, written by wave 0), whose reads both come
// before the second barrier.
template <class S>
__device__ __forceinline__ void jw_exchange(JWRegs<S> &J, double *xb, int w, int lane) {
  constexpr int B = S::B, RPL = S::RPL;
  constexpr int L = S::NW - 1;
  jw_put<S>(J, xb, (w == 0) ? L : w - 1, B, lane);  // bottoms, by destination wave
  __syncthreads();
  if (w < L) {
    jw_get<S>(J, xb, w, B, lane);
  } else {
#pragma unroll
    for (int j = 0; j < B; ++j) {
#pragma unroll
      for (int r = 0; r < RPL; ++r) J.a[B + j][r] = J.a[j][r];
    }
  }
  if (w >= 1 && w < L) jw_put<S>(J, xb, w, 0, lane);  // tops of waves 1..NW-2, by source wave
  if (w == 1) jw_get<S>(J, xb, L, 0, lane);
  __syncthreads();
  if (w >= 2) jw_get<S>(J, xb, w - 1, 0, lane);
}

// Issue priority through a round: the two waves that share a SIMD run the
// same steps, and with equal priorities the older one always wins the issue
// slot, finishes its round first and idles at the exchange while the other
// runs alone.  Priority falls with the step (3 for the first quarter of a
// round's cross steps, down to 0 for the last), so the wave that is behind
// wins instead.  Per C2 chunk: steps 513 / 805 us on the older / younger
// waves with no priorities, 670 / 750 with the falling priority.
template <int SH, int B>
__device__ __forceinline__ void jw_prio() {
  constexpr int Q = (B >= 4) ? B / 4 : 1;
  if constexpr (SH % Q == 0) __builtin_amdgcn_s_setprio(3 - (SH / Q < 3 ? SH / Q : 3));
}

// Steps sh .. sh + U - 1 of a cross round, the bottom offset by 0 .. U - 1 slots.
template <class S, int U, int... SH>
__device__ __forceinline__ void jw_cross_steps(JWRegs<S> &J, JNs *ns, double2 *bc, double floor2,
                                               double tol2, double conv2, int ht, int hb, int sh,
                                               int &rot, int &big, int &skip,
                                               std::integer_sequence<int, SH...>) {
  constexpr int B = S::B;
  ((jw_prio<SH, B>(),
    jw_step<S, JWCross<S, SH>>(J, ns, bc, floor2, tol2, conv2,
                               [&](int p, int &it, int &ib) {
                                 int q = p + sh + SH;
                                 if (q >= B) q -= B;
                                 it = ht * B + p;
                                 ib = hb * B + q;
                               },
                               rot, big, skip)),
   ...);
}

// Sweeps until one applies no rotation or all its rotations were below
// sqrt(tol) (or max_sweeps); returns the sweep count.  lds_flag points to 3
// ints of LDS; the third, cleared by the caller, counts the steps (over all
// waves) in which no pair rotated and whose shears were skipped.  A pair is rotated when |a_i . a_j| > tol ||a_i|| ||a_j|| and
// neither column is numerically zero (norm^2 below 1e-30 of the largest).
// Every thread of the 64 NW-thread workgroup calls it; on return the columns
// are back in their sweep-boundary slots (jw_col) and the squared norms are
// in lds[S::NS_OFF + 4 id] (jw_norm2).
template <class S>
__device__ __forceinline__ int jw_sweeps(JWRegs<S> &J, double *lds, int *lds_flag, int max_sweeps, double tol) {
  int skip = 0;  // this wave's steps without a rotation
  constexpr int B = S::B, RPL = S::RPL, XU = S::XU;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double *xb = lds;
  JNs *ns = reinterpret_cast<JNs *>(lds + S::NS_OFF);
  double2 *bc = reinterpret_cast<double2 *>(lds + S::BC_OFF) + w * B;
  for (int j = threadIdx.x; j < S::NP; j += blockDim.x) ns[j].d = ns[j].rd = 1.0;
  jw_norms<S>(J, ns, w);
  __syncthreads();
  const double tol2 = tol * tol, conv2 = tol;  // (sqrt(tol))^2
  int sweeps = 0;
  for (; sweeps < max_sweeps; ++sweeps) {
    int rot = 0, big = 0;
    double mx = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) mx = fmax(mx, ns[r * 64 + lane].n2);
    const double floor2 = 1e-30 * wave_max_d(mx);
    for (int round = 0; round < 2 * S::NW - 1; ++round) {
      const int ht = j16_top_id<2 * S::NW>(w, round), hb = j16_bot_id<2 * S::NW>(w, round);
      if (round == 0) {
        __builtin_amdgcn_s_setprio(3);
        // pairs inside each of the two half-blocks: a circle of B - 1 steps in each
        for (int st = 0; st < B - 1; ++st) {
          jw_step<S, JWIntra<S>>(J, ns, bc, floor2, tol2, conv2,
                                 [&](int p, int &it, int &ib) {
                                   const int i = (p < B / 2) ? p : p - B / 2;
                                   const int h = (p < B / 2) ? ht : hb;
                                   it = h * B + j16_top_id<B>(i, st);
                                   ib = h * B + j16_bot_id<B>(i, st);
                                 },
                                 rot, big, skip);
          jw_intra_move<S>(J);
        }
      }
      // cross pairs of the two half-blocks: B steps, XU per iteration (step u
      // with the bottom offset by u slots), then the bottom turned by XU
      for (int sh = 0; sh < B; sh += XU) {
        jw_cross_steps<S, XU>(J, ns, bc, floor2, tol2, conv2, ht, hb, sh, rot, big, skip,
                              std::make_integer_sequence<int, XU>{});
        jw_cross_move<S, XU>(J);
      }
      jw_exchange<S>(J, xb, w, lane);
    }
    // fold the scales into the columns (each wave its own sweep-boundary
    // columns), then exact norms; stop when no pair rotated in this sweep, or
    // when every rotation of this sweep was below sqrt(tol): Jacobi converges
    // quadratically, so the off-diagonal left after such a sweep is O(tol)
    // and another sweep would find nothing.
#pragma unroll
    for (int c = 0; c < S::C; ++c) {
      const double dc = ns[jw_col<S>(w, c)].d;
#pragma unroll
      for (int r = 0; r < RPL; ++r) J.a[c][r] *= dc;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < S::NP; j += blockDim.x) ns[j].d = ns[j].rd = 1.0;
    jw_norms<S>(J, ns, w);
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
  if (lane == 0) atomicAdd(lds_flag + 2, skip);
  return sweeps;
}

}  // namespace damf
