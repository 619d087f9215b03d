// launch_geom.h -- launch geometry of every kernel whose grid grows with the
// problem (nodes n, edges m, query rows q, rank l).  Plain C++ with no HIP
// dependency, so a host-only unit test can evaluate every launch at the
// largest sizes the library accepts (n = q = 2^30) and check that no dispatch
// asks for 2^32 or more work-items: a larger dispatch is not rejected by the
// runtime and leaves part of the grid unrun or faults the device.
//
// Kernels listed here loop over their range (grid stride) whenever the grid
// is capped, so a capped grid only changes how many passes each workgroup
// makes, never which items are processed.
#pragma once

#include <cstdint>

namespace damf {

struct Grid {
  uint32_t blocks;
  uint32_t threads;
};

inline int64_t grid_items(Grid g) { return (int64_t)g.blocks * (int64_t)g.threads; }

// Workgroups for a grid-stride loop over `count` items taken `per_block` per
// workgroup pass: at most 2^16 workgroups, at least one.
constexpr int64_t kMaxStrideBlocks = int64_t(1) << 16;
inline unsigned stride_grid(int64_t count, int64_t per_block) {
  const int64_t b = (count + per_block - 1) / per_block;
  return (unsigned)(b < 1 ? 1 : (b > kMaxStrideBlocks ? kMaxStrideBlocks : b));
}

// ---- one entry per launch site with a problem-sized grid
// state.hip: query rows, one wave per row, 4 rows per 256-thread workgroup
inline Grid geom_query(int64_t q) { return {stride_grid(q, 4), 256}; }
// state.hip: range check of a device node list
inline Grid geom_check_ids(int64_t q) { return {stride_grid(q, 256), 256}; }
// graph.hip: exclusive scan over n + 1 entries, 1024 per workgroup (not
// strided: one partial sum per workgroup; n + 1 <= 2^30 + 1 gives 2^20 + 1)
inline Grid geom_scan(int64_t count) {
  return {(unsigned)((count + 1023) / 1024 < 1 ? 1 : (count + 1023) / 1024), 1024};
}
// graph.hip: rows longer than the LDS sort, one 1024-thread workgroup per row
inline Grid geom_sort_large(int64_t nbig) { return {stride_grid(nbig, 1), 1024}; }
// graph.hip: per-node and per-edge elementwise kernels
inline Grid geom_elementwise(int64_t count) { return {stride_grid(count, 256), 256}; }
// graph.hip: one wave per row
inline Grid geom_rows(int64_t nrows) { return {stride_grid(nrows, 4), 256}; }
// graph.hip: one workgroup per row (row sort)
inline Grid geom_row_per_block(int64_t nrows) { return {stride_grid(nrows, 1), 256}; }
// rsvd.hip: tall product, B resident in LDS, one 16-wave workgroup per CU
inline Grid geom_gemm_tall_res(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return {(unsigned)(b < 1 ? 1 : (b > 256 ? 256 : b)), 1024};
}
// rsvd.hip: tall product for 144 < d <= 192, 64-row blocks, grid stride
inline Grid geom_gemm_tall(int64_t n) { return {stride_grid(n, 64), 256}; }
// rsvd.hip: Householder TSQR, one 1024-thread workgroup per 512-row block
// (not strided; 2 work-items per row)
inline Grid geom_tsqr(int64_t rows) {
  const int64_t b = (rows + 511) / 512;
  return {(unsigned)(b < 1 ? 1 : b), 1024};
}
// spmm.hip: row kernel (capped, grid stride), segment and long-row kernels
inline Grid geom_spmm_rows(int64_t n) {
  const int64_t b = (n + 3) / 4;
  return {(unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b)), 256};
}
// one wave per 256-entry segment of a long row (segments <= nnz / 256) and
// per long row; not strided
inline Grid geom_spmm_segments(int64_t nseg) {
  return {(unsigned)((nseg + 3) / 4 < 1 ? 1 : (nseg + 3) / 4), 256};
}
inline Grid geom_spmm_long(int64_t nlong) {
  return {(unsigned)((nlong + 3) / 4 < 1 ? 1 : (nlong + 3) / 4), 256};
}
// reorth.hip: precision-form rotation, 64-row blocks, at least 16 per workgroup
inline Grid geom_gemm_split(int64_t n) { return {stride_grid(n, 64 * 16), 256}; }

}  // namespace damf
