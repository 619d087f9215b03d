// Host-only check of the library's launch geometry (csrc/launch_geom.h): at
// the largest sizes the library accepts, no dispatch may ask for 2^32 or more
// work-items.  Prints one line per launch and exits non-zero on a violation.
#include <cstdint>
#include <cstdio>

#include "../../paper_2306_08967_amd/csrc/launch_geom.h"

using namespace damf;

int main() {
  const int64_t kLimit = int64_t(1) << 32;
  const int64_t n = int64_t(1) << 30;       // node cap
  const int64_t q = n;                      // a full-basis query
  const int64_t m = int64_t(1) << 33;       // edges (beyond what 288 GB holds)
  const int64_t l = 192;                    // widest tall product
  struct Case {
    const char *name;
    Grid g;
  } cases[] = {
      {"query(q)", geom_query(q)},
      {"check_ids(q)", geom_check_ids(q)},
      {"scan(n + 1)", geom_scan(n + 1)},
      {"sort_large(m / 2048)", geom_sort_large(m / 2048)},
      {"elementwise(n * l)", geom_elementwise(n * l)},
      {"elementwise(m)", geom_elementwise(m)},
      {"rows(n)", geom_rows(n)},
      {"row_per_block(n)", geom_row_per_block(n)},
      {"gemm_tall_res(n)", geom_gemm_tall_res(n)},
      {"gemm_tall(n)", geom_gemm_tall(n)},
      {"tsqr(n)", geom_tsqr(n)},
      {"spmm_rows(n)", geom_spmm_rows(n)},
      {"spmm_segments(m / 256)", geom_spmm_segments(m / 256)},
      {"spmm_long(m / 256)", geom_spmm_long(m / 256)},
      {"gemm_split(n)", geom_gemm_split(n)},
  };
  int bad = 0;
  for (const Case &c : cases) {
    const int64_t items = grid_items(c.g);
    const bool ok = c.g.blocks >= 1 && items < kLimit;
    std::printf("%-26s blocks %10u threads %5u items %14lld %s\n", c.name, c.g.blocks, c.g.threads,
                (long long)items, ok ? "ok" : "TOO LARGE");
    bad += ok ? 0 : 1;
  }
  // stride grids cover any count with at least one workgroup
  if (stride_grid(0, 256) != 1 || stride_grid(1, 256) != 1) ++bad;
  if (stride_grid(int64_t(1) << 40, 1) != (unsigned)kMaxStrideBlocks) ++bad;
  (void)l;
  return bad ? 1 : 0;
}
