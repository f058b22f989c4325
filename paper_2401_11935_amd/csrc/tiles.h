// Workgroup -> output-tile order shared by the GEMM kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace dcsd {

// Linear workgroup ids are dispatched round-robin over the 8 XCDs, each with
// its own L2.  Each XCD's ids are renumbered into one contiguous range of
// tiles, and that range is walked in groups of GROUP tile rows, row-fastest,
// so that the workgroups resident together on one XCD form a compact block of
// output tiles that share A rows and B columns in its L2.  The map is a
// bijection of [0, tiles_m * tiles_n) for any tile counts.
__device__ inline void tile_of(int64_t bid, int64_t tiles_m, int64_t tiles_n, int64_t& tm, int64_t& tn) {
  constexpr int64_t NXCD = 8, GROUP = 8;
  const int64_t T = tiles_m * tiles_n;
  const int64_t per = T / NXCD, extra = T % NXCD;
  const int64_t x = bid % NXCD, j = bid / NXCD;
  const int64_t L = x * per + (x < extra ? x : extra) + j;
  const int64_t span = GROUP * tiles_n;
  const int64_t grp = L / span, first = grp * GROUP;
  const int64_t rows = tiles_m - first < GROUP ? tiles_m - first : GROUP;
  const int64_t w = L - grp * span;
  tm = first + w % rows;
  tn = w / rows;
}

}  // namespace dcsd
