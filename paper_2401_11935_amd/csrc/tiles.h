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

// Split product on a one-dimensional grid of tiles x K chunks, the chunk count a multiple
// of 8: workgroup L runs on XCD L % 8, and every tile of one K chunk is given to the same
// XCD, dispatched together, so that the chunk's operand rows are fetched once into that
// XCD's L2 and shared by its tiles.  Returns the chunk of workgroup L; (tm, tn) is its tile.
// A bijection of [0, tiles_m * tiles_n * chunks) onto (chunk, tile).
__device__ inline int64_t split_tile_of(int64_t L, int64_t tiles_m, int64_t tiles_n, int64_t& tm, int64_t& tn) {
  const int64_t tiles = tiles_m * tiles_n, j = L / 8;
  tile_of(j % tiles, tiles_m, tiles_n, tm, tn);
  return L % 8 + 8 * (j / tiles);
}

// Diagonal pair batch of a pair-blocked product (rows (p, c), columns (q, d), both
// orbital blocks the same, vu values of c and d per orbital): the pair (p, q) equals the
// transpose of (q, p), so the tiles lying entirely in the p > q part are skipped and those
// pairs are filled from their mirrors afterwards.  The kept tiles thin out with the tile
// row, so the rows are dealt to the 8 XCDs in a snake, XCD x taking rows 16k + x and
// 16k + 15 - x, which evens out the kept tiles per XCD; each XCD walks its rows column by
// column (the rows of one column share its B panel in L2).  The grid is 8 * max_x rows_x
// * tiles_n workgroups.
__host__ __device__ inline int64_t diag_rows(int64_t tiles_m, int64_t x) {
  const int64_t rem = tiles_m % 16;
  return 2 * (tiles_m / 16) + (x < rem ? 1 : 0) + (15 - x < rem ? 1 : 0);
}

// Tile (tm, tn) of workgroup bid in a diagonal batch; false if it has none or if its
// tile is skipped.  N is the column count, BM x BN the tile.
__device__ inline bool diag_tile(int64_t bid, int64_t tiles_m, int64_t tiles_n, int64_t N, int64_t vu, int BM, int BN,
                                 int64_t& tm, int64_t& tn) {
  const int64_t x = bid % 8, j = bid / 8, rows = diag_rows(tiles_m, x);
  if (j >= rows * tiles_n) return false;
  const int64_t lr = j % rows;
  tn = j / rows;
  tm = 16 * (lr >> 1) + ((lr & 1) ? 15 - x : x);
  const int64_t n0 = tn * BN, nlast = (n0 + BN < N ? n0 + BN : N) - 1;
  return (tm * BM) / vu <= nlast / vu;
}

// Host side: whether a np x np diagonal batch with BM x BN tiles skips any tile, and the
// grid it then needs.
inline bool diag_skips(int64_t np, int64_t vu, int BM, int BN) {
  const int64_t M = np * vu, tm = (M + BM - 1) / BM, tn = (M + BN - 1) / BN;
  for (int64_t a = 0; a < tm; ++a)
    for (int64_t b = 0; b < tn; ++b)
      if ((a * BM) / vu > (((b + 1) * BN < M ? (b + 1) * BN : M) - 1) / vu) return true;
  return false;
}
inline int64_t diag_grid(int64_t tiles_m, int64_t tiles_n) {
  int64_t rmax = 0;
  for (int64_t x = 0; x < 8; ++x) rmax = diag_rows(tiles_m, x) > rmax ? diag_rows(tiles_m, x) : rmax;
  return 8 * rmax * tiles_n;
}

// The p > q pairs of a diagonal batch from their mirror images:
// V2[(p*np + q)*kp + c*vu + d] = V2[(q*np + p)*kp + d*vu + c].  One workgroup transposes
// a 32 x 32 tile of one pair through LDS; blockIdx.y is the index of the pair in the
// order (1,0), (2,0), (2,1), (3,0), ...
template <class T>
__global__ __launch_bounds__(256) void pair_mirror_kernel(T* V2, int64_t vu, int64_t kp, int64_t np, int tiles) {
  __shared__ T t[32][33];
  const int64_t k = blockIdx.y;
  int64_t p = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)k)) * 0.5);
  while (p * (p - 1) / 2 > k) --p;
  while ((p + 1) * p / 2 <= k) ++p;
  const int64_t q = k - p * (p - 1) / 2;
  const int64_t c0 = (blockIdx.x / tiles) * 32, d0 = (blockIdx.x % tiles) * 32;
  const T* src = V2 + (q * np + p) * kp;
  T* dst = V2 + (p * np + q) * kp;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8)
    if (d0 + r < vu && c0 + tx < vu) t[r][tx] = src[(d0 + r) * vu + c0 + tx];
  __syncthreads();
  for (int r = ty; r < 32; r += 8)
    if (c0 + r < vu && d0 + tx < vu) dst[(c0 + r) * vu + d0 + tx] = t[tx][r];
}

}  // namespace dcsd
