// Host check of the workgroup -> tile orders (test program, built and run by
// tests/test_tiles.py on the CPU).  The tile functions are device functions;
// redefining the attribute before the header makes them callable here too.
#include <hip/hip_runtime.h>
#undef __device__
#define __device__ __attribute__((host)) __attribute__((device))
#include "tiles.h"

#include <cstdio>
#include <vector>

using dcsd::diag_grid;
using dcsd::diag_skips;
using dcsd::diag_tile;
using dcsd::split_tile_of;
using dcsd::tile_of;

static int fails = 0;
#define CHECK(c, ...)                   \
  do {                                  \
    if (!(c)) {                         \
      if (fails < 20) {                 \
        std::printf("FAIL: " __VA_ARGS__); \
        std::printf("\n");              \
      }                                 \
      ++fails;                          \
    }                                   \
  } while (0)

// every tile exactly once for bid in [0, tm * tn)
static void check_tile_of(int64_t tm, int64_t tn) {
  std::vector<int> seen(tm * tn, 0);
  for (int64_t bid = 0; bid < tm * tn; ++bid) {
    int64_t a = -1, b = -1;
    tile_of(bid, tm, tn, a, b);
    CHECK(a >= 0 && a < tm && b >= 0 && b < tn, "tile_of(%lld; %lld x %lld) -> (%lld, %lld) out of range",
          (long long)bid, (long long)tm, (long long)tn, (long long)a, (long long)b);
    if (a >= 0 && a < tm && b >= 0 && b < tn) ++seen[a * tn + b];
  }
  for (int64_t t = 0; t < tm * tn; ++t)
    CHECK(seen[t] == 1, "tile_of %lld x %lld: tile %lld seen %d times", (long long)tm, (long long)tn, (long long)t,
          seen[t]);
}

// diagonal batch of np orbitals with vu values each: the kept tiles (some row orbital <= some
// column orbital) exactly once over the grid, no other tile, every p <= q element inside a kept
// tile, and diag_skips true exactly when a tile is left out
static void check_diag(int64_t np, int64_t vu, int BM, int BN) {
  const int64_t M = np * vu, tm = (M + BM - 1) / BM, tn = (M + BN - 1) / BN;
  auto kept = [&](int64_t a, int64_t b) {
    const int64_t nlast = ((b + 1) * BN < M ? (b + 1) * BN : M) - 1;
    return (a * BM) / vu <= nlast / vu;
  };
  std::vector<int> seen(tm * tn, 0);
  const int64_t grid = diag_grid(tm, tn);
  for (int64_t bid = 0; bid < grid; ++bid) {
    int64_t a = -1, b = -1;
    if (!diag_tile(bid, tm, tn, M, vu, BM, BN, a, b)) continue;
    CHECK(a >= 0 && a < tm && b >= 0 && b < tn, "diag_tile np=%lld vu=%lld: (%lld, %lld) out of range", (long long)np,
          (long long)vu, (long long)a, (long long)b);
    if (a >= 0 && a < tm && b >= 0 && b < tn) ++seen[a * tn + b];
  }
  bool any_skipped = false;
  for (int64_t a = 0; a < tm; ++a)
    for (int64_t b = 0; b < tn; ++b) {
      const int want = kept(a, b) ? 1 : 0;
      any_skipped |= want == 0;
      CHECK(seen[a * tn + b] == want, "diag_tile np=%lld vu=%lld BM=%d: tile (%lld, %lld) seen %d, want %d",
            (long long)np, (long long)vu, BM, (long long)a, (long long)b, seen[a * tn + b], want);
    }
  CHECK(diag_skips(np, vu, BM, BN) == any_skipped, "diag_skips np=%lld vu=%lld", (long long)np, (long long)vu);
  if (M <= 1024)
    for (int64_t r = 0; r < M; ++r)
      for (int64_t c = 0; c < M; ++c)
        if (r / vu <= c / vu) CHECK(kept(r / BM, c / BN), "element (%lld, %lld) with p <= q in a skipped tile",
                                    (long long)r, (long long)c);
}

// split products on a one-dimensional grid: every (chunk, tile) exactly once for L in
// [0, tiles * chunks), and every tile of a chunk on the XCD L % 8 == chunk % 8
static void check_split(int64_t tm, int64_t tn, int64_t chunks) {
  const int64_t tiles = tm * tn;
  std::vector<int> seen(tiles * chunks, 0);
  for (int64_t L = 0; L < tiles * chunks; ++L) {
    int64_t a = -1, b = -1;
    const int64_t z = split_tile_of(L, tm, tn, a, b);
    const bool ok = z >= 0 && z < chunks && a >= 0 && a < tm && b >= 0 && b < tn;
    CHECK(ok, "split_tile_of(%lld; %lld x %lld, %lld chunks) -> chunk %lld tile (%lld, %lld) out of range",
          (long long)L, (long long)tm, (long long)tn, (long long)chunks, (long long)z, (long long)a, (long long)b);
    if (!ok) continue;
    CHECK(L % 8 == z % 8, "split_tile_of: chunk %lld on XCD %lld", (long long)z, (long long)(L % 8));
    ++seen[z * tiles + a * tn + b];
  }
  for (int64_t t = 0; t < tiles * chunks; ++t)
    CHECK(seen[t] == 1, "split_tile_of %lld x %lld, %lld chunks: (chunk, tile) %lld seen %d times", (long long)tm,
          (long long)tn, (long long)chunks, (long long)t, seen[t]);
}

int main() {
  for (int64_t tm = 1; tm <= 9; ++tm)
    for (int64_t tn = 1; tn <= 9; ++tn)
      for (int64_t chunks = 8; chunks <= 32; chunks += 8) check_split(tm, tn, chunks);
  check_split(4, 8, 16);  // the ladder contraction at the metric shape, 128-wide tiles
  check_split(2, 4, 32);  // the same on 256-wide tiles
  for (int64_t tm = 1; tm <= 48; ++tm)
    for (int64_t tn = 1; tn <= 48; ++tn) check_tile_of(tm, tn);
  const int64_t big[][2] = {{101, 101}, {145, 3}, {3, 145}, {82, 82}, {4, 1024}, {257, 129}, {1, 513}};
  for (auto& s : big) check_tile_of(s[0], s[1]);
  const int64_t vus[] = {2, 3, 17, 64, 127, 128, 129, 200, 402, 602};
  for (int64_t vu : vus)
    for (int64_t np = 1; np <= 40; ++np) {
      check_diag(np, vu, 128, 128);
      check_diag(np, vu, 64, 64);
    }
  check_diag(46, 402, 128, 128);
  check_diag(70, 602, 128, 128);
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  std::printf("tiles ok\n");
  return 0;
}
