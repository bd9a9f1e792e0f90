// Host-only driver for the CPU test of the edge-tile layout: reads n, m and
// the n + 1 row offsets from stdin, prints the layout built by
// gm::tiles::tile_layout (rows, ntiles, mpad, the row-start bitmap words,
// the first row of each tile, the rows that span tiles). No device code runs.
#include <cstdio>
#include <vector>

#include "tiles.h"

int main() {
  long long n = 0, m = 0;
  if (std::scanf("%lld %lld", &n, &m) != 2) return 2;
  std::vector<uint32_t> noff((size_t)n + 1);
  for (auto& x : noff)
    if (std::scanf("%u", &x) != 1) return 2;
  const gm::tiles::TileLayout L = gm::tiles::tile_layout(noff, n, m);
  std::printf("%lld %lld %lld\n", (long long)L.rows, (long long)L.ntiles, (long long)L.mpad);
  for (uint32_t w : L.starts) std::printf("%u ", w);
  std::printf("\n");
  for (uint32_t r : L.tile_row) std::printf("%u ", r);
  std::printf("\n");
  for (const auto& c : L.cross) std::printf("%u %u %u ", c.row, c.ta, c.tb);
  std::printf("\n");
  return 0;
}
