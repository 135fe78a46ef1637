// Host check of the grey-level-window kernel's tile layout (csrc/window_geom.hpp,
// the same code the kernel and the launch set-up run): for many image sizes,
// segment heights, GPU sizes and radii, the tiles of a launch cover every
// (strip, row) of the image exactly once, each tile holds at least one row,
// and the tile count is what the launch's grid is sized from.  Prints
// "mismatches N"; exit status 0 only when N = 0.
#include <cstdio>
#include <vector>

#include "window_geom.hpp"

using namespace hrrm;

static long long cases = 0, bad = 0;

static void check(int64_t w, int64_t h, int64_t seg, int64_t slots, bool alone, int r) {
  WindowArgs a{};
  a.w = w;
  a.h = h;
  window_geometry(a, w, h, seg, slots, alone, r);
  ++cases;
  std::vector<int> cover((size_t)a.strips * h, 0);
  const int64_t n = window_tile_count(a);
  int strip = 0, y0 = 0, y1 = 0;
  for (int64_t t = 0; t < n; ++t) {
    if (!window_tile_rows(a, t, strip, y0, y1) || strip < 0 || strip >= a.strips || y0 < 0 ||
        y0 >= y1 || y1 > h) {
      ++bad;
      std::printf("bad tile w=%lld h=%lld seg=%lld slots=%lld alone=%d r=%d tile=%lld: strip %d "
                  "rows [%d, %d)\n",
                  (long long)w, (long long)h, (long long)seg, (long long)slots, (int)alone, r,
                  (long long)t, strip, y0, y1);
      return;
    }
    for (int y = y0; y < y1; ++y) ++cover[(size_t)strip * h + y];
  }
  if (window_tile_rows(a, n, strip, y0, y1)) ++bad;  // nothing past the last tile
  for (size_t i = 0; i < cover.size(); ++i)
    if (cover[i] != 1) {
      ++bad;
      std::printf("coverage %d at strip %zu row %zu (w=%lld h=%lld seg=%lld slots=%lld alone=%d)\n",
                  cover[i], i / (size_t)h, i % (size_t)h, (long long)w, (long long)h,
                  (long long)seg, (long long)slots, (int)alone);
      return;
    }
}

int main() {
  const int64_t ws[] = {1, 5, 63, 64, 65, 128, 129, 190, 300, 1000, 4096};
  const int64_t hs[] = {1, 2, 3, 7, 16, 17, 63, 64, 65, 100, 129, 300, 1000, 4096};
  const int64_t segs[] = {1, 2, 5, 16, 32, 64, 128};
  const int64_t slots[] = {1, 7, 40, 2816};
  for (int64_t w : ws)
    for (int64_t h : hs)
      for (int64_t seg : segs)
        for (int64_t sl : slots)
          for (int alone = 0; alone < 2; ++alone)
            for (int r : {6, 15, 50}) check(w, h, seg, sl, alone != 0, r);
  std::printf("cases %lld mismatches %lld\n", cases, bad);
  return bad == 0 ? 0 : 1;
}
