// Host check of the clamped-row walk (RowWalk) used by the window builds:
// every offset it visits over a window equals the clamp-to-edge row offset
// written out directly, and rows it visits past the window stay inside the
// image.  Exhaustive over small images, plus rows near the ends of very tall
// images (the walk's int bounds are cut there).  Prints the number of
// mismatches; exit status 0 only when there are none.
#include <cstdio>

#include "wave.hpp"

using hrrm::RowWalk;
using hrrm::clampi;

static long long cases = 0, bad = 0;

template <bool D3>
static void check(int64_t y, int64_t z, int64_t h, int64_t d, int r, int extra) {
  const int64_t srs = 1000, sss = 1000 * (h + 7);
  const int zr = D3 ? r : 0;
  const int nw = (2 * zr + 1) * (2 * r + 1);
  RowWalk<D3> w(y, z, h, d, srs, sss, r, zr);
  int j = -r, dz = -zr;
  ++cases;
  for (int q = 0; q < nw + extra; ++q) {
    if (q < nw) {
      const int64_t want = (D3 ? clampi(z + dz, d - 1) : z) * sss + clampi(y + j, h - 1) * srs;
      if (w.off != want) {
        ++bad;
        return;
      }
      if (++j > r) {
        j = -r;
        ++dz;
      }
    } else {  // past the window: any row of the image
      const int64_t o = w.off - (D3 ? 0 : z * sss);
      const int64_t zz = o / sss, yy = (o % sss) / srs;
      if (o % srs || yy < 0 || yy >= h || zz < 0 || (D3 && zz >= d)) {
        ++bad;
        return;
      }
    }
    w.next();
  }
}

int main() {
  for (int r = 0; r <= 6; ++r)
    for (int64_t h = 1; h <= 10; ++h)
      for (int64_t y = 0; y < h; ++y) {
        check<false>(y, 0, h, 1, r, 9);
        check<false>(y, 3, h, 1, r, 9);  // a 2-D slice of a stack: z offset kept
        for (int64_t d = 1; d <= 6; ++d)
          for (int64_t z = 0; z < d; ++z) check<true>(y, z, h, d, r, 9);
      }
  const int64_t H = (int64_t)1 << 34;
  for (int r : {0, 1, 15, 127})
    for (int64_t y : {(int64_t)0, (int64_t)1, H / 2, H - 3, H - 2, H - 1}) {
      check<false>(y, 0, H, 1, r, 9);
      check<true>(y, 2, H, 5, r > 15 ? 15 : r, 9);
    }
  std::printf("cases %lld mismatches %lld\n", cases, bad);
  return bad != 0;
}
