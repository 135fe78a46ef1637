// Host check of the workgroup-to-tile map of the median kernels (xcd_remap):
// for every grid size up to 20000 workgroups it is a permutation of the tiles
// (none skipped, none done twice), and the workgroups that land on one XCD
// (every eighth, as the hardware deals them out) get one contiguous band of
// tiles in dispatch order.  Prints the number of failing grid sizes; exit
// status 0 only when there are none.
#include <cstdio>
#include <vector>

#include "wave.hpp"

int main() {
  int bad = 0;
  for (int nb = 1; nb <= 20000; ++nb) {
    std::vector<int> seen(nb, 0);
    bool ok = true;
    for (int b = 0; b < nb && ok; ++b) {
      const int t = hrrm::xcd_remap(b, nb);
      if (t < 0 || t >= nb || seen[t]++) ok = false;
      // the next workgroup on the same XCD takes the next tile
      if (ok && b + 8 < nb && hrrm::xcd_remap(b + 8, nb) != t + 1) ok = false;
    }
    bad += !ok;
  }
  std::printf("grid sizes with a bad map: %d\n", bad);
  return bad != 0;
}
