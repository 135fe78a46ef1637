// Host check of the adaptive tree's register-held subtree masks: for random
// topologies (absent children, negative splits, every level limit), the mask
// from a lane's subtree split values (load_subtree_regs + amask_regs, cut to
// the maintained levels) equals the topology walk's (amask) for every value.
// Prints the number of mismatches; exit status 0 only when there are none.
#include <cstdio>
#include <random>
#include <vector>

#include "topo_mask.hpp"

using namespace hrrm;

int main() {
  std::mt19937 g(7);
  long long cases = 0, bad = 0;
  for (int trial = 0; trial < 4000; ++trial) {
    const int n = 1 + (int)(g() % 40);
    std::vector<TopoNode> topo(n);
    for (auto& t : topo) {
      t.split = g() % 10 ? (int)(g() % 301) : -1 - (int)(g() % 5);
      t.left = g() % 5 ? (int)(g() % (n + 1)) - 1 : -1;
      t.right = g() % 5 ? (int)(g() % (n + 1)) - 1 : -1;
      t.pad = 0;
    }
    const int node = (int)(g() % (n + 1)) - 1;
    const int dep = (int)(g() % 13);
    const int stops[6] = {dep + 1, dep + 2, dep + 3, dep + 4, dep + 9, 1000};
    const int stop = stops[g() % 6];
    // bytes of the maintained levels: levels 0..L-1 are heap positions
    // 1 .. 2^L - 1, bytes 0 .. 2^L - 2
    const int levels = stop - dep < kTierLevels ? stop - dep : kTierLevels;
    uint32_t lim[4] = {0, 0, 0, 0};
    for (int b = 0; b < (1 << levels) - 1; ++b) lim[b >> 2] |= 0xffu << (8 * (b & 3));
    const SubtreeRegs q = load_subtree_regs(topo.data(), node);
    for (int v = 0; v <= 300; v += 1 + (int)(g() % 7)) {
      const uint4 want = amask(topo.data(), node, dep, stop, v);
      const uint4 got = amask_regs(q, v);
      ++cases;
      if (want.x != (got.x & lim[0]) || want.y != (got.y & lim[1]) || want.z != (got.z & lim[2]) ||
          want.w != (got.w & lim[3]))
        ++bad;
    }
  }
  std::printf("cases %lld mismatches %lld\n", cases, bad);
  return bad != 0;
}
