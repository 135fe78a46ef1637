// Insertion masks of a value in a tier subtree of an adaptive tree: the
// topology walk, and the same mask from the subtree's split values held in
// registers.  Host-callable so that the two can be checked against each other
// on the CPU.
#pragma once
#include "hrrm_internal.h"

namespace hrrm {

// Insertion mask of value v in the adaptive subtree rooted at internal node
// `node` (depth dep, interval starting at lo): walk at most four levels of the
// topology, marking the left nodes the value counts in.
__host__ __device__ __forceinline__ uint4 amask(const TopoNode* topo, int node, int dep, int stop,
                                                int v) {
  uint32_t m[4] = {0u, 0u, 0u, 0u};
  int p = 1;
#pragma unroll
  for (int k = 0; k < kTierLevels; ++k) {
    if (node < 0 || dep + k >= stop) break;
    const TopoNode t = topo[node];
    const bool left = v < t.split;
    if (left) {
      const int b = p - 1;
      m[b >> 2] |= 1u << ((b & 3) * 8);
    }
    node = left ? t.left : t.right;
    p = 2 * p + (left ? 0 : 1);
  }
  return make_uint4(m[0], m[1], m[2], m[3]);
}

// A lane's adaptive tier subtree held in registers: the split value of the
// node at each heap position 1..15 below `node` (field s<p - 1>), -1 where the
// walk of amask would find no node (no value is below -1, so it counts
// nowhere there and under it).  Children are followed as amask follows them.
// Named fields, not an array: selects between array elements get folded into
// a private-memory load at a selected address.
struct SubtreeRegs {
  int s0, s1, s2, s3, s4, s5, s6, s7, s8, s9, s10, s11, s12, s13, s14;
};

__host__ __device__ __forceinline__ SubtreeRegs load_subtree_regs(const TopoNode* topo,
                                                                  int node) {
  const TopoNode none = {-1, -1, -1, 0};
  auto at = [&](int i) -> TopoNode { return i >= 0 ? topo[i] : none; };
  auto split = [&](int i) -> int { return i >= 0 ? topo[i].split : -1; };
  const TopoNode t1 = at(node);
  const TopoNode t2 = at(t1.left), t3 = at(t1.right);
  const TopoNode t4 = at(t2.left), t5 = at(t2.right), t6 = at(t3.left), t7 = at(t3.right);
  SubtreeRegs q;
  q.s0 = t1.split;
  q.s1 = t2.split;
  q.s2 = t3.split;
  q.s3 = t4.split;
  q.s4 = t5.split;
  q.s5 = t6.split;
  q.s6 = t7.split;
  q.s7 = split(t4.left);
  q.s8 = split(t4.right);
  q.s9 = split(t5.left);
  q.s10 = split(t5.right);
  q.s11 = split(t6.left);
  q.s12 = split(t6.right);
  q.s13 = split(t7.left);
  q.s14 = split(t7.right);
  return q;
}

// amask from a register-held subtree, before the level limit: the path of v
// through the four levels is chosen by selects, and each level's left node
// on the path gets its byte when v goes left there.
__host__ __device__ __forceinline__ uint4 amask_regs(const SubtreeRegs q, int v) {
  const bool l0 = v < q.s0;
  const int s1 = l0 ? q.s1 : q.s2;
  const bool l1 = v < s1;
  const int i2 = (l0 ? 0 : 2) + (l1 ? 0 : 1);  // heap position 4 + i2
  const int s2 = l0 ? (l1 ? q.s3 : q.s4) : (l1 ? q.s5 : q.s6);
  const bool l2 = v < s2;
  const int a0 = l2 ? q.s7 : q.s8, a1 = l2 ? q.s9 : q.s10;
  const int a2 = l2 ? q.s11 : q.s12, a3 = l2 ? q.s13 : q.s14;
  const int s3 = l0 ? (l1 ? a0 : a1) : (l1 ? a2 : a3);
  const bool l3 = v < s3;
  const int b1 = l0 ? 1 : 2, b2 = 3 + i2, b3 = 7 + 2 * i2 + (l2 ? 0 : 1);  // bytes (position - 1)
  const uint64_t lo = (l0 ? 1ull : 0ull) | (l1 ? 1ull << (8 * b1) : 0ull) |
                      (l2 ? 1ull << (8 * b2) : 0ull) | (l3 && b3 == 7 ? 1ull << 56 : 0ull);
  const uint64_t hi = l3 && b3 > 7 ? 1ull << (8 * (b3 - 8)) : 0ull;
  return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
}

}  // namespace hrrm
