// Fused running-median kernel for gfx950 (MI355X).
//
// Method: Alekseychuk, "Hierarchical Recursive Running Median".
//  * Every image column of a strip keeps an implicit interval-occurrences tree
//    (IOT) over the 2r+1 rows of the current window (Sec. III; implicit tree
//    with left nodes only and the top node elided, Sec. III-A).  A node's
//    counter holds the number of column values that fall in its LEFT child.
//  * Moving down one row removes one value from and inserts one value into
//    every column tree (Sec. III, column update; Sec. III-B, add_value: walk
//    the levels, count at the left node when the value lies below the split).
//  * For each output pixel the descent of get_order_statistic (Sec. III) walks
//    the levels: the window count of the current left node is compared with
//    K minus the left-occurrence accumulator; go left, or add and go right.
//  * Window counts are built on demand from the column trees (Sec. III, window
//    IOT updated on demand).  On the GPU a wave holds 64 consecutive pixels of a
//    row.  Lanes that need the same node form a group (ballot); every lane
//    reads the column counter entering and leaving its window and a DPP prefix
//    sum over the wave turns these differences into the running window count,
//    anchored at the window of the wave's first pixel - the paper's elementary
//    update (one add, one subtract per visited node), done for 64 pixels at
//    once.  Small groups instead sum their 2r+1 column counters directly (the
//    paper's non-elementary catch-up).
//
// Storage (LDS, byte counters, level-major, node-major/column-minor so that 64
// lanes reading one node hit 64 consecutive bytes):
//  * dense: all 255 left-node counters of an 8-bit tree per column (u8 data).
//  * tiered: the tree is cut into 4-level tiers (15 counters per column each).
//    Tier 1 (the top) is always held.  A deeper tier subtree is materialised in
//    a slot only when some pixel of the current row descends into it - the
//    paper's on-demand principle applied to the column trees - and is kept
//    (least recently used replacement) while rows keep needing it.  A pixel
//    whose subtree finds no free slot counts its window values directly.
//    This is what lets 16-bit trees (65535 counters per column) live in LDS.
//
// Topology: uniform (each split halves its interval, Sec. III) or adaptive
// (split points from a table, leaf test at every visit, Sec. III-C).
#include "hrrm_internal.h"

namespace hrrm {
namespace {

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4, 8 inside
// each 16-lane row, then lane 15 of a row added into the next row and lane 31
// into the upper half.  Lanes whose DPP source is outside the row keep 0.
__device__ __forceinline__ uint32_t wave_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
  return v;
}

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t hi) {
  return v < 0 ? 0 : (v > hi ? hi : v);
}

__device__ __forceinline__ size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Tier-slot bookkeeping (tiered storage only).
struct TierMeta {
  uint32_t ht[kHash];  // (key + 1) << 8 | slot, 0 = empty; open addressing
  int32_t key[kMaxSlots], lo[kMaxSlots], hi[kMaxSlots], dep[kMaxSlots], stamp[kMaxSlots];
  int32_t miss_n[3];
  int32_t flag[3][kWaves];
  int32_t reb_n;
  int32_t pad;
  int32_t miss[kMaxMiss][4];  // key, lo, hi, depth of a subtree root nobody holds
  int32_t reb[kMaxSlots][4];  // slot, key, lo, depth of a slot to rebuild
};

__device__ __forceinline__ uint32_t ht_hash(int key) {
  return ((uint32_t)key * 2654435761u) >> 25;  // 7 bits for kHash = 128
}

__device__ __forceinline__ int ht_find(const uint32_t* ht, int key) {
  uint32_t h = ht_hash(key);
  const uint32_t tag = (uint32_t)(key + 1);
  for (int i = 0; i < kHash; ++i) {
    const uint32_t e = ht[(h + i) & (kHash - 1)];
    if (e == 0) return -1;
    if ((e >> 8) == tag) return (int)(e & 0xffu);
  }
  return -1;
}

__device__ __forceinline__ void ht_insert(uint32_t* ht, int key, int slot) {
  uint32_t h = ht_hash(key);
  for (int i = 0; i < kHash; ++i) {
    uint32_t& e = ht[(h + i) & (kHash - 1)];
    if (e == 0) {
      e = ((uint32_t)(key + 1) << 8) | (uint32_t)slot;
      return;
    }
  }
}

// Adds +1/-1 to the byte counter of (row, column) with one dword LDS atomic.
// Counters never leave 0..255 (removals precede insertions), so no carry or
// borrow crosses into a neighbouring byte.
__device__ __forceinline__ void cnt_add(uint8_t* cnt, int cp, int row, int lc, bool inc) {
  uint32_t* wp = (uint32_t*)(cnt + (size_t)row * cp + (lc & ~3));
  const uint32_t one = 1u << ((lc & 3) * 8);
  if (inc)
    __hip_atomic_fetch_add(wp, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else
    __hip_atomic_fetch_sub(wp, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One node of the tree: split point and children.
template <bool ADAPT>
struct Step {
  int split, lch, rch;
  bool lleaf, rleaf;
};

template <bool ADAPT>
__device__ __forceinline__ Step<ADAPT> node_step(const TopoNode* topo, int node, int lo, int depth,
                                                 int bits) {
  Step<ADAPT> s;
  if constexpr (ADAPT) {
    const TopoNode t = topo[node];
    s.split = t.split;
    s.lch = t.left;
    s.rch = t.right;
    s.lleaf = t.left < 0;
    s.rleaf = t.right < 0;
  } else {
    s.split = lo + (1 << (bits - 1 - depth));
    s.lch = 2 * node;
    s.rch = 2 * node + 1;
    s.lleaf = s.rleaf = (depth + 1 >= bits);
  }
  return s;
}

// Window count of each lane's counter row (lanes with want=true), see the file
// comment.  Must be called with all 64 lanes active.
__device__ __forceinline__ uint32_t window_count(const uint8_t* __restrict__ cnt, int cp, int row,
                                                 bool want, int lx, int span, int lane, int wbase,
                                                 int min_group, int max_groups) {
  uint64_t pending = ballot(want);
  uint64_t direct = 0;
  uint32_t w = 0;
  int ng = 0;
  while (pending) {
    const int leader = __builtin_ctzll(pending);
    const int grow = readlane(row, leader);
    const uint64_t m = ballot(row == grow) & pending;
    pending &= ~m;
    if (__builtin_popcountll(m) < min_group || ng >= max_groups) {
      direct |= m;
      continue;
    }
    ++ng;
    const uint8_t* base = cnt + (size_t)grow * cp;
    const uint32_t vout = base[lx];         // column of x - r - 1
    const uint32_t vin = base[lx + span];   // column of x + r
    const uint32_t sc = wave_scan((vin << 16) | vout);
    uint32_t b;
    if (span <= 64) {
      b = (uint32_t)readlane((int)(sc & 0xffffu), span - 1);
    } else {
      uint32_t e = 0;
      for (int k = 64 + lane; k < span; k += 64) e += base[wbase + k];
      const uint32_t es = wave_scan(e);
      b = (uint32_t)readlane((int)(sc & 0xffffu), 63) + (uint32_t)readlane((int)es, 63);
    }
    const uint32_t wl = b + (sc >> 16) - (sc & 0xffffu);
    if ((m >> lane) & 1) w = wl;
  }
  if (direct) {
    if ((direct >> lane) & 1) {
      const uint8_t* p = cnt + (size_t)row * cp + lx + 1;
      uint32_t s = 0;
      for (int j = 0; j < span; ++j) s += p[j];
      w = s;
    }
  }
  return w;
}

template <typename T, bool D3>
__device__ __forceinline__ uint32_t brute_count(const T* __restrict__ src, const MedianArgs& a,
                                                int64_t x, int64_t y, int64_t z, int lo,
                                                int split) {
  const int r = a.r;
  uint32_t c = 0;
  const int zr = D3 ? r : 0;
  for (int dz = -zr; dz <= zr; ++dz) {
    const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
    for (int dy = -r; dy <= r; ++dy) {
      const T* rowp = src + zz * a.sss + clampi(y + dy, a.h - 1) * a.srs;
      for (int dx = -r; dx <= r; ++dx) {
        const int v = rowp[clampi(x + dx, a.w - 1)];
        c += (v >= lo && v < split) ? 1u : 0u;
      }
    }
  }
  return c;
}

// Walk of one value through the column tree of local column lc: count it
// (inc) or uncount it at every left node it passes, through tier 1 and then
// through every deeper tier whose slot is held (a held slot's ancestors are
// always held, so the walk stops at the first missing tier).
template <bool TIERED, bool ADAPT>
__device__ __forceinline__ void column_walk(uint8_t* cnt, int cp, const TierMeta* tm,
                                            const TopoNode* topo, int root, int bits, int stop,
                                            int v, int lc, bool inc) {
  int node = root, lo = 0, depth = 0, slot = 0, p = 1;
  const int maxdepth = ADAPT ? 3 * bits : bits;  // bound on any tree's height
  for (int it = 0; it < maxdepth; ++it) {
    const Step<ADAPT> s = node_step<ADAPT>(topo, node, lo, depth, bits);
    const bool left = v < s.split;
    const int row = TIERED ? slot * kTierNodes + p - 1 : (ADAPT ? node : node - 1);
    if (left) cnt_add(cnt, cp, row, lc, inc);
    bool leaf;
    if (left) {
      node = s.lch;
      leaf = s.lleaf;
    } else {
      node = s.rch;
      lo = s.split;
      leaf = s.rleaf;
    }
    ++depth;
    if (leaf || depth >= stop) return;
    if constexpr (TIERED) {
      p = 2 * p + (left ? 0 : 1);
      if (p > kTierNodes) {
        slot = ht_find(tm->ht, node);
        if (slot < 0) return;
        p = 1;
      }
    }
  }
}

// Count value v into the 4-level subtree held by `slot` (rebuild of a slot).
template <bool ADAPT>
__device__ __forceinline__ void tier_insert(uint8_t* cnt, int cp, const TopoNode* topo, int bits,
                                            int stop, int v, int slot, int node, int lo, int depth,
                                            int lc) {
  int p = 1;
  for (int k = 0; k < kTierLevels; ++k) {
    const Step<ADAPT> s = node_step<ADAPT>(topo, node, lo, depth, bits);
    const bool left = v < s.split;
    if (left) cnt_add(cnt, cp, slot * kTierNodes + p - 1, lc, true);
    bool leaf;
    if (left) {
      node = s.lch;
      leaf = s.lleaf;
    } else {
      node = s.rch;
      lo = s.split;
      leaf = s.rleaf;
    }
    ++depth;
    if (leaf || depth >= stop) return;
    p = 2 * p + (left ? 0 : 1);
  }
}

// Serial slot assignment for this round's misses (thread 0).  Victims are the
// least recently used slots not used by the current row; evicting a slot also
// evicts the held subtrees below it.
__device__ void assign_slots(TierMeta* tm, int nmiss, int buf, int stamp, int nslots) {
  int nreb = 0;
  for (int i = 0; i < nmiss; ++i) {
    const int key = tm->miss[i][0];
    if (ht_find(tm->ht, key) >= 0) continue;  // duplicate from another wave
    int victim = -1, best = 0x7fffffff;
    for (int s = 1; s < nslots; ++s) {
      const int st = tm->stamp[s];
      if (st != stamp && st < best) {
        best = st;
        victim = s;
      }
    }
    if (victim < 0) continue;  // all slots serve this row: the pixels count directly
    if (tm->key[victim] >= 0) {
      const int vlo = tm->lo[victim], vhi = tm->hi[victim], vdep = tm->dep[victim];
      for (int s = 1; s < nslots; ++s) {
        if (tm->key[s] >= 0 && (s == victim || (tm->dep[s] > vdep && tm->lo[s] >= vlo &&
                                                tm->lo[s] <= vhi))) {
          tm->key[s] = -1;
          tm->stamp[s] = -1;
        }
      }
      for (int h = 0; h < kHash; ++h) tm->ht[h] = 0;
      for (int s = 1; s < nslots; ++s)
        if (tm->key[s] >= 0) ht_insert(tm->ht, tm->key[s], s);
    }
    tm->key[victim] = key;
    tm->lo[victim] = tm->miss[i][1];
    tm->hi[victim] = tm->miss[i][2];
    tm->dep[victim] = tm->miss[i][3];
    tm->stamp[victim] = stamp;
    ht_insert(tm->ht, key, victim);
    tm->reb[nreb][0] = victim;
    tm->reb[nreb][1] = key;
    tm->reb[nreb][2] = tm->miss[i][1];
    tm->reb[nreb][3] = tm->miss[i][3];
    ++nreb;
  }
  tm->reb_n = nreb;
}

template <typename T, bool TIERED, bool ADAPT, bool D3>
__global__ __launch_bounds__(kBlock) void k_median(MedianArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  constexpr int NODES = TIERED ? kTierNodes : kDenseNodes;
  const T* __restrict__ src = (const T*)a.src;
  T* __restrict__ dst = (T*)a.dst;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = a.r, cp = a.cp, ncols = a.ncols, bits = a.bits, stop = a.stop;
  const int span = 2 * r + 1;

  // Tile of this workgroup.  Consecutive workgroups land on consecutive XCDs;
  // remap so each XCD works on a contiguous band of tiles (shared halos stay in
  // that XCD's L2).
  int bid = blockIdx.x;
  {
    const int nb = gridDim.x, q = nb >> 3, rem = nb & 7, xcd = bid & 7, i = bid >> 3;
    bid = xcd * q + (xcd < rem ? xcd : rem) + i;
  }
  const int strip = bid % a.strips;
  const int rest = bid / a.strips;
  const int seg = rest % a.segs;
  const int64_t z = rest / a.segs;
  const int64_t x0 = (int64_t)strip * kBlock;
  const int64_t yb = (int64_t)seg * a.seg_rows;
  const int64_t ye = yb + a.seg_rows < a.h ? yb + a.seg_rows : a.h;

  uint8_t* cnt = lds;
  const size_t cnt_bytes = align16((size_t)(TIERED ? a.nslots : 1) * NODES * cp);
  TierMeta* tm = (TierMeta*)(lds + cnt_bytes);
  const TopoNode* topo = a.topo;
  if constexpr (ADAPT && !TIERED) {
    TopoNode* tl = (TopoNode*)(lds + cnt_bytes);
    for (int i = tid; i <= kDenseNodes; i += kBlock) tl[i] = a.topo[i];
    topo = tl;
    __syncthreads();
  }
  // adaptive: the entry after the last node holds the root's index
  const int root = ADAPT ? topo[(1 << bits) - 1].split : 1;

  for (int i = tid; i < NODES * cp / 4; i += kBlock) ((uint32_t*)cnt)[i] = 0;
  if constexpr (TIERED) {
    for (int i = tid; i < kHash; i += kBlock) tm->ht[i] = 0;
    for (int s = tid; s < kMaxSlots; s += kBlock) {
      tm->key[s] = -1;
      tm->stamp[s] = -1;
      tm->lo[s] = tm->hi[s] = tm->dep[s] = 0;
    }
    if (tid < 3) tm->miss_n[tid] = 0;
    if (tid < 3 * kWaves) tm->flag[tid / kWaves][tid % kWaves] = 0;
    if (tid == 0) {
      tm->reb_n = 0;
      tm->key[0] = root;  // slot 0 holds tier 1, never evicted
      tm->stamp[0] = 0x7fffffff;
    }
  }
  __syncthreads();

  // Column trees of the first window of the segment.
  const int zr = D3 ? r : 0;
  for (int lc = tid; lc < ncols; lc += kBlock) {
    const int64_t cx = clampi(x0 - r - 1 + lc, a.w - 1);
    for (int dz = -zr; dz <= zr; ++dz) {
      const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
      for (int j = -r; j <= r; ++j) {
        const int v = src[zz * a.sss + clampi(yb + j, a.h - 1) * a.srs + cx];
        column_walk<TIERED, ADAPT>(cnt, cp, tm, topo, root, bits, stop, v, lc, true);
      }
    }
  }
  __syncthreads();

  const int lx = wv * 64 + lane;  // output x = x0 + lx; window columns lx+1 .. lx+span
  const int64_t x = x0 + lx;
  const uint32_t K = (uint32_t)a.rank;
  int gr = 0;  // running round counter (triple-buffered round state)

  for (int64_t y = yb; y < ye; ++y) {
    int node = root, lo = 0, hi = (1 << bits) - 1, depth = 0;
    uint32_t acc = 0;
    bool done = (x >= a.w) || (stop == 0);
    int res = 0;
    int slot = 0, p = 1;
    bool exited = false;

    const int maxdepth = ADAPT ? 3 * bits : bits;  // bound on any tree's height
    int steps = 0;
    for (int round = 0; round <= maxdepth; ++round) {
      for (int k = 0; (!TIERED || k < kTierLevels) && steps < maxdepth; ++k, ++steps) {
        const bool act = !done && !exited;
        if (ballot(act) == 0) break;
        const Step<ADAPT> s = node_step<ADAPT>(topo, node, lo, depth, bits);
        const int row = TIERED ? (slot >= 0 ? slot * kTierNodes + p - 1 : 0)
                               : (ADAPT ? node : node - 1);
        const bool coop = act && (!TIERED || slot >= 0);
        uint32_t wl = window_count(cnt, cp, row, coop, lx, span, lane, wv * 64, a.min_group,
                                   a.max_groups);
        if (TIERED && act && slot < 0) wl = brute_count<T, D3>(src, a, x, y, z, lo, s.split);
        if (act) {
          const bool left = acc + wl > K;
          bool leaf;
          if (left) {
            node = s.lch;
            hi = s.split - 1;
            leaf = s.lleaf;
          } else {
            acc += wl;
            node = s.rch;
            lo = s.split;
            leaf = s.rleaf;
          }
          ++depth;
          if (leaf || depth >= stop) {
            done = true;
            res = lo;
          } else if (TIERED) {
            p = 2 * p + (left ? 0 : 1);
            if (p > kTierNodes) exited = true;
          }
        }
      }
      if constexpr (!TIERED) break;
      if constexpr (TIERED) {
        // Tier transition: lanes that left their 4-level subtree look up the
        // slot of the next one; subtrees no slot holds are queued as misses.
        const int b = gr % 3;
        if (tid == 0) tm->miss_n[(gr + 1) % 3] = 0;
        const uint64_t ex = ballot(exited);
        if (lane == 0) tm->flag[b][wv] = ex != 0;
        int newslot = -1;
        uint64_t pend = ex;
        while (pend) {
          const int leader = __builtin_ctzll(pend);
          const int key = readlane(node, leader);
          const uint64_t m = ballot(node == key) & pend;
          pend &= ~m;
          const int hs = ht_find(tm->ht, key);
          if (hs >= 0) {
            if (lane == leader) tm->stamp[hs] = (int)y;
            if ((m >> lane) & 1) newslot = hs;
          } else {
            if (lane == leader) {
              const int i = atomicAdd(&tm->miss_n[b], 1);
              tm->miss[i][0] = key;
              tm->miss[i][1] = lo;
              tm->miss[i][2] = hi;
              tm->miss[i][3] = depth;
            }
            if ((m >> lane) & 1) newslot = -2;
          }
        }
        __syncthreads();
        bool any = false;
        for (int w2 = 0; w2 < kWaves; ++w2) any |= tm->flag[b][w2] != 0;
        const int nmiss = tm->miss_n[b];
        ++gr;
        if (!any) break;
        if (nmiss > 0) {
          if (tid == 0) assign_slots(tm, nmiss, b, (int)y, a.nslots);
          __syncthreads();
          const int nreb = tm->reb_n;
          if (nreb > 0) {
            for (int i = 0; i < nreb; ++i) {
              uint32_t* sb = (uint32_t*)(cnt + (size_t)tm->reb[i][0] * kTierNodes * cp);
              for (int j = tid; j < kTierNodes * cp / 4; j += kBlock) sb[j] = 0;
            }
            __syncthreads();
            for (int lc = tid; lc < ncols; lc += kBlock) {
              const int64_t cx = clampi(x0 - r - 1 + lc, a.w - 1);
              for (int dz = -zr; dz <= zr; ++dz) {
                const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
                for (int j = -r; j <= r; ++j) {
                  const int v = src[zz * a.sss + clampi(y + j, a.h - 1) * a.srs + cx];
                  for (int i = 0; i < nreb; ++i) {
                    const int rlo = tm->reb[i][2];
                    const int rs = tm->reb[i][0];
                    if (v >= rlo && v <= tm->hi[rs]) {
                      tier_insert<ADAPT>(cnt, cp, topo, bits, stop, v, rs, tm->reb[i][1], rlo,
                                         tm->reb[i][3], lc);
                      break;
                    }
                  }
                }
              }
            }
            __syncthreads();
          }
          if (exited && newslot == -2) newslot = ht_find(tm->ht, node);
        }
        if (exited) {
          slot = newslot;  // -1: no slot, count directly
          p = 1;
          exited = false;
        }
      }
    }
    if (x < a.w) dst[z * a.dss + y * a.drs + x] = (T)res;
    __syncthreads();

    // Next window: every column drops row y-r and takes row y+r+1.
    if (y + 1 < ye) {
      const int64_t yo = clampi(y - r, a.h - 1), yi = clampi(y + r + 1, a.h - 1);
      if (yo != yi) {
        for (int lc = tid; lc < ncols; lc += kBlock) {
          const int64_t cx = clampi(x0 - r - 1 + lc, a.w - 1);
          for (int dz = -zr; dz <= zr; ++dz) {
            const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
            const int v = src[zz * a.sss + yo * a.srs + cx];
            column_walk<TIERED, ADAPT>(cnt, cp, tm, topo, root, bits, stop, v, lc, false);
          }
          for (int dz = -zr; dz <= zr; ++dz) {
            const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
            const int v = src[zz * a.sss + yi * a.srs + cx];
            column_walk<TIERED, ADAPT>(cnt, cp, tm, topo, root, bits, stop, v, lc, true);
          }
        }
      }
      __syncthreads();
    }
  }
}

template <typename T, bool TIERED, bool ADAPT, bool D3>
hipError_t launch_t(const MedianArgs& a, size_t lds, hipStream_t stream) {
  auto kern = k_median<T, TIERED, ADAPT, D3>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t grid = (int64_t)a.strips * a.segs * a.d;
  hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(kBlock), lds, stream, a);
  return hipGetLastError();
}

}  // namespace

size_t median_lds_bytes(int bytes, bool adaptive, bool tiered, int ncols, int cp, int nslots) {
  (void)bytes;
  (void)ncols;
  const size_t nodes = tiered ? kTierNodes : kDenseNodes;
  size_t b = ((size_t)(tiered ? nslots : 1) * nodes * cp + 15) & ~(size_t)15;
  if (tiered) b += sizeof(TierMeta);
  else if (adaptive) b += sizeof(TopoNode) * (kDenseNodes + 1);
  return b;
}

hipError_t launch_median(const MedianArgs& a, int bytes, int dims, bool adaptive, bool tiered,
                         hipStream_t stream) {
  const size_t lds = median_lds_bytes(bytes, adaptive, tiered, a.ncols, a.cp, a.nslots);
  const bool d3 = dims == 3;
#define HRRM_L(T, TI, AD, D3)                                            \
  if (tiered == TI && adaptive == AD && d3 == D3)                        \
    return launch_t<T, TI, AD, D3>(a, lds, stream);
  if (bytes == 1) {
    HRRM_L(uint8_t, false, false, false)
    HRRM_L(uint8_t, false, false, true)
    HRRM_L(uint8_t, false, true, false)
    HRRM_L(uint8_t, false, true, true)
    HRRM_L(uint8_t, true, false, false)
    HRRM_L(uint8_t, true, false, true)
    HRRM_L(uint8_t, true, true, false)
    HRRM_L(uint8_t, true, true, true)
  } else {
    HRRM_L(uint16_t, true, false, false)
    HRRM_L(uint16_t, true, false, true)
    HRRM_L(uint16_t, true, true, false)
    HRRM_L(uint16_t, true, true, true)
  }
#undef HRRM_L
  return hipErrorInvalidValue;
}

}  // namespace hrrm
