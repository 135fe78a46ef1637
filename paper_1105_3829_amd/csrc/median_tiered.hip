// Tiered running-median kernel for gfx950: 16-bit data (uniform or adaptive
// tree) and adaptive 8-bit data.
//
// Method: Alekseychuk, "Hierarchical Recursive Running Median".  Every column
// of a strip keeps an implicit interval-occurrences tree over the 2r+1 rows of
// the current window (Sec. III, Sec. III-A): one counter per left node, the
// top node elided.  A row step removes one value from and inserts one value
// into each column tree (Sec. III-B).  The descent of get_order_statistic
// (Sec. III) compares window counts of left nodes with K minus the
// left-occurrence accumulator, level by level.
//
// Tiers.  The tree is cut into 4-level subtrees ("tiers").  A column keeps the
// 15 left-node counters of one tier subtree as a 16-byte vector, so one 128-bit
// LDS read delivers a column's counts for four levels and the descent resolves
// four levels per window count (radix 16).  Tier 1 (the top) is always held.
// Deeper subtrees are materialised in LDS slots only when a pixel of the current
// row descends into them and are then maintained by the row updates while rows
// keep using them (least recently used replacement) - the paper's on-demand
// principle (window counts only for nodes the descent visits) applied to the
// column trees.
//
// Window counts of a tier for the 64 pixels of a wave:
//  * cooperative: lanes sharing a slot read the counters of the column entering
//    and leaving their window; a DPP prefix sum over the wave gives every
//    pixel's count as the count of the wave's first window plus the running
//    sum of (entering - leaving) - the paper's elementary window update
//    (one add, one subtract per node), for 64 pixels at once;
//  * direct: each lane sums the 2r+1 column vectors of its own window (the
//    paper's non-elementary catch-up), used when the wave's pixels are spread
//    over several subtrees.
// A subtree no slot holds (every slot serves the current row, or too few lanes
// want it to be worth a slot) is counted by the wave itself: for a few such
// subtrees the wave builds each one's column vectors for just its own 64+2r
// columns from the raw window values in a per-wave scratch area and sums
// those; when its lanes want many different subtrees (medians that change fast
// along the row, as at edges) every such lane instead histograms the raw
// values of its own window that fall in its subtree, one LDS-staged window row
// at a time - the paper's non-elementary update from scratch, O(window) per
// pixel, with no slot traffic.
//
// Uniform trees locate tier roots arithmetically (prefix of the value) and map
// them to slots with a direct table; adaptive trees (Sec. III-C) follow the
// topology table and map tier roots with a small hash.
#include "hrrm_internal.h"
#include "topo_mask.hpp"
#include "wave.hpp"

#include <type_traits>

namespace hrrm {
namespace {

constexpr int kMissGroups = 8;  // subtree groups per wave and round offered to the slots
constexpr int kMissCap = kMissGroups * kWaves;  // misses queued per round
constexpr int kSlotLanes = 4;   // lanes that must share a subtree to claim a slot in a wave
                                // that wants more than kMissGroups different subtrees
constexpr int kRebRows = 8;     // window rows a slot rebuild loads per column before using any
constexpr int kSmap = 16 + 256 + 4096;  // roots of tiers 2..4 of a 16-bit uniform tree
constexpr uint32_t kNone = 0xffu;

template <int NSMAP>
struct TierStateT {
  uint4 lut[16];                 // uniform insertion masks of a 4-level subtree
  uint8_t smap[NSMAP];           // uniform: tier-root key -> slot (kNone = absent)
  uint32_t ht[kHash];            // adaptive: (node + 1) << 8 | slot, 0 = empty
  int32_t key[kMaxSlots], lo[kMaxSlots], hi[kMaxSlots], dep[kMaxSlots], stamp[kMaxSlots];
  int32_t miss_n[3];
  int32_t flag[3][kWaves];
  int32_t reb_n;
  int32_t pad;
  uint32_t vand, vor;            // AND / OR of every value the tile reads
  int32_t miss[kMissCap][4];     // key, lo, hi, depth of a subtree root nobody holds
  int32_t reb[kMissCap][4];      // slot, key, lo, depth of a slot to rebuild
};
// 8-bit trees have one tier below the first: 16 possible subtree roots
template <typename T>
using TierState = TierStateT<sizeof(T) == 1 ? 16 : kSmap>;

__device__ __forceinline__ uint32_t ht_hash(int key) {
  return ((uint32_t)key * 2654435761u) >> 25;  // 7 bits for kHash = 128
}

__device__ __forceinline__ int ht_find(const uint32_t* ht, int key) {
  const uint32_t h = ht_hash(key), tag = (uint32_t)(key + 1);
  for (int i = 0; i < kHash; ++i) {
    const uint32_t e = ht[(h + i) & (kHash - 1)];
    if (e == 0) return -1;
    if ((e >> 8) == tag) return (int)(e & 0xffu);
  }
  return -1;
}

__device__ __forceinline__ void ht_insert(uint32_t* ht, int key, int slot) {
  const uint32_t h = ht_hash(key);
  for (int i = 0; i < kHash; ++i) {
    uint32_t& e = ht[(h + i) & (kHash - 1)];
    if (e == 0) {
      e = ((uint32_t)(key + 1) << 8) | (uint32_t)slot;
      return;
    }
  }
}

// Uniform tree: table index of the tier subtree whose root lies `rel` (4, 8,
// 12) levels below the tile's first tier, for values whose `rel` bits below
// the tile's common prefix are `pre`.
__device__ __forceinline__ int ukey(int rel, int pre) { return (((1 << rel) - 16) / 15) + pre; }

// Uniform tree: the four value bits that choose the path through the tier
// subtree rooted at depth `dep` (bits past the last level read as zero; the
// level mask drops the levels they would select).
__device__ __forceinline__ int nib(int v, int dep, int bits) {
  const int s = bits - dep - kTierLevels;
  return (s >= 0 ? v >> s : v << -s) & 15;
}

// Bytes of the levels of a tier subtree that are maintained: levels
// 0..nlev-1 occupy bytes 0 .. 2^nlev - 2.
__device__ __forceinline__ uint4 level_mask(int nlev) {
  const int nb = (1 << nlev) - 1;  // bytes kept
  uint4 m;
  m.x = nb >= 4 ? 0xffffffffu : (nb <= 0 ? 0u : (0xffffffffu >> (32 - 8 * nb)));
  m.y = nb >= 8 ? 0xffffffffu : (nb <= 4 ? 0u : (0xffffffffu >> (32 - 8 * (nb - 4))));
  m.z = nb >= 12 ? 0xffffffffu : (nb <= 8 ? 0u : (0xffffffffu >> (32 - 8 * (nb - 8))));
  m.w = nb >= 16 ? 0xffffffffu : (nb <= 12 ? 0u : (0xffffffffu >> (32 - 8 * (nb - 12))));
  return m;
}

__device__ __forceinline__ uint4 and4(uint4 a, uint4 b) {
  return make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w);
}
__device__ __forceinline__ uint4 add4(uint4 a, uint4 b) {
  return make_uint4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ uint4 sub4(uint4 a, uint4 b) {
  return make_uint4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}

__device__ __forceinline__ uint4& vec(uint8_t* slots, size_t cp16, int slot, int col) {
  return *(uint4*)(slots + (size_t)slot * cp16 + (size_t)col * 16);
}

// Adaptive trees: LDS copy of a held tier subtree's topology, 16 entries per
// slot (entry p-1 = the node at heap position p of the subtree, split < 0 =
// no node there).  The children of positions 8..15 are the roots of the next
// tier.  Filled from the global table when a slot is assigned.
__device__ __forceinline__ void fill_subtree(TopoNode* st, const TopoNode* topo, int root) {
  st[0] = topo[root];
  for (int p = 1; p <= 7; ++p) {
    const TopoNode e = st[p - 1];
    const TopoNode none = {-1, -1, -1, 0};
    st[2 * p - 1] = (e.split >= 0 && e.left >= 0) ? topo[e.left] : none;
    st[2 * p] = (e.split >= 0 && e.right >= 0) ? topo[e.right] : none;
  }
  const TopoNode none = {-1, -1, -1, 0};
  st[15] = none;
}

// Insertion mask of value v in a held adaptive subtree (its LDS topology);
// *next receives the node the value reaches below the subtree (< 0: a leaf).
__device__ __forceinline__ uint4 smask(const TopoNode* st, int dep, int stop, int v, int* next) {
  uint32_t m[4] = {0u, 0u, 0u, 0u};
  int p = 1, nd = 0;
#pragma unroll
  for (int k = 0; k < kTierLevels; ++k) {
    if (dep + k >= stop) {
      nd = -1;
      break;
    }
    const TopoNode t = st[p - 1];
    const bool left = v < t.split;
    if (left) {
      const int b = p - 1;
      m[b >> 2] |= 1u << ((b & 3) * 8);
    }
    nd = left ? t.left : t.right;
    if (nd < 0) break;
    p = 2 * p + (left ? 0 : 1);
  }
  *next = nd;
  return make_uint4(m[0], m[1], m[2], m[3]);
}

// Count of node q (0..14) from the packed window counts: word 2i holds nodes
// 4i and 4i+2, word 2i+1 nodes 4i+1 and 4i+3 (16-bit fields).  The words come
// in by value: selecting between elements of an array argument lets the
// compiler turn the selects into one dynamically indexed load, which keeps the
// caller's counts in private (scratch) memory.
__device__ __forceinline__ uint32_t wsel(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                         uint32_t w4, uint32_t w5, uint32_t w6, uint32_t w7,
                                         int q) {
  const int i = q >> 2;
  const bool odd = q & 1;
  const uint32_t a0 = odd ? w1 : w0;
  const uint32_t a1 = odd ? w3 : w2;
  const uint32_t a2 = odd ? w5 : w4;
  const uint32_t a3 = odd ? w7 : w6;
  const uint32_t b0 = (i & 1) ? a1 : a0;
  const uint32_t b1 = (i & 1) ? a3 : a2;
  const uint32_t c = (i & 2) ? b1 : b0;
  return (q & 2) ? (c >> 16) : (c & 0xffffu);
}

// Cooperative window counts of slot s for all lanes (see file comment); lanes
// with member=true keep the result.  All 64 lanes must be active.
__device__ __forceinline__ void coop_counts(uint32_t (&W)[8], const uint8_t* slots, size_t cp16,
                                            int s, bool member, int lx, int span, int lane,
                                            int wbase) {
  const uint8_t* sb = slots + (size_t)s * cp16;
  const uint4 vin = *(const uint4*)(sb + (size_t)(lx + span) * 16);  // column x + r
  const uint4 vout = *(const uint4*)(sb + (size_t)lx * 16);          // column x - r - 1
  uint32_t ex[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  if (span > 64) {  // the first window spans more than the wave's 64 leaving columns
    for (int k = 64 + lane; k < span; k += 64) {
      const uint4 e = *(const uint4*)(sb + (size_t)(wbase + k) * 16);
      const uint32_t ev[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ex[2 * i] += ev[i] & 0x00ff00ffu;
        ex[2 * i + 1] += (ev[i] >> 8) & 0x00ff00ffu;
      }
    }
  }
  const int bl = span <= 64 ? span - 1 : 63;
  const uint32_t vi[4] = {vin.x, vin.y, vin.z, vin.w};
  const uint32_t vo[4] = {vout.x, vout.y, vout.z, vout.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t il = wave_scan(vi[i] & 0x00ff00ffu);
    const uint32_t ih = wave_scan((vi[i] >> 8) & 0x00ff00ffu);
    const uint32_t ol = wave_scan(vo[i] & 0x00ff00ffu);
    const uint32_t oh = wave_scan((vo[i] >> 8) & 0x00ff00ffu);
    uint32_t bl0 = readlane_u(ol, bl), bh0 = readlane_u(oh, bl);
    if (span > 64) {
      bl0 += readlane_u(wave_scan(ex[2 * i]), 63);
      bh0 += readlane_u(wave_scan(ex[2 * i + 1]), 63);
    }
    if (member) {
      W[2 * i] = bl0 + il - ol;
      W[2 * i + 1] = bh0 + ih - oh;
    }
  }
}

typedef int v2i_t __attribute__((ext_vector_type(2)));
typedef int v4i_t __attribute__((ext_vector_type(4)));

// Window counts as a matrix product on the matrix cores.  For the tier subtree
// of one slot and the wave's 64 pixels, counts[node][pixel] =
// sum_k col[k][node] * band[k][pixel], where k runs over the 64 + 2r columns
// the wave's windows cover and band[k][pixel] = 1 when column k lies in the
// pixel's window - the paper's window update (Sec. III) summed for all nodes
// of the tier at once.  Column counts enter as signed bytes (8-bit 2-D
// windows of 2r + 1 <= 127 rows: the only launches that enable it).
//
// Operands of v_mfma_i32_16x16x64_i8: lane l holds A[i = l % 16][k = 16(l/16)
// + b] and B[k = 16(l/16) + b][j = l % 16] for b = 0..15, and receives
// D[4(l/16) + v][l % 16] for v = 0..3.  Here A = column counts (node x k),
// read transposed from the column-major slot by ds_read_b64_tr_b8: lane t of a
// 16-lane group names half t % 2 of column c0 + t / 2, and receives node t of
// columns c0 .. c0 + 7.  B = band (k x pixel), built once per tile.  The sum
// runs over k in any order, so k = 16g + 8h + j of a 64-column step stands for
// column 32h + 8g + j: each of the two reads of a step then covers 32
// consecutive columns (512 contiguous bytes) across the wave.
struct Band {
  v4i_t f[3][4];  // [64-column step][16-pixel tile]
  int steps;      // 64-column steps (64 + 2r columns: 2r + 1 <= 129)
};

__device__ __forceinline__ void band_init(Band& bd, int span, int lane) {
  const int g = lane >> 4, t = lane & 15;
  bd.steps = (64 + span - 1 + 63) >> 6;
#pragma unroll
  for (int ks = 0; ks < 3; ++ks)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      uint32_t w[4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // bytes j of half h with 0 <= column - p < span, column = 64ks + 32h
        // + 8g + j, p = 16nt + t
        const int d = 64 * ks + 32 * h + 8 * g - 16 * nt - t;
        const int jlo = -d < 0 ? 0 : (-d > 8 ? 8 : -d);
        const int jhi = span - d < 0 ? 0 : (span - d > 8 ? 8 : span - d);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          uint32_t x = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b)
            x |= (4 * q + b >= jlo && 4 * q + b < jhi) ? 1u << (8 * b) : 0u;
          w[2 * h + q] = x;
        }
      }
      bd.f[ks][nt] = v4i_t{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
    }
}

// Counts of slot s for the pixels of `m` into the wave's staging area, in
// the packed layout wsel reads: the two words of node rows 4g..4g+3 of pixel
// p at g * 512 + p * 8 bytes, so that 16 lanes of one row group store, and
// all 64 lanes load, consecutive 8-byte words (no bank conflicts).  All 64
// lanes must call it.
__device__ __forceinline__ void mfma_group(const Band& bd, const uint8_t* slots, size_t cp16,
                                           int cmax, int s, uint64_t m, int wbase, int lane,
                                           uint8_t* stage) {
  const int g = lane >> 4, t = lane & 15;
  const uint8_t* sb = slots + (size_t)s * cp16;
  const int cb = wbase + 1;  // first window column of the wave's first pixel
  v4i_t acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
  for (int ks = 0; ks < 3; ++ks) {
    if (ks < bd.steps) {
      v4i_t a;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        int c = cb + 64 * ks + 32 * h + 8 * g + (t >> 1);
        c = c < cmax ? c : cmax;  // past the slot's columns: band weight 0
        const v2i_t rr = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
            (v2i_t __attribute__((address_space(3)))*)(sb + (size_t)c * 16 + 8 * (t & 1)));
        a[2 * h] = rr.x;
        a[2 * h + 1] = rr.y;
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bd.f[ks][nt], acc[nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int p = 16 * nt + t;
    if ((m >> p) & 1) {
      const uint32_t w0 = (uint32_t)acc[nt][0] | ((uint32_t)acc[nt][2] << 16);
      const uint32_t w1 = (uint32_t)acc[nt][1] | ((uint32_t)acc[nt][3] << 16);
      *(uint2*)(stage + g * 512 + p * 8) = make_uint2(w0, w1);
    }
  }
}

// Direct window counts: this lane sums the 2r+1 column vectors of its window.
// Bytes are summed `batch` columns at a time (no byte overflows) and then
// widened to 16-bit fields.
__device__ __forceinline__ void direct_counts(uint32_t (&W)[8], const uint8_t* slots, size_t cp16,
                                              int s, int lx, int span, int batch) {
  const uint8_t* p = slots + (size_t)s * cp16 + (size_t)(lx + 1) * 16;
#pragma unroll
  for (int i = 0; i < 8; ++i) W[i] = 0;
  for (int j0 = 0; j0 < span; j0 += batch) {
    const int jn = j0 + batch < span ? j0 + batch : span;
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll 4
    for (int j = j0; j < jn; ++j) {
      const uint4 v = *(const uint4*)(p + (size_t)j * 16);
      a0 += v.x;
      a1 += v.y;
      a2 += v.z;
      a3 += v.w;
    }
    W[0] += a0 & 0x00ff00ffu;
    W[1] += (a0 >> 8) & 0x00ff00ffu;
    W[2] += a1 & 0x00ff00ffu;
    W[3] += (a1 >> 8) & 0x00ff00ffu;
    W[4] += a2 & 0x00ff00ffu;
    W[5] += (a2 >> 8) & 0x00ff00ffu;
    W[6] += a3 & 0x00ff00ffu;
    W[7] += (a3 >> 8) & 0x00ff00ffu;
  }
}

// Wave-local stand-in for a subtree no slot holds: the wave's lanes build its
// column vectors for the 64+2r columns the wave's windows cover, from the raw
// window values (loads coalesced across lanes), into the wave's scratch area.
// The caller then sums them per lane like a held slot.  Nothing is kept for
// later rows.
template <typename T, bool ADAPT, bool D3, int NB = kRebRows, typename TS>
__device__ __forceinline__ void scratch_build(uint8_t* scr, const T* __restrict__ src,
                                              const MedianArgs& a, const TS* ts,
                                              const TopoNode* topo, int64_t x0w, int64_t y,
                                              int64_t z, int lane, int span, int node, int rlo,
                                              int rhi, int rdep) {
  constexpr int bits = 8 * sizeof(T);
  const int r = a.r, zr = D3 ? r : 0, stop = a.stop;
  const uint4 lim = level_mask(stop - rdep < kTierLevels ? stop - rdep : kTierLevels);
  if constexpr (NB <= 1) {  // one row at a time: fewest registers
    if constexpr (D3) {  // stepped row offsets (measured faster here)
      for (int c = lane; c <= 64 + span - 1; c += 64) {
        const T* col = src + clampi(x0w - r - 1 + c, a.w - 1);
        uint4 acc = make_uint4(0u, 0u, 0u, 0u);
        RowWalk<D3> rw(y, z, a.h, a.d, a.srs, a.sss, r, zr);
        for (int dz = -zr; dz <= zr; ++dz) {
#pragma unroll 4
          for (int j = -r; j <= r; ++j) {
            const int v = col[rw.off];
            rw.next();
            if (v >= rlo && v <= rhi) {
              if constexpr (ADAPT)
                acc = add4(acc, amask(topo, node, rdep, stop, v));
              else
                acc = add4(acc, and4(ts->lut[nib(v, rdep, bits)], lim));
            }
          }
        }
        *(uint4*)(scr + (size_t)c * 16) = acc;
      }
      return;
    }
    for (int c = lane; c <= 64 + span - 1; c += 64) {
      const int64_t cx = clampi(x0w - r - 1 + c, a.w - 1);
      uint4 acc = make_uint4(0u, 0u, 0u, 0u);
      for (int dz = -zr; dz <= zr; ++dz) {
        const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
#pragma unroll 4
        for (int j = -r; j <= r; ++j) {
          const int v = src[zz * a.sss + clampi(y + j, a.h - 1) * a.srs + cx];
          if (v >= rlo && v <= rhi) {
            if constexpr (ADAPT)
              acc = add4(acc, amask(topo, node, rdep, stop, v));
            else
              acc = add4(acc, and4(ts->lut[nib(v, rdep, bits)], lim));
          }
        }
      }
      *(uint4*)(scr + (size_t)c * 16) = acc;
    }
    return;
  }
  // the (2zr + 1) x span window rows of each column, slice-major, NB loaded
  // before any is used (their latencies overlap)
  const int nrows = (2 * zr + 1) * span;
  if constexpr (sizeof(T) == 2) {  // stepped row offsets (measured faster here)
    for (int c = lane; c <= 64 + span - 1; c += 64) {
      const T* col = src + clampi(x0w - r - 1 + c, a.w - 1);
      uint4 acc = make_uint4(0u, 0u, 0u, 0u);
      RowWalk<D3> rw(y, z, a.h, a.d, a.srs, a.sss, r, zr);
      for (int q0 = 0; q0 < nrows; q0 += NB) {
        int v[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          // rows past the window are clamped into the image, loaded and skipped
          v[k] = col[rw.off];
          rw.next();
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          if (q0 + k < nrows && v[k] >= rlo && v[k] <= rhi) {
            if constexpr (ADAPT)
              acc = add4(acc, amask(topo, node, rdep, stop, v[k]));
            else
              acc = add4(acc, and4(ts->lut[nib(v[k], rdep, bits)], lim));
          }
        }
      }
      *(uint4*)(scr + (size_t)c * 16) = acc;
    }
    return;
  }
  for (int c = lane; c <= 64 + span - 1; c += 64) {
    const int64_t cx = clampi(x0w - r - 1 + c, a.w - 1);
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    int dz = -zr, j = -r;
    for (int q0 = 0; q0 < nrows; q0 += NB) {
      int v[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        // rows past the window are clamped into the image, loaded and skipped
        const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
        v[k] = src[zz * a.sss + clampi(y + j, a.h - 1) * a.srs + cx];
        if (++j > r) {
          j = -r;
          ++dz;
        }
      }
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (q0 + k < nrows && v[k] >= rlo && v[k] <= rhi) {
          if constexpr (ADAPT)
            acc = add4(acc, amask(topo, node, rdep, stop, v[k]));
          else
            acc = add4(acc, and4(ts->lut[nib(v[k], rdep, bits)], lim));
        }
      }
    }
    *(uint4*)(scr + (size_t)c * 16) = acc;
  }
}

// Per-lane counts of a tier subtree straight from the raw window values (for
// small windows this is cheaper than building the subtree's column vectors).
template <typename T, bool ADAPT, bool D3, typename TS>
__device__ __forceinline__ void raw_counts(uint32_t (&W)[8], const T* __restrict__ src,
                                           const MedianArgs& a, const TS* ts,
                                           const TopoNode* topo, int64_t x, int64_t y, int64_t z,
                                           int node, int rlo, int rhi, int rdep) {
  constexpr int bits = 8 * sizeof(T);
  const int r = a.r, zr = D3 ? r : 0, stop = a.stop;
  const uint4 lim = level_mask(stop - rdep < kTierLevels ? stop - rdep : kTierLevels);
#pragma unroll
  for (int i = 0; i < 8; ++i) W[i] = 0;
  // adaptive: the lane's subtree is read once and held in registers, so a
  // value's mask takes no memory access
  SubtreeRegs sq = {};
  if constexpr (ADAPT) sq = load_subtree_regs(topo, node);
  for (int dz = -zr; dz <= zr; ++dz) {
    const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
    for (int dy = -r; dy <= r; ++dy) {
      const T* rowp = src + zz * a.sss + clampi(y + dy, a.h - 1) * a.srs;
      for (int dx = -r; dx <= r; ++dx) {
        const int v = rowp[clampi(x + dx, a.w - 1)];
        if (v >= rlo && v <= rhi) {
          uint4 m;
          if constexpr (ADAPT)
            m = and4(amask_regs(sq, v), lim);
          else
            m = and4(ts->lut[nib(v, rdep, bits)], lim);
          W[0] += m.x & 0x00ff00ffu;
          W[1] += (m.x >> 8) & 0x00ff00ffu;
          W[2] += m.y & 0x00ff00ffu;
          W[3] += (m.y >> 8) & 0x00ff00ffu;
          W[4] += m.z & 0x00ff00ffu;
          W[5] += (m.z >> 8) & 0x00ff00ffu;
          W[6] += m.w & 0x00ff00ffu;
          W[7] += (m.w >> 8) & 0x00ff00ffu;
        }
      }
    }
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Uniform tree: window counts of each needing lane's own tier subtree (root at
// depth dep, interval starting at lo) from the raw window values.  The wave
// stages every window row (64 + 2r values) in LDS once; each needing lane adds
// the values of its window that fall in its interval to a private 16-bin
// histogram of the four value bits below dep; the 15 left-node counts follow
// from the bins.  All 64 lanes must call it; buf is the wave's scratch area.
template <typename T, bool D3, bool PIPE>
__device__ __forceinline__ void raw_wave(uint32_t (&W)[8], bool need, int lo, int dep,
                                         uint8_t* buf, const T* __restrict__ src,
                                         const MedianArgs& a, int64_t x0w, int64_t y, int64_t z,
                                         int lane) {
  constexpr int bits = 8 * sizeof(T);
  const int r = a.r, span = 2 * r + 1, zr = D3 ? r : 0;
  uint32_t* hist = (uint32_t*)buf;  // bins 2k, 2k+1 of lane l: 16-bit halves of hist[k * 64 + l]
  T* stage = (T*)(buf + 8 * 64 * 4);
  const uint32_t width = need ? 1u << (bits - dep) : 0u;
#pragma unroll
  for (int k = 0; k < 8; ++k) hist[k * 64 + lane] = 0;
  if constexpr (!PIPE) {  // one row at a time: fewest registers
    for (int dz = -zr; dz <= zr; ++dz) {
      const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
      for (int dy = -r; dy <= r; ++dy) {
        const T* rowp = src + zz * a.sss + clampi(y + dy, a.h - 1) * a.srs;
        for (int c = lane; c < 64 + 2 * r; c += 64) stage[c] = rowp[clampi(x0w - r + c, a.w - 1)];
        wave_sync_lds();
        if (need) {
          for (int dx = 0; dx < span; ++dx) {
            const uint32_t v = stage[lane + dx];
            if (v - (uint32_t)lo < width) {
              const int bn = nib((int)v, dep, bits);
              atomicAdd(&hist[(bn >> 1) * 64 + lane], 1u << ((bn & 1) * 16));
            }
          }
        }
        wave_sync_lds();
      }
    }
  } else {
    // lane l stages columns l, l + 64, ... of each window row (64 + 2r
    // values); the first two of the next row are loaded into registers before
    // the current row is counted, so their latency overlaps the counting
    const int nrows = (2 * zr + 1) * span;
    const int nstage = 64 + 2 * r;
    auto row_ptr = [&](int dz, int dy) -> const T* {
      const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
      return src + zz * a.sss + clampi(y + dy, a.h - 1) * a.srs;
    };
    int qdz = -zr, qdy = -r;  // the current row
    const T* rp = row_ptr(qdz, qdy);
    T c0 = rp[clampi(x0w - r + lane, a.w - 1)];
    T c1 = lane + 64 < nstage ? rp[clampi(x0w - r + lane + 64, a.w - 1)] : (T)0;
    for (int q = 0; q < nrows; ++q) {
      stage[lane] = c0;
      if (lane + 64 < nstage) stage[lane + 64] = c1;
      for (int c = lane + 128; c < nstage; c += 64) stage[c] = rp[clampi(x0w - r + c, a.w - 1)];
      int ndz = qdz, ndy = qdy + 1;
      if (ndy > r) {
        ndy = -r;
        ++ndz;
      }
      const T* np = row_ptr(ndz, ndy);  // clamped into the image past the last row
      T n0 = (T)0, n1 = (T)0;
      if (q + 1 < nrows) {
        n0 = np[clampi(x0w - r + lane, a.w - 1)];
        if (lane + 64 < nstage) n1 = np[clampi(x0w - r + lane + 64, a.w - 1)];
      }
      wave_sync_lds();
      if (need) {
        for (int dx = 0; dx < span; ++dx) {
          const uint32_t v = stage[lane + dx];
          if (v - (uint32_t)lo < width) {
            const int bn = nib((int)v, dep, bits);
            atomicAdd(&hist[(bn >> 1) * 64 + lane], 1u << ((bn & 1) * 16));
          }
        }
      }
      wave_sync_lds();
      c0 = n0;
      c1 = n1;
      qdz = ndz;
      qdy = ndy;
      rp = np;
    }
  }
  if (need) {
    uint32_t bin[16];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t hk = hist[k * 64 + lane];
      bin[2 * k] = hk & 0xffffu;
      bin[2 * k + 1] = hk >> 16;
    }
    // left-node counts in heap order (node q = heap position q + 1)
    uint32_t c[15];
    c[0] = bin[0] + bin[1] + bin[2] + bin[3] + bin[4] + bin[5] + bin[6] + bin[7];
    c[1] = bin[0] + bin[1] + bin[2] + bin[3];
    c[2] = bin[8] + bin[9] + bin[10] + bin[11];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[3 + i] = bin[4 * i] + bin[4 * i + 1];
#pragma unroll
    for (int i = 0; i < 8; ++i) c[7 + i] = bin[2 * i];
#pragma unroll
    for (int i = 0; i < 8; ++i) W[i] = 0;
#pragma unroll
    for (int q = 0; q < 15; ++q) W[2 * (q >> 2) + (q & 1)] |= c[q] << (16 * ((q >> 1) & 1));
  }
  wave_sync_lds();  // the scratch area is reused right after
}

// Slot assignment for this round's misses (thread 0): least recently used
// slots not used by the current row are replaced.  Adaptive trees also drop the
// held subtrees below a replaced slot (their updates walk down from the top and
// stop at the first subtree no slot holds).
// Adaptive trees: are all tier subtrees above the one rooted at `key` (depth
// dep, interval starting at lo) held?  Column updates walk down from the top
// and stop at the first subtree no slot holds, so a subtree below one that is
// not held would go stale.  The path follows lo through the topology.
template <typename TS>
__device__ __forceinline__ bool ancestors_held(const TS* ts, const TopoNode* topo, int root,
                                               int lo, int dep) {
  int nd = root;
  for (int d = kTierLevels; d < dep; d += kTierLevels) {
    for (int k = 0; k < kTierLevels && nd >= 0; ++k) {
      const TopoNode t = topo[nd];
      nd = lo < t.split ? t.left : t.right;
    }
    if (nd < 0 || ht_find(ts->ht, nd) < 0) return false;
  }
  return true;
}

template <bool ADAPT, typename TS>
__device__ void assign_slots(TS* ts, int nmiss, int stamp, int nslots, TopoNode* stopo,
                             const TopoNode* topo, int root) {
  int nreb = 0;
  for (int i = 0; i < nmiss; ++i) {
    const int key = ts->miss[i][0];
    const bool held = ADAPT ? ht_find(ts->ht, key) >= 0 : ts->smap[key] != kNone;
    if (held) continue;  // duplicate from another wave
    if constexpr (ADAPT) {
      if (!ancestors_held(ts, topo, root, ts->miss[i][1], ts->miss[i][3])) continue;
    }
    int victim = -1, best = 0x7fffffff;
    for (int s = 1; s < nslots; ++s) {
      const int st = ts->stamp[s];
      if (st != stamp && st < best) {
        best = st;
        victim = s;
      }
    }
    if (victim < 0) continue;  // every slot serves this row: these pixels count directly
    if (ts->key[victim] >= 0) {
      if constexpr (ADAPT) {
        const int vlo = ts->lo[victim], vhi = ts->hi[victim], vdep = ts->dep[victim];
        for (int s = 1; s < nslots; ++s)
          if (ts->key[s] >= 0 &&
              (s == victim || (ts->dep[s] > vdep && ts->lo[s] >= vlo && ts->lo[s] <= vhi))) {
            ts->key[s] = -1;
            ts->stamp[s] = -1;
          }
        for (int h = 0; h < kHash; ++h) ts->ht[h] = 0;
        for (int s = 1; s < nslots; ++s)
          if (ts->key[s] >= 0) ht_insert(ts->ht, ts->key[s], s);
      } else {
        ts->smap[ts->key[victim]] = (uint8_t)kNone;
      }
    }
    ts->key[victim] = key;
    ts->lo[victim] = ts->miss[i][1];
    ts->hi[victim] = ts->miss[i][2];
    ts->dep[victim] = ts->miss[i][3];
    ts->stamp[victim] = stamp;
    if constexpr (ADAPT) {
      ht_insert(ts->ht, key, victim);
      fill_subtree(stopo + victim * 16, topo, key);
    } else {
      ts->smap[key] = (uint8_t)victim;
    }
    ts->reb[nreb][0] = victim;
    ts->reb[nreb][1] = key;
    ts->reb[nreb][2] = ts->miss[i][1];
    ts->reb[nreb][3] = ts->miss[i][3];
    ++nreb;
  }
  ts->reb_n = nreb;
}

// One workgroup tile: output columns [strip*256, strip*256 + 256) of rows
// [seg*seg_rows, seg*seg_rows + seg_rows) of slice z.  `lds` is the dynamic LDS
// of the workgroup (slots, tier state, per-wave scratch).  MF = false leaves
// the matrix-core counts (and the 48 registers of their band) out; such
// builds serve only launches that count no subtree wave-wide (max_groups 0).
// WPS = true (uniform 2-D trees): the workgroup shares only slot 0 (tier 1);
// each wave holds its own a.wslots slots of deeper subtrees, for just the
// 64 + 2r + 1 columns its windows cover, and finds, builds, evicts and updates
// them by itself, so tier transitions need no workgroup barrier.
template <typename T, bool ADAPT, bool D3, bool MF = true, bool WPS = false>
__device__ __forceinline__ void tile_body(const MedianArgs& a, uint8_t* lds, int strip, int seg,
                                          int64_t z) {
  const T* __restrict__ src = (const T*)a.src;
  T* __restrict__ dst = (T*)a.dst;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int bits = 8 * sizeof(T);  // the tree height of the uniform tree
  const int r = a.r, ncols = a.ncols, stop = a.stop;
  const int span = 2 * r + 1;
  const int zr = D3 ? r : 0;
  const size_t cp16 = (size_t)a.cp * 16;  // bytes of one slot (cp >= ncols columns)
  const TopoNode* __restrict__ topo = a.topo;

  const int64_t x0 = (int64_t)strip * kBlock;
  const int64_t yb = (int64_t)seg * a.seg_rows;
  const int64_t ye = yb + a.seg_rows < a.h ? yb + a.seg_rows : a.h;

  static_assert(!WPS || (!ADAPT && !D3), "wave-private slots serve uniform 2-D trees");
  uint8_t* slots = lds;
  using TS = TierStateT<(sizeof(T) == 1 || WPS) ? 16 : kSmap>;
  TS* ts = (TS*)(lds + align16((size_t)a.nslots * cp16));
  // per-wave scratch of (64 + 2r + 1) column vectors for subtrees no slot
  // holds (WPS: followed by the wave's own slots)
  const size_t wpitch16 = (size_t)a.wpitch * 16;
  const size_t warea = wave_scratch_bytes(r) + (WPS ? (size_t)a.wslots * wpitch16 : 0);
  uint8_t* scr = lds + align16((size_t)a.nslots * cp16) + align16(sizeof(TS)) + (size_t)wv * warea;
  // WPS: the wave's slots, addressed by tile column (the wave's columns
  // 64 wv .. 64 wv + 64 + 2r start at its first slot)
  uint8_t* wslots = scr + wave_scratch_bytes(r) - (size_t)wv * 64 * 16;
  const int wcmax = wv * 64 + 64 + 2 * r;  // last tile column of the wave's slots
  // lane s < a.wslots describes wave slot s: interval start, depth (-1: empty)
  // and the last row that used it
  int wlo = -1, wdep = -1, wst = -1;
  // adaptive: topology of each held subtree (16 entries per slot) after the scratch
  TopoNode* stopo = (TopoNode*)(lds + align16((size_t)a.nslots * cp16) +
                                align16(sizeof(TS)) + (size_t)kWaves * wave_scratch_bytes(r));
  const int root = ADAPT ? topo[(1 << bits) - 1].split : 1;
  const int maxv = (1 << bits) - 1;
  constexpr int ntiers = (bits + kTierLevels - 1) / kTierLevels;

  // ---- set-up: tables, empty slots
  if (tid < 16) {
    uint32_t m[4] = {0u, 0u, 0u, 0u};
    for (int k = 0; k < kTierLevels; ++k) {
      const int pos = ((1 << k) | (tid >> (4 - k))) - 1;
      if (!((tid >> (3 - k)) & 1)) m[pos >> 2] |= 1u << ((pos & 3) * 8);
    }
    ts->lut[tid] = make_uint4(m[0], m[1], m[2], m[3]);
  }
  if constexpr (ADAPT) {
    for (int i = tid; i < kHash; i += kBlock) ts->ht[i] = 0;
  } else {
    for (int i = tid; i < (int)sizeof(ts->smap); i += kBlock) ts->smap[i] = (uint8_t)kNone;
  }
  for (int s = tid; s < kMaxSlots; s += kBlock) {
    ts->key[s] = -1;
    ts->stamp[s] = -1;
    ts->lo[s] = ts->hi[s] = ts->dep[s] = 0;
  }
  if (tid < 3) ts->miss_n[tid] = 0;
  if (tid < 3 * kWaves) ts->flag[tid / kWaves][tid % kWaves] = 0;
  if (tid == 0) {
    ts->reb_n = 0;
    ts->vand = 0xffffffffu;
    ts->vor = 0u;
    ts->key[0] = root;  // slot 0 holds tier 1 and is never replaced
    ts->stamp[0] = 0x7fffffff;
    ts->hi[0] = maxv;
    if constexpr (ADAPT) fill_subtree(stopo, topo, root);
  }
  __syncthreads();

  // Uniform 2-D trees of 16-bit data: the top `pl` levels of every window's
  // descent are fixed when all values the tile reads share their top `pl`
  // bits (12-bit data in 16-bit pixels: the top four levels always go left).
  // The tile's first tier then starts at depth pl with the common prefix `pfx`
  // as its interval's lower bound; the output is the same.
  int pl = 0, pfx = 0;
  if constexpr (!ADAPT && !D3 && sizeof(T) == 2) {
    const int64_t r0 = yb - r > 0 ? yb - r : 0;
    const int64_t r1 = ye - 1 + r < a.h - 1 ? ye - 1 + r : a.h - 1;
    uint32_t va = 0xffffffffu, vo = 0u;
    for (int lc = tid; lc < ncols; lc += kBlock) {
      const T* p = src + z * a.sss + clampi(x0 - r - 1 + lc, a.w - 1);
#pragma unroll 4
      for (int64_t yy = r0; yy <= r1; ++yy) {
        const uint32_t v = p[yy * a.srs];
        va &= v;
        vo |= v;
      }
    }
    atomicAnd(&ts->vand, va);
    atomicOr(&ts->vor, vo);
    __syncthreads();
    const uint32_t diff = __builtin_amdgcn_readfirstlane(ts->vand ^ ts->vor);
    pl = diff == 0u ? bits : __builtin_clz(diff) - (32 - bits);
    if (pl > stop) pl = stop;
    pfx = pl >= bits ? (int)__builtin_amdgcn_readfirstlane(ts->vand)
                     : (int)(__builtin_amdgcn_readfirstlane(ts->vand) & ~((1u << (bits - pl)) - 1u));
  }

  // First-tier insertion mask of value v.
  const uint4 lim1 = level_mask(stop - pl < kTierLevels ? stop - pl : kTierLevels);
  auto mask1 = [&](int v) -> uint4 {
    if constexpr (ADAPT) {
      int nx;
      return smask(stopo, 0, stop, v, &nx);
    } else
      return and4(ts->lut[nib(v, pl, bits)], lim1);
  };

  // ---- column trees (tier 1) of the segment's first window
  for (int lc = tid; lc < ncols; lc += kBlock) {
    const int64_t cx = clampi(x0 - r - 1 + lc, a.w - 1);
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    for (int dz = -zr; dz <= zr; ++dz) {
      const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
      for (int j = -r; j <= r; ++j) {
        const int v = src[zz * a.sss + clampi(yb + j, a.h - 1) * a.srs + cx];
        acc = add4(acc, mask1(v));
      }
    }
    vec(slots, cp16, 0, lc) = acc;
  }
  // the padding columns past ncols are never read
  __syncthreads();

  const int lx = wv * 64 + lane;  // output x = x0 + lx; window columns lx+1 .. lx+span
  const int64_t x = x0 + lx;
  const uint32_t K = (uint32_t)a.rank;
  const int maxcol = D3 ? span * span : span;  // largest column count
  // windows of at most kRawWindow values count a subtree no slot holds from the
  // raw values; windows of at most a.raw_window values never hold deeper tiers
  // in slots at all (every deeper tier is counted raw: no misses, no rebuilds)
  const bool raw_fallback = maxcol * span <= kRawWindow;
  const bool raw_only = maxcol * span <= a.raw_window;
  const int batch = 255 / maxcol > 0 ? 255 / maxcol : 1;
  // a wave whose slot-less lanes want more than `gs` different subtrees counts
  // them raw (one pass over the window per lane) rather than building each
  // one's column vectors (about (64 + 2r) / 64 window columns per lane each)
  const int gs = (9 * span) / ((12 * (64 + 2 * r)) / 64 + 6) > 1
                     ? (9 * span) / ((12 * (64 + 2 * r)) / 64 + 6)
                     : 1;
  const int maxrounds = ADAPT ? (3 * bits) / kTierLevels + 1 : (stop + kTierLevels - 1) / kTierLevels;
  Band band;
  if (MF && a.mfma) band_init(band, span, lane);
  int gr = 0;

  for (int64_t y = yb; y < ye; ++y) {
    // 2-D: fetch the values this row's column update will remove and insert now,
    // so their latency overlaps the descent (a thread owns at most 2 columns)
    int pre_o[2] = {0, 0}, pre_i[2] = {0, 0};
    if (!D3 && y + 1 < ye) {
      const int64_t yo = clampi(y - r, a.h - 1), yi = clampi(y + r + 1, a.h - 1);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int lc = tid + k * kBlock;
        if (lc < ncols) {
          const int64_t cx = clampi(x0 - r - 1 + lc, a.w - 1);
          pre_o[k] = src[z * a.sss + yo * a.srs + cx];
          pre_i[k] = src[z * a.sss + yi * a.srs + cx];
        }
      }
    }
    int node = root, lo = pfx, hi = pfx + (int)((1u << (bits - pl)) - 1u), depth = pl;
    uint32_t acc = 0;
    bool done = (x >= a.w) || (pl >= stop);
    int res = pfx;
    int slot = 0;

    for (int round = 0; round <= maxrounds; ++round) {
      const bool act = !done;
      // the slots this round's counts read: tier 1 and shared slots, or
      // (WPS, deeper tiers) the wave's own
      const bool own = WPS && round > 0;
      const uint8_t* cslots = own ? wslots : slots;
      const size_t ccp16 = own ? wpitch16 : cp16;
      const int cmax = own ? wcmax : a.cp - 1;
      const uint64_t pend = ballot(act && slot >= 0);
      uint32_t W[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
      if (pend) {
        // How many distinct subtrees do this wave's pixels need?
        int groups = 0;
        for (uint64_t t = pend; t && groups <= a.max_groups; ++groups)
          t &= ~ballot(slot == readlane(slot, __builtin_ctzll(t)));
        if (MF && groups <= a.max_groups && a.mfma) {
          for (uint64_t t = pend; t;) {
            const int s = readlane(slot, __builtin_ctzll(t));
            const uint64_t m = ballot(slot == s) & t;
            t &= ~m;
            mfma_group(band, cslots, ccp16, cmax, s, m, wv * 64, lane, scr);
          }
          wave_sync_lds();
          if ((pend >> lane) & 1) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              const uint2 u = *(const uint2*)(scr + g * 512 + lane * 8);
              W[2 * g] = u.x;
              W[2 * g + 1] = u.y;
            }
          }
          wave_sync_lds();  // the scratch area is reused below
        } else if (groups <= a.max_groups) {
          for (uint64_t t = pend; t;) {
            const int s = readlane(slot, __builtin_ctzll(t));
            const uint64_t m = ballot(slot == s) & t;
            t &= ~m;
            coop_counts(W, cslots, ccp16, s, (m >> lane) & 1, lx, span, lane, wv * 64);
          }
        } else if (act && slot >= 0) {
          direct_counts(W, cslots, ccp16, slot, lx, span, batch);
        }
      }
      // Pixels whose subtree no slot holds: small windows, and waves whose
      // lanes want many different subtrees, count their raw values; otherwise
      // the wave builds each such subtree once in scratch.
      const uint64_t nos = ballot(act && slot < 0);
      bool use_raw = raw_fallback;
      if (nos && !use_raw) {
        int g = 0;
        for (uint64_t t = nos; t && g <= gs; ++g) {
          const int leader = __builtin_ctzll(t);
          t &= ~ballot(lo == readlane(lo, leader) && depth == readlane(depth, leader));
        }
        use_raw = g > gs;
      }
      if (nos && use_raw) {
        if constexpr (ADAPT) {
          if (act && slot < 0) raw_counts<T, ADAPT, D3>(W, src, a, ts, topo, x, y, z, node, lo, hi,
                                                        depth);
        } else {
          // (the builds without matrix-core counts, which run raw-counted
          // windows at four or six workgroups per CU, load the next row
          // while counting the current one)
          raw_wave<T, D3, !MF>(W, act && slot < 0, lo, depth, scr, src, a, x0 + wv * 64, y, z,
                               lane);
        }
      } else
      for (uint64_t fb = nos; fb;) {
        const int leader = __builtin_ctzll(fb);
        const int klo = readlane(lo, leader), khi = readlane(hi, leader);
        const int kdep = readlane(depth, leader), knode = readlane(node, leader);
        const uint64_t m = ballot(act && slot < 0 && lo == klo && depth == kdep) & fb;
        fb &= ~m;
        // (builds without the matrix cores keep to few registers: they run
        // many workgroups per CU; adaptive volumes walk the topology per
        // value, where batched loads measured slower)
        scratch_build<T, ADAPT, D3, (MF && !(ADAPT && D3) ? kRebRows : 1)>(
            scr, src, a, ts, topo, x0 + wv * 64, y, z, lane, span, knode, klo, khi, kdep);
        wave_sync_lds();
        if ((m >> lane) & 1) direct_counts(W, scr - (size_t)wv * 64 * 16, 0, 0, lx, span, batch);
        wave_sync_lds();
      }
      // Descend (up to) the four levels of this tier.
      if (!ADAPT && act) {
        // uniform tree: every level halves the interval, so the levels taken
        // right spell the next value bits; the lane's levels in this tier end
        // at the stop depth
        const int lv = stop - depth < kTierLevels ? stop - depth : kTierLevels;
        int p = 1;
#pragma unroll
        for (int k = 0; k < kTierLevels; ++k) {
          if (k < lv) {
            const uint32_t wl = k == 0 ? (W[0] & 0xffffu)
                                        : wsel(W[0], W[1], W[2], W[3], W[4], W[5], W[6], W[7], p - 1);
            const bool right = acc + wl <= K;
            acc += right ? wl : 0u;
            p = 2 * p + (right ? 1 : 0);
          }
        }
        lo += (p - (1 << lv)) << (bits - depth - lv);
        hi = lo + (1 << (bits - depth - lv)) - 1;
        depth += lv;
        if (depth >= stop) {
          done = true;
          res = lo;
        }
      } else if (act) {
        int p = 1;
#pragma unroll
        for (int k = 0; k < kTierLevels; ++k) {
          if (!done) {
            int split, lch = 0, rch = 0;
            bool lleaf, rleaf;
            if constexpr (ADAPT) {
              const TopoNode t = slot >= 0 ? stopo[slot * 16 + p - 1] : topo[node];
              split = t.split;
              lch = t.left;
              rch = t.right;
              lleaf = lch < 0;
              rleaf = rch < 0;
            } else {
              split = lo + (1 << (bits - 1 - depth));
              lleaf = rleaf = depth + 1 >= bits;
            }
            const uint32_t wl = wsel(W[0], W[1], W[2], W[3], W[4], W[5], W[6], W[7], p - 1);
            const bool left = acc + wl > K;
            bool leaf;
            if (left) {
              hi = split - 1;
              node = lch;
              leaf = lleaf;
            } else {
              acc += wl;
              lo = split;
              node = rch;
              leaf = rleaf;
            }
            ++depth;
            p = 2 * p + (left ? 0 : 1);
            if (leaf || depth >= stop) {
              done = true;
              res = lo;
            }
          }
        }
      }
      // Uniform trees: after the tier that reaches the stop depth every pixel
      // is done, in every wave, so no transition (and no barrier) follows.
      if (!ADAPT && pl + kTierLevels * (round + 1) >= stop) break;
      // Tier transition: pixels entering a deeper subtree look up its slot;
      // subtrees no slot holds are queued as misses for thread 0.
      const bool exited = !done;
      if (raw_only) {  // deeper tiers are all counted raw: no shared state, no barrier
        if (exited) slot = -1;
        if (ballot(exited) == 0) break;
        continue;
      }
      if constexpr (WPS) {
        // Wave-private slots: per subtree the exited lanes enter (lanes
        // grouped by interval start and depth), the wave finds it among its
        // own slots or builds it into the least recently used slot no lane
        // used in this row - when a group of kSlotLanes lanes shares it, or
        // the wave wants at most kMissGroups subtrees; other lanes are counted
        // wave-locally in the next round.
        const uint64_t ex = ballot(exited);
        if (ex == 0) break;
        int ng = 0;
        for (uint64_t u = ex; u && ng <= kMissGroups; ++ng) {
          const int l = __builtin_ctzll(u);
          u &= ~ballot(lo == readlane(lo, l) && depth == readlane(depth, l));
        }
        const int min_lanes = ng <= kMissGroups ? 1 : kSlotLanes;
        int newslot = -1;
        for (uint64_t u = ex; u;) {
          const int l = __builtin_ctzll(u);
          const int klo = readlane(lo, l), kdep = readlane(depth, l);
          const uint64_t m = ballot(exited && lo == klo && depth == kdep) & u;
          u &= ~m;
          // lane s holds slot s: one ballot finds the subtree among them
          const uint64_t hit = ballot(lane < a.wslots && wdep == kdep && wlo == klo);
          int found = hit ? (int)__builtin_ctzll(hit) : -1, victim = -1;
          if (found < 0 && __builtin_popcountll(m) >= min_lanes) {
            int best = 0x7fffffff;
            for (int s = 0; s < a.wslots; ++s) {
              const int sst = readlane(wst, s);
              if (sst != (int)y && sst < best) {
                best = sst;
                victim = s;
              }
            }
          }
          if (victim >= 0) {
            scratch_build<T, false, false>(wslots + (size_t)victim * wpitch16 +
                                               (size_t)wv * 64 * 16,
                                           src, a, ts, topo, x0 + wv * 64, y, z, lane, span, 0,
                                           klo, klo + (1 << (bits - kdep)) - 1, kdep);
            wave_sync_lds();
            if (lane == victim) {
              wlo = klo;
              wdep = kdep;
            }
            found = victim;
          }
          if (found >= 0) {
            if (lane == found) wst = (int)y;
            if ((m >> lane) & 1) newslot = found;
          }
        }
        if (exited) slot = newslot;  // -1: counted wave-locally
        continue;
      }
      const int key = exited ? (ADAPT ? node
                                      : ukey(depth - pl, (lo >> (bits - depth)) &
                                                             ((1 << (depth - pl)) - 1)))
                              : 0;
      const int b = gr % 3;
      if (tid == 0) ts->miss_n[(gr + 1) % 3] = 0;
      const uint64_t ex = ballot(exited);
      if (lane == 0) ts->flag[b][wv] = ex != 0;
      // every exited lane looks its subtree up itself
      int newslot = -1;
      if (exited) {
        newslot = ADAPT ? ht_find(ts->ht, key) : (ts->smap[key] == kNone ? -1 : (int)ts->smap[key]);
        if (newslot >= 0) ts->stamp[newslot] = (int)y;  // the same value from every lane using it
      }
      // subtrees nobody holds are offered slots, at most kMissGroups per wave;
      // when the wave wants more different subtrees than that (medians that
      // change fast along the row), only those a group of lanes shares - the
      // others would churn the slots - and the lanes left over are counted by
      // the wave itself
      uint64_t t = ballot(exited && newslot < 0);
      int gm = 0;
      for (uint64_t u = t; u && gm <= kMissGroups; ++gm)
        u &= ~ballot(key == readlane(key, __builtin_ctzll(u)));
      const int min_lanes = gm <= kMissGroups ? 1 : kSlotLanes;
      for (int g = 0; t && g < kMissGroups; ++g) {
        const int leader = __builtin_ctzll(t);
        const int k = readlane(key, leader);
        const uint64_t m = ballot(key == k) & t;
        t &= ~m;
        if (__builtin_popcountll(m) >= min_lanes) {
          if (lane == leader) {
            const int i = atomicAdd(&ts->miss_n[b], 1);
            if (i < kMissCap) {
              ts->miss[i][0] = k;
              ts->miss[i][1] = lo;
              ts->miss[i][2] = hi;
              ts->miss[i][3] = depth;
            }
          }
          if ((m >> lane) & 1) newslot = -2;
        }
      }
      __syncthreads();
      bool any = false;
      for (int w2 = 0; w2 < kWaves; ++w2) any |= ts->flag[b][w2] != 0;
      const int nmiss = ts->miss_n[b] < kMissCap ? ts->miss_n[b] : kMissCap;
      ++gr;
      if (!any) break;
      if (nmiss > 0) {
        if (tid == 0) assign_slots<ADAPT>(ts, nmiss, (int)y, a.nslots, stopo, topo, root);
        __syncthreads();
        const int nreb = ts->reb_n;
        if (nreb > 0) {
          // Rebuild the new slots from the window's raw values (each thread
          // owns columns tid and tid + 256: no atomics, no barrier between
          // clear and fill).  The rows of both columns are loaded kRebRows at
          // a time before any is used, so their latencies overlap.
          // Two forms, each where it measured faster: 16-bit builds with
          // matrix cores step the row offsets (RowWalk) and load second
          // columns wave by wave; the others clamp each row's offset and load
          // second columns under the lanes' own mask.
          if constexpr (sizeof(T) == 2 && MF) {
            const bool two = tid + kBlock < ncols;
            const T* col0 = src + clampi(x0 - r - 1 + tid, a.w - 1);
            const T* col1 = src + clampi(x0 - r - 1 + tid + kBlock, a.w - 1);
            // a wave that holds any second column loads it on every lane (the
            // column is clamped into the image, so the address is valid)
            const bool wave_two = __builtin_amdgcn_readfirstlane((tid & ~63) + kBlock < ncols);
            for (int i = 0; i < nreb; ++i) {
              const int rs = ts->reb[i][0], rlo = ts->reb[i][2];
              const int rdep = ts->reb[i][3];
              const int rhi = ts->hi[rs];
              const uint4 lim = level_mask(stop - rdep < kTierLevels ? stop - rdep : kTierLevels);
              auto tmask = [&](int v) -> uint4 {
                if constexpr (ADAPT) {
                  int nx;
                  return smask(stopo + rs * 16, rdep, stop, v, &nx);
                } else {
                  return and4(ts->lut[nib(v, rdep, bits)], lim);
                }
              };
              // the (2zr + 1) x span window rows of the columns, slice-major,
              // kRebRows at a time; ALL: second columns loaded on every lane
              auto fill = [&](auto all_tag) {
                constexpr bool ALL = decltype(all_tag)::value;
                uint4 c0 = make_uint4(0u, 0u, 0u, 0u), c1 = c0;
                const int nrows = (2 * zr + 1) * span;
                RowWalk<D3> rw(y, z, a.h, a.d, a.srs, a.sss, r, zr);
                for (int q0 = 0; q0 < nrows; q0 += kRebRows) {
                  int v0[kRebRows], v1[kRebRows];
#pragma unroll
                  for (int k = 0; k < kRebRows; ++k) {
                    // rows past the window (slice zr + 1 onwards) are clamped
                    // into the volume, loaded and skipped
                    v0[k] = col0[rw.off];
                    v1[k] = ALL ? (int)col1[rw.off] : -1;
                    rw.next();
                  }
#pragma unroll
                  for (int k = 0; k < kRebRows; ++k) {
                    if (ALL && !two) v1[k] = -1;
                    if (q0 + k < nrows) {
                      if (v0[k] >= rlo && v0[k] <= rhi) c0 = add4(c0, tmask(v0[k]));
                      if (ALL && v1[k] >= rlo && v1[k] <= rhi) c1 = add4(c1, tmask(v1[k]));
                    }
                  }
                }
                vec(slots, cp16, rs, tid) = c0;
                if (two) vec(slots, cp16, rs, tid + kBlock) = c1;
              };
              if (wave_two)
                fill(std::true_type{});
              else
                fill(std::false_type{});
            }
          } else {
            const bool two = tid + kBlock < ncols;
            const int64_t cx0 = clampi(x0 - r - 1 + tid, a.w - 1);
            const int64_t cx1 = clampi(x0 - r - 1 + tid + kBlock, a.w - 1);
            for (int i = 0; i < nreb; ++i) {
              const int rs = ts->reb[i][0], rlo = ts->reb[i][2];
              const int rdep = ts->reb[i][3];
              const int rhi = ts->hi[rs];
              const uint4 lim = level_mask(stop - rdep < kTierLevels ? stop - rdep : kTierLevels);
              auto tmask = [&](int v) -> uint4 {
                if constexpr (ADAPT) {
                  int nx;
                  return smask(stopo + rs * 16, rdep, stop, v, &nx);
                } else {
                  return and4(ts->lut[nib(v, rdep, bits)], lim);
                }
              };
              uint4 c0 = make_uint4(0u, 0u, 0u, 0u), c1 = c0;
              // the (2zr + 1) x span window rows of the columns, slice-major;
              // (dz, j) walks them kRebRows at a time
              const int nrows = (2 * zr + 1) * span;
              int dz = -zr, j = -r;
              for (int q0 = 0; q0 < nrows; q0 += kRebRows) {
                int v0[kRebRows], v1[kRebRows];
#pragma unroll
                for (int k = 0; k < kRebRows; ++k) {
                  // rows past the window (slice zr + 1 onwards) are clamped into
                  // the volume, loaded and skipped
                  const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
                  const int64_t off = zz * a.sss + clampi(y + j, a.h - 1) * a.srs;
                  v0[k] = src[off + cx0];
                  v1[k] = two ? (int)src[off + cx1] : -1;
                  if (++j > r) {
                    j = -r;
                    ++dz;
                  }
                }
#pragma unroll
                for (int k = 0; k < kRebRows; ++k) {
                  if (q0 + k < nrows) {
                    if (v0[k] >= rlo && v0[k] <= rhi) c0 = add4(c0, tmask(v0[k]));
                    if (v1[k] >= rlo && v1[k] <= rhi) c1 = add4(c1, tmask(v1[k]));
                  }
                }
              }
              vec(slots, cp16, rs, tid) = c0;
              if (two) vec(slots, cp16, rs, tid + kBlock) = c1;
            }
          }
          __syncthreads();
        }
        if (exited && newslot == -2)
          newslot = ADAPT ? ht_find(ts->ht, key) : (ts->smap[key] == kNone ? -1 : ts->smap[key]);
      }
      if (exited) slot = newslot;  // -1: no slot, count directly
    }
    if (x < a.w) dst[z * a.dss + y * a.drs + x] = (T)res;
    __syncthreads();

    // ---- next window: every column drops row y-r and takes row y+r+1
    if (y + 1 < ye) {
      const int64_t yo = clampi(y - r, a.h - 1), yi = clampi(y + r + 1, a.h - 1);
      // one column of the uniform tree: value vo leaves, vi enters; a subtree
      // holding both is updated once, removal first (no byte ever exceeds the
      // column's value count)
      auto pair_update = [&](int lc, int so, int si, uint4 mo, uint4 mi) {
        if (so == si) {
          if (so != (int)kNone) {
            uint4& cv = vec(slots, cp16, so, lc);
            cv = add4(sub4(cv, mo), mi);
          }
        } else {
          if (so != (int)kNone) {
            uint4& cv = vec(slots, cp16, so, lc);
            cv = sub4(cv, mo);
          }
          if (si != (int)kNone) {
            uint4& cv = vec(slots, cp16, si, lc);
            cv = add4(cv, mi);
          }
        }
      };
      if (!ADAPT && D3 && yo != yi) {
        // uniform 3-D: per column and slice, the leaving and entering values
        for (int lc = tid; lc < ncols; lc += kBlock) {
          const int64_t cx = clampi(x0 - r - 1 + lc, a.w - 1);
          for (int dz = -zr; dz <= zr; ++dz) {
            const int64_t zz = clampi(z + dz, a.d - 1);
            const int vo = src[zz * a.sss + yo * a.srs + cx];
            const int vi = src[zz * a.sss + yi * a.srs + cx];
#pragma unroll
            for (int t = 0; t < ntiers; ++t) {
              const int rel = t * kTierLevels, dep = pl + rel;
              if (dep >= stop) break;
              const uint4 lim = level_mask(stop - dep < kTierLevels ? stop - dep : kTierLevels);
              int so = 0, si = 0;
              if (t > 0) {
                const int mk = (1 << rel) - 1;
                so = ts->smap[ukey(rel, (vo >> (bits - dep)) & mk)];
                si = ts->smap[ukey(rel, (vi >> (bits - dep)) & mk)];
              }
              pair_update(lc, so, si, and4(ts->lut[nib(vo, dep, bits)], lim),
                          and4(ts->lut[nib(vi, dep, bits)], lim));
            }
          }
        }
      } else if (WPS && yo != yi) {
        // wave-private slots: tier 1 in slot 0 for columns tid and tid + 256;
        // then each wave brings its own slots up to date for its columns
        // 64 wv + j, j = lane, lane + 64, ... up to 64 + 2r
        const uint4 lim1 = level_mask(stop - pl < kTierLevels ? stop - pl : kTierLevels);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int lc = tid + k * kBlock;
          if (lc < ncols && pl < stop)
            pair_update(lc, 0, 0, and4(ts->lut[nib(pre_o[k], pl, bits)], lim1),
                        and4(ts->lut[nib(pre_i[k], pl, bits)], lim1));
        }
        const uint64_t held = ballot(lane < a.wslots && wdep >= 0);
        for (int k = 0; tid + 64 * k <= wcmax; ++k) {
          const int lc = tid + 64 * k;  // tile column 64 wv + lane + 64 k
          int vo = pre_o[0], vi = pre_i[0];
          if (k > 0) {
            const int64_t cx = clampi(x0 - r - 1 + lc, a.w - 1);
            vo = src[z * a.sss + yo * a.srs + cx];
            vi = src[z * a.sss + yi * a.srs + cx];
          }
          for (uint64_t hs = held; hs; hs &= hs - 1) {
            const int s = __builtin_ctzll(hs);
            const int sdep = readlane(wdep, s);
            const int slo = readlane(wlo, s), shi = slo + (1 << (bits - sdep)) - 1;
            const bool io = vo >= slo && vo <= shi, ii = vi >= slo && vi <= shi;
            if (io || ii) {
              const uint4 lim = level_mask(stop - sdep < kTierLevels ? stop - sdep : kTierLevels);
              uint4& cv = *(uint4*)(wslots + (size_t)s * wpitch16 + (size_t)lc * 16);
              uint4 c = cv;
              if (io) c = sub4(c, and4(ts->lut[nib(vo, sdep, bits)], lim));
              if (ii) c = add4(c, and4(ts->lut[nib(vi, sdep, bits)], lim));
              cv = c;
            }
          }
        }
      } else if (!ADAPT && !D3 && yo != yi) {
        // uniform 2-D: the thread owns columns tid and tid + 256 (if any); per
        // tier the slots and masks of both columns' leaving and entering values
        // are looked up together
        const bool two = tid + kBlock < ncols;
#pragma unroll
        for (int t = 0; t < ntiers; ++t) {
          const int rel = t * kTierLevels, dep = pl + rel;
          if (dep >= stop) break;
          const uint4 lim = level_mask(stop - dep < kTierLevels ? stop - dep : kTierLevels);
          const int mk = (1 << rel) - 1;
          int so[2] = {0, 0}, si[2] = {0, 0};
          uint4 mo[2], mi[2];
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            if (t > 0) {
              so[k] = ts->smap[ukey(rel, (pre_o[k] >> (bits - dep)) & mk)];
              si[k] = ts->smap[ukey(rel, (pre_i[k] >> (bits - dep)) & mk)];
            }
            mo[k] = and4(ts->lut[nib(pre_o[k], dep, bits)], lim);
            mi[k] = and4(ts->lut[nib(pre_i[k], dep, bits)], lim);
          }
          pair_update(tid, so[0], si[0], mo[0], mi[0]);
          if (two) pair_update(tid + kBlock, so[1], si[1], mo[1], mi[1]);
        }
      } else if (yo != yi) {
        for (int lc = tid; lc < ncols; lc += kBlock) {
          const int64_t cx = clampi(x0 - r - 1 + lc, a.w - 1);
          for (int pass = 0; pass < 2; ++pass) {  // removals first, then insertions
            const int64_t yy = pass == 0 ? yo : yi;
            for (int dz = -zr; dz <= zr; ++dz) {
              const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
              const int v = D3 ? (int)src[zz * a.sss + yy * a.srs + cx]
                               : (pass == 0 ? pre_o[lc >= kBlock] : pre_i[lc >= kBlock]);
              if constexpr (ADAPT) {
                // walk down the tiers while their subtrees are held (each held
                // subtree's topology is in LDS)
                int nd = root, s = 0, dep = 0;
                for (int t = 0; t <= (3 * bits) / kTierLevels && nd >= 0 && dep < stop; ++t) {
                  if (t > 0) {
                    s = ht_find(ts->ht, nd);
                    if (s < 0) break;
                  }
                  uint4& cv = vec(slots, cp16, s, lc);
                  const uint4 m = smask(stopo + s * 16, dep, stop, v, &nd);
                  cv = pass == 0 ? sub4(cv, m) : add4(cv, m);
                  dep += kTierLevels;
                }
              } else {
                for (int t = 0; t < ntiers; ++t) {
                  const int rel = t * kTierLevels, dep = pl + rel;
                  if (dep >= stop) break;
                  int s = 0;
                  if (t > 0) {
                    s = ts->smap[ukey(rel, (v >> (bits - dep)) & ((1 << rel) - 1))];
                    if (s == (int)kNone) continue;
                  }
                  const uint4 m = and4(ts->lut[nib(v, dep, bits)],
                                       level_mask(stop - dep < kTierLevels ? stop - dep
                                                                           : kTierLevels));
                  uint4& cv = vec(slots, cp16, s, lc);
                  cv = pass == 0 ? sub4(cv, m) : add4(cv, m);
                }
              }
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

// WPE = 3 asks for three waves per SIMD (at most 168 registers per lane), so
// that three workgroups with budgets of kLdsThird bytes share a CU; WPE = 4
// and 6 (at most 128 / 85 registers, no matrix-core counts) let four or six
// workgroups of kLdsQuarter / kLdsSixth bytes share one; WPE = 1 leaves the
// register allocation free (workgroups with larger budgets run at most two
// per CU anyway).
template <typename T, bool ADAPT, bool D3, int WPE, bool WPS = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void k_median_tiered(
    MedianArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (a.need) {  // recompute only flagged tiles, and clear the flag once read
    if (a.need[bid] == 0u) return;
    __syncthreads();
    if (threadIdx.x == 0) a.need[bid] = 0u;
  }
  const int rest = bid / a.strips;
  tile_body<T, ADAPT, D3, (WPE <= 3), WPS>(a, lds, bid % a.strips, rest % a.segs, rest / a.segs);
}

// Persistent batched launch: every workgroup repeatedly takes the next tile
// index from a device counter and runs the tile body for whichever image the
// tile belongs to (plain 2-D median, 8- or 16-bit).  Tiles of one image are
// contiguous in the index space, images in descriptor order.  The index space
// is cut into 8 contiguous chunks with a counter each; workgroups start on the
// chunk of their XCD (workgroups are dealt to XCDs round-robin) so that tiles
// sharing halo rows stay in one XCD's L2, and move on to the other chunks when
// theirs is exhausted.  LIGHT = true builds the kernel without the
// matrix-core counts, for four workgroups per CU (images whose tiles count no
// subtree wave-wide); LIGHT = false serves every image with two per CU.
template <bool LIGHT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LIGHT ? 4 : 1))) void
k_median_batched(const BatchImage* __restrict__ imgs, const int32_t* __restrict__ hdr,
                 uint32_t* __restrict__ counter) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ int s_tile;
  const int n = hdr[0];
  const int64_t total = n > 0 ? imgs[n - 1].tile_end : 0;
  const int64_t per = (total + 7) / 8;
  const int home = blockIdx.x & 7;
  for (int c = 0; c < 8; ++c) {
    const int chunk = (home + c) & 7;
    const int64_t c0 = chunk * per, c1 = c0 + per < total ? c0 + per : total;
    for (;;) {
      if (threadIdx.x == 0) s_tile = (int)atomicAdd(&counter[chunk], 1u);
      __syncthreads();
      // uniform by construction; readfirstlane lets the compiler keep the tile
      // index, the image search and the image's arguments in scalar registers
      const int64_t t = c0 + __builtin_amdgcn_readfirstlane(s_tile);
      __syncthreads();  // every thread has read s_tile before thread 0 overwrites it
      if (t >= c1) break;
      int lo = 0, hi = n - 1;  // first image whose tile range ends after t
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (imgs[mid].tile_end > t)
          hi = mid;
        else
          lo = mid + 1;
      }
      // the image's arguments into registers once (the tile body reads them in
      // its inner loops)
      const MedianArgs args = imgs[lo].args;
      const int bytes = imgs[lo].bytes;
      const int64_t local = t - (imgs[lo].tile_end - (int64_t)args.strips * args.segs);
      const int strip = (int)(local % args.strips), seg = (int)(local / args.strips);
      if (bytes == 1)
        tile_body<uint8_t, false, false, !LIGHT>(args, lds, strip, seg, 0);
      else
        tile_body<uint16_t, false, false, !LIGHT>(args, lds, strip, seg, 0);
      __syncthreads();  // LDS is reused by the next tile
    }
  }
}

__global__ void k_zero_counter(uint32_t* counter) {
  if (threadIdx.x < 8 && blockIdx.x == 0) counter[threadIdx.x] = 0;
}

template <typename T, bool ADAPT, bool D3>
hipError_t launch_t(const MedianArgs& a, size_t lds, hipStream_t stream) {
  auto kern = k_median_tiered<T, ADAPT, D3, 1>;
  if constexpr (!ADAPT && !D3) {
    if (a.wslots > 0) {
      kern = lds <= (size_t)kLdsThird ? k_median_tiered<T, false, false, 3, true>
                                      : k_median_tiered<T, false, false, 1, true>;
      hipError_t e = ensure_dynamic_lds((const void*)kern, lds);
      if (e != hipSuccess) return e;
      const int64_t grid = (int64_t)a.strips * a.segs * a.d;
      hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(kBlock), lds, stream, a);
      return hipGetLastError();
    }
  }
  // the register cap that lets the LDS budget's workgroups share a CU (both
  // trees: adaptive 16-bit volumes at r = 1 26.9 -> 14.4 ms with the uniform
  // tree's tiles, 8-bit 8192^2 r = 64 7.8 -> 6.6 ms)
  if (lds <= (size_t)kLdsSixth && a.max_groups == 0)
    kern = k_median_tiered<T, ADAPT, D3, 6>;
  else if (lds <= (size_t)kLdsQuarter && a.max_groups == 0)
    kern = k_median_tiered<T, ADAPT, D3, 4>;
  else if (lds <= (size_t)kLdsThird)
    kern = k_median_tiered<T, ADAPT, D3, 3>;
  hipError_t e = ensure_dynamic_lds((const void*)kern, lds);
  if (e != hipSuccess) return e;
  const int64_t grid = (int64_t)a.strips * a.segs * a.d;
  hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(kBlock), lds, stream, a);
  return hipGetLastError();
}

size_t align16_host(size_t b) { return (b + 15) & ~(size_t)15; }

// Raise the LDS limit of every build of the tiered kernel for one element type.
template <typename T>
hipError_t prime_type() {
  const void* ks[] = {
      (const void*)k_median_tiered<T, false, false, 1>, (const void*)k_median_tiered<T, false, false, 3>,
      (const void*)k_median_tiered<T, false, false, 4>, (const void*)k_median_tiered<T, false, false, 6>,
      (const void*)k_median_tiered<T, false, true, 1>,  (const void*)k_median_tiered<T, false, true, 3>,
      (const void*)k_median_tiered<T, false, true, 4>,  (const void*)k_median_tiered<T, false, true, 6>,
      (const void*)k_median_tiered<T, true, false, 1>,  (const void*)k_median_tiered<T, true, false, 3>,
      (const void*)k_median_tiered<T, true, false, 4>,  (const void*)k_median_tiered<T, true, false, 6>,
      (const void*)k_median_tiered<T, true, true, 1>,   (const void*)k_median_tiered<T, true, true, 3>,
      (const void*)k_median_tiered<T, true, true, 4>,   (const void*)k_median_tiered<T, true, true, 6>,
      (const void*)k_median_tiered<T, false, false, 1, true>,
      (const void*)k_median_tiered<T, false, false, 3, true>};
  for (const void* k : ks) {
    const hipError_t e = ensure_dynamic_lds(k, kLdsLimit);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t prime_tiered_lds() {
  hipError_t e = prime_type<uint8_t>();
  if (e == hipSuccess) e = prime_type<uint16_t>();
  // (the persistent kernel declares a few static bytes of its own)
  if (e == hipSuccess)
    e = ensure_dynamic_lds((const void*)k_median_batched<true>, kLdsLimit - 256);
  if (e == hipSuccess)
    e = ensure_dynamic_lds((const void*)k_median_batched<false>, kLdsLimit - 256);
  return e;
}

hipError_t launch_batched_prepare(size_t lds, bool light) {
  return ensure_dynamic_lds(light ? (const void*)k_median_batched<true>
                                  : (const void*)k_median_batched<false>,
                            lds);
}

hipError_t launch_batched(const BatchImage* d_imgs, const int32_t* d_hdr, uint32_t* d_counter,
                          int grid, size_t lds, bool light, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, d_counter);
  if (light)
    hipLaunchKernelGGL(k_median_batched<true>, dim3(grid), dim3(kBlock), lds, stream, d_imgs,
                       d_hdr, d_counter);
  else
    hipLaunchKernelGGL(k_median_batched<false>, dim3(grid), dim3(kBlock), lds, stream, d_imgs,
                       d_hdr, d_counter);
  return hipGetLastError();
}

size_t tiered_meta_bytes(int r, int bytes) {
  const size_t st = bytes == 1 ? sizeof(TierState<uint8_t>) : sizeof(TierState<uint16_t>);
  return align16_host(st) + (size_t)kWaves * wave_scratch_bytes(r);
}

size_t wps_lds_bytes(int r, int cp, int wslots, int wpitch) {
  return align16_host((size_t)cp * 16) + align16_host(sizeof(TierStateT<16>)) +
         (size_t)kWaves * (wave_scratch_bytes(r) + (size_t)wslots * wpitch * 16);
}

size_t tiered_topo_bytes(int nslots) { return (size_t)nslots * 16 * sizeof(TopoNode); }

hipError_t launch_median_tiered(const MedianArgs& a, int bytes, int dims, bool adaptive,
                                size_t lds, hipStream_t stream) {
  const bool d3 = dims == 3;
  if (bytes == 1) {
    if (adaptive) return d3 ? launch_t<uint8_t, true, true>(a, lds, stream)
                            : launch_t<uint8_t, true, false>(a, lds, stream);
    return d3 ? launch_t<uint8_t, false, true>(a, lds, stream)
              : launch_t<uint8_t, false, false>(a, lds, stream);
  }
  if (adaptive) return d3 ? launch_t<uint16_t, true, true>(a, lds, stream)
                          : launch_t<uint16_t, true, false>(a, lds, stream);
  return d3 ? launch_t<uint16_t, false, true>(a, lds, stream)
            : launch_t<uint16_t, false, false>(a, lds, stream);
}

}  // namespace hrrm
