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
// Storage (LDS): all 255 left-node counters of the 8-bit tree per column, one
// byte each, node-major/column-minor so that 64 lanes reading one node hit 64
// consecutive bytes.  (16-bit trees use the tiered kernel, median_tiered.hip.)
//
// Full-update form (FULL): instead of counting only the nodes the descent
// visits, every node of the window tree is brought to the current window at
// every pixel (Sec. III: the unconditional update of the entire window tree,
// strictly constant work per pixel, 2^d - 1 node updates).  A wave does it as
// one prefix sum per node; each lane keeps the count of the node it is at.
//
// Topology: uniform (each split halves its interval, Sec. III) or adaptive
// (split points from a table, leaf test at every visit, Sec. III-C).
#include "hrrm_internal.h"

#include "wave.hpp"

namespace hrrm {
namespace {

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

// Window count of counter row `row` (wave-uniform) for every lane: count of
// the wave's first window plus the running sum of (entering - leaving column).
// Must be called with all 64 lanes active.
__device__ __forceinline__ uint32_t scan_count(const uint8_t* __restrict__ cnt, int cp, int row,
                                               int lx, int span, int lane, int wbase) {
  const uint8_t* base = cnt + (size_t)row * cp;
  const uint32_t vout = base[lx];        // column of x - r - 1
  const uint32_t vin = base[lx + span];  // column of x + r
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
  return b + (sc >> 16) - (sc & 0xffffu);
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
    const uint32_t wl = scan_count(cnt, cp, grow, lx, span, lane, wbase);
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

// Walk of one value through the column tree of local column lc: count it
// (inc) or uncount it at every left node it passes (Sec. III-B, add_value and
// its removal twin).
template <bool ADAPT>
__device__ __forceinline__ void column_walk(uint8_t* cnt, int cp, const TopoNode* topo, int root,
                                            int bits, int stop, int v, int lc, bool inc) {
  int node = root, lo = 0, depth = 0;
  const int maxdepth = ADAPT ? 3 * bits : bits;  // bound on any tree's height
  for (int it = 0; it < maxdepth; ++it) {
    const Step<ADAPT> s = node_step<ADAPT>(topo, node, lo, depth, bits);
    const bool left = v < s.split;
    if (left) cnt_add(cnt, cp, ADAPT ? node : node - 1, lc, inc);
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
  }
}

template <typename T, bool ADAPT, bool D3, bool FULL>
__global__ __launch_bounds__(kBlock) void k_median_dense(MedianArgs a) {
  static_assert(!(FULL && ADAPT), "the full update walks the uniform tree");
  extern __shared__ __align__(16) uint8_t lds[];
  const T* __restrict__ src = (const T*)a.src;
  T* __restrict__ dst = (T*)a.dst;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = a.r, cp = a.cp, ncols = a.ncols, bits = a.bits, stop = a.stop;
  const int span = 2 * r + 1;
  const int zr = D3 ? r : 0;

  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int strip = bid % a.strips;
  const int rest = bid / a.strips;
  const int seg = rest % a.segs;
  const int64_t z = rest / a.segs;
  const int64_t x0 = (int64_t)strip * kBlock;
  const int64_t yb = (int64_t)seg * a.seg_rows;
  const int64_t ye = yb + a.seg_rows < a.h ? yb + a.seg_rows : a.h;

  uint8_t* cnt = lds;
  const size_t cnt_bytes = align16((size_t)kDenseNodes * cp);
  const TopoNode* topo = a.topo;
  if constexpr (ADAPT) {
    TopoNode* tl = (TopoNode*)(lds + cnt_bytes);
    for (int i = tid; i <= kDenseNodes; i += kBlock) tl[i] = a.topo[i];
    topo = tl;
  }
  for (int i = tid; i < kDenseNodes * cp / 4; i += kBlock) ((uint32_t*)cnt)[i] = 0;
  __syncthreads();
  // adaptive: the entry after the last node holds the root's index
  const int root = ADAPT ? topo[(1 << bits) - 1].split : 1;

  // Column trees of the first window of the segment.
  for (int lc = tid; lc < ncols; lc += kBlock) {
    const int64_t cx = clampi(x0 - r - 1 + lc, a.w - 1);
    for (int dz = -zr; dz <= zr; ++dz) {
      const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
      for (int j = -r; j <= r; ++j) {
        const int v = src[zz * a.sss + clampi(yb + j, a.h - 1) * a.srs + cx];
        column_walk<ADAPT>(cnt, cp, topo, root, bits, stop, v, lc, true);
      }
    }
  }
  __syncthreads();

  const int lx = wv * 64 + lane;  // output x = x0 + lx; window columns lx+1 .. lx+span
  const int64_t x = x0 + lx;
  const uint32_t K = (uint32_t)a.rank;
  const int maxdepth = ADAPT ? 3 * bits : bits;  // bound on any tree's height

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
    int node = root, lo = 0, depth = 0;
    uint32_t acc = 0;
    bool done = (x >= a.w) || (stop == 0);
    int res = 0;
    if constexpr (FULL) {
      // level k holds the nodes with heap indices 2^k .. 2^(k+1)-1; all of them
      // are brought to this pixel's window, the lane keeps its own node's count
      for (int k = 0; k < stop; ++k) {
        uint32_t wl = 0;
        for (int q = 1 << k; q < (2 << k); ++q) {
          const uint32_t w = scan_count(cnt, cp, q - 1, lx, span, lane, wv * 64);
          wl = node == q ? w : wl;
        }
        if (!done) {
          if (acc + wl > K) {
            node = 2 * node;
          } else {
            acc += wl;
            lo += 1 << (bits - 1 - k);
            node = 2 * node + 1;
          }
          if (k + 1 >= stop) {
            done = true;
            res = lo;
          }
        }
      }
    }
    for (int k = 0; k < (FULL ? 0 : maxdepth); ++k) {
      const bool act = !done;
      if (ballot(act) == 0) break;
      const Step<ADAPT> s = node_step<ADAPT>(topo, node, lo, depth, bits);
      const uint32_t wl = window_count(cnt, cp, ADAPT ? node : node - 1, act, lx, span, lane,
                                       wv * 64, a.min_group, a.max_groups);
      if (act) {
        const bool left = acc + wl > K;
        bool leaf;
        if (left) {
          node = s.lch;
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
            const int v = D3 ? (int)src[zz * a.sss + yo * a.srs + cx] : pre_o[lc >= kBlock];
            column_walk<ADAPT>(cnt, cp, topo, root, bits, stop, v, lc, false);
          }
          for (int dz = -zr; dz <= zr; ++dz) {
            const int64_t zz = D3 ? clampi(z + dz, a.d - 1) : z;
            const int v = D3 ? (int)src[zz * a.sss + yi * a.srs + cx] : pre_i[lc >= kBlock];
            column_walk<ADAPT>(cnt, cp, topo, root, bits, stop, v, lc, true);
          }
        }
      }
      __syncthreads();
    }
  }
}

template <bool ADAPT, bool D3, bool FULL>
hipError_t launch_dense(const MedianArgs& a, size_t lds, hipStream_t stream) {
  auto kern = k_median_dense<uint8_t, ADAPT, D3, FULL>;
  hipError_t e = ensure_dynamic_lds((const void*)kern, lds);
  if (e != hipSuccess) return e;
  const int64_t grid = (int64_t)a.strips * a.segs * a.d;
  hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(kBlock), lds, stream, a);
  return hipGetLastError();
}

}  // namespace

hipError_t prime_dense_lds() {
  const void* ks[] = {(const void*)k_median_dense<uint8_t, false, false, false>,
                      (const void*)k_median_dense<uint8_t, true, false, false>,
                      (const void*)k_median_dense<uint8_t, false, true, false>,
                      (const void*)k_median_dense<uint8_t, true, true, false>,
                      (const void*)k_median_dense<uint8_t, false, false, true>,
                      (const void*)k_median_dense<uint8_t, false, true, true>};
  for (const void* k : ks) {
    const hipError_t e = ensure_dynamic_lds(k, kLdsLimit);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_median_tiered(const MedianArgs& a, int bytes, int dims, bool adaptive,
                                size_t lds, hipStream_t stream);

size_t median_lds_bytes(int bytes, bool adaptive, bool tiered, int ncols, int cp, int nslots) {
  // ncols = 256 + 2r + 1
  if (tiered)
    return (((size_t)nslots * cp * 16 + 15) & ~(size_t)15) + tiered_meta_bytes((ncols - 257) / 2, bytes) +
           (adaptive ? tiered_topo_bytes(nslots) : 0);
  size_t b = ((size_t)kDenseNodes * cp + 15) & ~(size_t)15;
  if (adaptive) b += sizeof(TopoNode) * (kDenseNodes + 1);
  return b;
}

hipError_t launch_median(const MedianArgs& a, int bytes, int dims, bool adaptive, bool tiered,
                         bool full, hipStream_t stream) {
  const size_t lds = a.wslots > 0 ? wps_lds_bytes(a.r, a.cp, a.wslots, a.wpitch)
                                  : median_lds_bytes(bytes, adaptive, tiered, a.ncols, a.cp,
                                                     a.nslots);
  if (tiered) return launch_median_tiered(a, bytes, dims, adaptive, lds, stream);
  if (bytes != 1) return hipErrorInvalidValue;  // dense storage holds 8-bit trees only
  if (full) {
    if (adaptive) return hipErrorInvalidValue;
    return dims == 3 ? launch_dense<false, true, true>(a, lds, stream)
                     : launch_dense<false, false, true>(a, lds, stream);
  }
  if (adaptive) return dims == 3 ? launch_dense<true, true, false>(a, lds, stream)
                                 : launch_dense<true, false, false>(a, lds, stream);
  return dims == 3 ? launch_dense<false, true, false>(a, lds, stream)
                   : launch_dense<false, false, false>(a, lds, stream);
}

}  // namespace hrrm
