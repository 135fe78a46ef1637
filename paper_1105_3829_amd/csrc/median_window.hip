// Grey-level-window running-median kernel for gfx950: 2-D images, 8- and
// 16-bit data, any rank K.
//
// Method: Alekseychuk, "Hierarchical Recursive Running Median" (Sec. III).
// Column histograms are updated recursively as the window moves down one row
// (one removal, one insertion per column), the window histogram of a pixel is
// built from column histograms by the elementary update W(x) = W(x-1) +
// col(x+r) - col(x-r-1), and the order statistic is found by descending the
// tree of interval counts: go left when accumulator + left count > K, else
// add the left count and go right (get_order_statistic).
//
// Level skipping.  The medians of neighbouring pixels lie close together
// (their windows share all but two columns), so the descents of a wave's 64
// pixels share their top levels.  A wave keeps, per column of its strip,
// only the leaves of one window of 128 consecutive grey levels [bc, bc+128)
// as byte counters, plus the number of column values below and above the
// range of leaves it scans (`lohi`, two 16-bit fields).  For a pixel whose
// window count below the scanned range (lo) satisfies lo <= K < lo + (count
// inside), every descent step above the scanned range is fixed - the
// accumulator after those steps is exactly lo - so the descent starts at
// the scanned range with accumulator lo and walks its levels, whose node
// counts are sums of leaf counts.  The scanned range is
//   * SQ = 32 (uniform tree): the whole 128 leaves [bc, bc+128), bc a
//     multiple of 64: two neighbouring 6-level subtrees of the uniform tree
//     (the descent reaches one of them after the skipped levels);
//   * SQ = 16 (adaptive tree, Sec. III-C): 64 leaves starting anywhere in the
//     range on a 16-level step, placed where the previous rows' medians lie
//     (the estimate of the median distribution that shapes the topology):
//     two short paths to "below" and "above", six levels inside.
// The range moves with the medians: shifted (SQ = 16) or rebuilt from the
// raw window (both) when the medians approach its edge, and rebuilt around
// the exact median of one pixel when a pixel's median falls outside.
//
// Exactness.  Window leaf counts are byte fields summed in 32-bit modular
// arithmetic; the lo/hi fields are exact.  The digit sum of the leaf bytes
// equals the true count inside the range (N - lo - hi) exactly when no leaf
// count exceeded 255, so every result is checked; a strip segment whose
// window counts overflow a byte, or whose medians in one row spread wider
// than the scanned range, stops and flags its rows for the tiered kernel,
// which recomputes them (the tiles it covers are flagged in `need`).
//
// Work split: one wave per strip of 64 output columns x seg_rows rows, with
// its own 64 + 2r columns in LDS (no barriers; the waves of a workgroup are
// independent).  Window counts: every lane reads the bins of the column
// entering and leaving its window, one DPP prefix sum over the wave per
// dword turns the differences into running window counts, anchored at the
// window of the wave's first pixel (`base`, kept up to date by the row steps
// of its 2r + 1 columns).
#include "hrrm_internal.h"
#include "wave.hpp"
#include "window_geom.hpp"

namespace hrrm {
namespace {

// Layout of a column's counters for BQ dwords of byte counters (4 BQ grey
// levels: 128 or 256).
template <int BQ>
struct Layout {
  static constexpr int kBinQ = BQ;       // dwords of byte counters per column
  static constexpr int kPitch = BQ + 4;  // dwords per column (= 4 mod 32: the 128-bit
                                         // reads of 8 consecutive lanes hit distinct banks)
  static constexpr int kLohi = BQ;       // lo/hi counts of a column (and of the base)
  static constexpr int kSink = BQ + 1;   // pad dword taking the zero updates of values
                                         // outside the leaves
  static constexpr int kSpare = BQ + 2;  // pad dwords BQ + 2, BQ + 3 of columns 0..15:
                                         // row16's 16-bit counts
};
constexpr int kMaxPasses = 6;  // passes over one row before it is left to the tiered kernel

// Where a value goes: leaf dword q with byte increment inc (values outside
// the 128 leaves: the pad dword kSink, increment 0), and its lo/hi increment
// relative to the scanned dwords [q0, q0 + sq).
struct Cls {
  int q;
  uint32_t inc, lh;
};

template <int BQ>
__device__ __forceinline__ Cls classify(int v, int bc, int q0, int sq) {
  using Y = Layout<BQ>;
  const int rel = v - bc;
  const bool in = (uint32_t)rel < 4u * Y::kBinQ;
  Cls c;
  c.q = in ? rel >> 2 : Y::kSink;
  c.inc = in ? 1u << ((rel & 3) << 3) : 0u;
  // below the scanned dwords (also below the leaves), or above them
  c.lh = rel < 4 * q0 ? 1u : (rel >= 4 * (q0 + sq) ? 0x10000u : 0u);
  return c;
}

__device__ __forceinline__ void lds_add(uint32_t* p, uint32_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t dsum(uint32_t v, uint32_t acc) {
  return __builtin_amdgcn_sad_u8(v, 0u, acc);  // acc + sum of the four bytes
}

// One wave's LDS: bins[ncols][kPitch] (a column's lo/hi counts in its dword
// kLohi), base[kPitch] (the leaf counts of the window of the wave's first
// pixel; base[kLohi] its lo/hi), then kPitch dwords that stay zero.  (LDS is
// granted in blocks of 1,280 bytes: at r = 15 these 13,824 bytes take 11
// blocks, so 11 one-wave workgroups share a CU; at r = 7, 11,520 bytes take
// 9: 14 waves.)
struct WaveLds {
  uint32_t* bins;
  uint32_t* base;
};

__host__ __device__ constexpr size_t window_base_offset(int ncols, int bq) {
  return (size_t)ncols * (bq + 4) * 4;
}

// The lo/hi word of column c.
template <int BQ>
__device__ __forceinline__ uint32_t* lohi_of(const WaveLds& L, int c) {
  return L.bins + c * (BQ + 4) + BQ;
}

template <int N>
using vu = uint32_t __attribute__((ext_vector_type(N)));

// x as a value the compiler cannot see through (emits nothing).
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm("" : "+v"(x));
  return x;
}

// v[i] among M = 2^k values, i given by its bits from the most significant
// (the first descent decision) down: one two-way select per value and level.
// Both candidates of every select pass through opaque(): a select between two
// elements of one vector (or array) is otherwise turned into a read at a
// computed index, lowered to a compare and a select per element (or, for an
// array in memory, a scratch-memory load).
template <int M>
__device__ __forceinline__ uint32_t pick(vu<M> v, bool msb) {
  static_assert(M == 2, "one bit selects between two values");
  const uint32_t lo = opaque(v[0]), hi = opaque(v[1]);
  return msb ? hi : lo;
}
template <int M, typename... B>
__device__ __forceinline__ uint32_t pick(vu<M> v, bool msb, bool next, B... rest) {
  vu<M / 2> h;
#pragma unroll
  for (int k = 0; k < M / 2; ++k) {
    const uint32_t lo = opaque(v[k]), hi = opaque(v[M / 2 + k]);
    h[k] = msb ? hi : lo;
  }
  return pick<M / 2>(h, next, rest...);
}

// Pairwise sums out[k] = v[2k] + v[2k + 1] (counts of the parent nodes).
template <int M>
__device__ __forceinline__ vu<M / 2> pairs(vu<M> v) {
  vu<M / 2> o;
#pragma unroll
  for (int k = 0; k < M / 2; ++k) o[k] = v[2 * k] + v[2 * k + 1];
  return o;
}

// Even elements out[k] = v[2k]: the left children of the next level's nodes.
template <int M>
__device__ __forceinline__ vu<M / 2> evens(vu<M> v) {
  vu<M / 2> o;
#pragma unroll
  for (int k = 0; k < M / 2; ++k) o[k] = v[2 * k];
  return o;
}

// One step of get_order_statistic: left-child count c; the remaining rank k
// goes right (and drops c) when it reaches c.
__device__ __forceinline__ bool step(uint32_t c, uint32_t& k) {
  const bool rt = k >= c;
  k -= rt ? c : 0u;
  return rt;
}

// Window counts of the scanned range for every lane's pixel: W[k] = leaf
// bytes of dword q0 + k, wl = lo | hi << 16.  Lane x >= 1 contributes the
// difference of the columns entering and leaving its window; lane 0 the base
// (block ncols) minus the zero block (block ncols + 1), so that the prefix sum
// over the wave is the window counts themselves.  All 64 lanes active.
template <int BQ, int SQ>
__device__ __forceinline__ vu<SQ> window_counts(const WaveLds& L, int q0, int lane, int r2,
                                                int ncols, uint32_t& wl) {
  using Y = Layout<BQ>;
  const int ci = lane ? lane + r2 : ncols;      // column x + r
  const int co = lane ? lane - 1 : ncols + 1;   // column x - r - 1
  const uint32_t* pi = L.bins + ci * Y::kPitch + q0;
  const uint32_t* po = L.bins + co * Y::kPitch + q0;
  vu<SQ> W;
#pragma unroll
  for (int k = 0; k < SQ; k += 4) {
    const uint4 a = *(const uint4*)(pi + k);
    const uint4 b = *(const uint4*)(po + k);
    W[k] = wave_scan(a.x - b.x);
    W[k + 1] = wave_scan(a.y - b.y);
    W[k + 2] = wave_scan(a.z - b.z);
    W[k + 3] = wave_scan(a.w - b.w);
  }
  wl = wave_scan(*lohi_of<BQ>(L, ci) - *lohi_of<BQ>(L, co));
  return W;
}

// Descent over the 4*SQ leaves from accumulator lo (kp = K - lo): returns the
// leaf offset of the K-th value; ok = the order statistic lies in the
// scanned range and no leaf count overflowed a byte.
template <int SQ>
__device__ __forceinline__ int descend(vu<SQ> W, int kp, int win, bool& ok) {
  // node counts of the dword-level tree: t0 per dword (4 leaves), t1 per
  // pair of dwords, t2 per four, t3 per eight (32 leaves)
  vu<SQ> t0;
#pragma unroll
  for (int k = 0; k < SQ; ++k) t0[k] = dsum(W[k], 0u);
  const vu<SQ / 2> t1 = pairs<SQ>(t0);
  const vu<SQ / 4> t2 = pairs<SQ / 2>(t1);
  const vu<SQ / 8> t3 = pairs<SQ / 4>(t2);
  uint32_t total = 0;
#pragma unroll
  for (int k = 0; k < SQ / 8; ++k) total += t3[k];
  ok = kp >= 0 && kp < win && (int)total == win;
  uint32_t k = (uint32_t)kp;
  int off;
  if constexpr (SQ == 16) {
    const bool b1 = step(t3[0], k);
    const bool b2 = step(pick<2>(evens<4>(t2), b1), k);
    const bool b3 = step(pick<4>(evens<8>(t1), b1, b2), k);
    const bool b4 = step(pick<8>(evens<16>(t0), b1, b2, b3), k);
    const uint32_t d = pick<16>(W, b1, b2, b3, b4);
    const bool b5 = step((d & 0xffu) + ((d >> 8) & 0xffu), k);
    const bool b6 = step((d >> (b5 ? 16 : 0)) & 0xffu, k);
    off = (b1 ? 32 : 0) + (b2 ? 16 : 0) + (b3 ? 8 : 0) + (b4 ? 4 : 0) + (b5 ? 2 : 0) + (b6 ? 1 : 0);
  } else if constexpr (SQ == 64) {
    const vu<4> t4 = pairs<8>(t3);
    const bool bh = step(t4[0] + t4[1], k);
    const bool b0 = step(pick<2>(evens<4>(t4), bh), k);
    const bool b1 = step(pick<4>(evens<8>(t3), bh, b0), k);
    const bool b2 = step(pick<8>(evens<16>(t2), bh, b0, b1), k);
    const bool b3 = step(pick<16>(evens<32>(t1), bh, b0, b1, b2), k);
    const bool b4 = step(pick<32>(evens<64>(t0), bh, b0, b1, b2, b3), k);
    const uint32_t d = pick<64>(W, bh, b0, b1, b2, b3, b4);
    const bool b5 = step((d & 0xffu) + ((d >> 8) & 0xffu), k);
    const bool b6 = step((d >> (b5 ? 16 : 0)) & 0xffu, k);
    off = (bh ? 128 : 0) + (b0 ? 64 : 0) + (b1 ? 32 : 0) + (b2 ? 16 : 0) + (b3 ? 8 : 0) +
          (b4 ? 4 : 0) + (b5 ? 2 : 0) + (b6 ? 1 : 0);
  } else {
    const bool b0 = step(t3[0] + t3[1], k);
    const bool b1 = step(pick<2>(evens<4>(t3), b0), k);
    const bool b2 = step(pick<4>(evens<8>(t2), b0, b1), k);
    const bool b3 = step(pick<8>(evens<16>(t1), b0, b1, b2), k);
    const bool b4 = step(pick<16>(evens<32>(t0), b0, b1, b2, b3), k);
    const uint32_t d = pick<32>(W, b0, b1, b2, b3, b4);
    const bool b5 = step((d & 0xffu) + ((d >> 8) & 0xffu), k);
    const bool b6 = step((d >> (b5 ? 16 : 0)) & 0xffu, k);
    off = (b0 ? 64 : 0) + (b1 ? 32 : 0) + (b2 ? 16 : 0) + (b3 ? 8 : 0) + (b4 ? 4 : 0) +
          (b5 ? 2 : 0) + (b6 ? 1 : 0);
  }
  return off;
}

// Exact rank-K value of the clamp-to-edge window of pixel (xc, yc), by two
// 256-bin histograms (high byte, then low byte among values with that high
// byte; 8-bit data: one).  hist: 256 dwords of the wave's LDS.
template <typename T, bool D3>
__device__ __forceinline__ int window_rank_exact(const T* __restrict__ src, int64_t srs, int64_t w, int64_t h,
                                 int64_t xc, int64_t yc, int r, int rank, uint32_t* hist,
                                 int lane, int64_t sss, int64_t d, int64_t zc) {
  const int zr = D3 ? r : 0;
  constexpr int kPasses = sizeof(T) == 2 ? 2 : 1;
  constexpr int kB = 32;  // window rows loaded before any is counted
  int k = rank, prefix = 0;
  for (int pass = 0; pass < kPasses; ++pass) {
    *(uint4*)(hist + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
    __builtin_amdgcn_wave_barrier();
    for (int dz = -zr; dz <= zr; ++dz)
    for (int dx0 = -r; dx0 <= r; dx0 += 64) {
      const T* sz = D3 ? src + clampi(zc + dz, d - 1) * sss : src;
      const int dx = dx0 + lane;
      const int64_t col = clampi(xc + dx, w - 1);
      for (int dy0 = -r; dy0 <= r; dy0 += kB) {
        int v[kB];
#pragma unroll
        for (int t = 0; t < kB; ++t) v[t] = (int)sz[clampi(yc + dy0 + t, h - 1) * srs + col];
#pragma unroll
        for (int t = 0; t < kB; ++t) {
          if (dx <= r && dy0 + t <= r) {
            if (kPasses == 1) {
              lds_add(hist + v[t], 1u);
            } else if (pass == 0) {
              lds_add(hist + (v[t] >> 8), 1u);
            } else if ((v[t] >> 8) == prefix) {
              lds_add(hist + (v[t] & 255), 1u);
            }
          }
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    const uint4 hb = *(const uint4*)(hist + 4 * lane);
    const uint32_t s = hb.x + hb.y + hb.z + hb.w;
    const uint32_t inc = wave_scan(s), exc = inc - s;
    const bool mine = exc <= (uint32_t)k && (uint32_t)k < inc;
    int bin = 4 * lane;
    uint32_t below = exc;
    if ((uint32_t)k >= below + hb.x) {
      below += hb.x;
      ++bin;
      if ((uint32_t)k >= below + hb.y) {
        below += hb.y;
        ++bin;
        if ((uint32_t)k >= below + hb.z) {
          below += hb.z;
          ++bin;
        }
      }
    }
    const uint64_t bm = ballot(mine);
    const int L = bm ? (int)__builtin_ctzll(bm) : 0;
    bin = readlane(bin, L);
    k -= readlane((int)below, L);
    prefix = kPasses == 2 && pass == 0 ? bin : (prefix << 8) | bin;
    __builtin_amdgcn_wave_barrier();
  }
  return prefix;
}


// Rebuild every held column's counters, and the base, for the window of row
// y from the raw values: zero, insert the 2r + 1 clamped rows of each column
// (volumes: of each of the 2r + 1 clamped slices around z), then base = sum
// of columns 0..2r.  Values are loaded sixteen rows at a time before any is
// inserted, so their latencies overlap.
template <typename T, int KC, int BQ, bool D3>
__device__ __forceinline__ void rebuild(const T* __restrict__ src, int64_t srs, int h, int r,
                                        const int (&gx)[KC], int ncols, const WaveLds& L,
                                        int wave_dwords, int y, int bc, int q0, int sq,
                                        int lane, int64_t sss, int64_t d, int64_t zc) {
  const int zr = D3 ? r : 0;
  using Y = Layout<BQ>;
  uint4* z = (uint4*)L.bins;
  for (int i = lane; i < wave_dwords / 4; i += 64) z[i] = make_uint4(0u, 0u, 0u, 0u);
  __builtin_amdgcn_wave_barrier();
  constexpr int kBatch = 16;
  uint32_t lohi[KC];  // each lane alone updates its columns' lo/hi: kept in registers
#pragma unroll
  for (int k = 0; k < KC; ++k) lohi[k] = 0u;
  for (int dz = -zr; dz <= zr; ++dz)
  for (int j0 = -r; j0 <= r; j0 += kBatch) {
    const T* sz = D3 ? src + clampi(zc + dz, d - 1) * sss : src;
    const T* rows[kBatch];
#pragma unroll
    for (int t = 0; t < kBatch; ++t) {
      const int yy = y + j0 + t;
      rows[t] = sz + (int64_t)(yy < 0 ? 0 : (yy > h - 1 ? h - 1 : yy)) * srs;
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int c = lane + 64 * k;
      if (c < ncols) {
        int v[kBatch];
#pragma unroll
        for (int t = 0; t < kBatch; ++t) v[t] = (int)rows[t][gx[k]];
#pragma unroll
        for (int t = 0; t < kBatch; ++t) {
          if (j0 + t <= r) {
            const Cls cl = classify<BQ>(v[t], bc, q0, sq);
            lds_add(L.bins + c * Y::kPitch + cl.q, cl.inc);
            lohi[k] += cl.lh;
          }
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KC; ++k)
    if (lane + 64 * k < ncols) *lohi_of<BQ>(L, lane + 64 * k) = lohi[k];
  __builtin_amdgcn_wave_barrier();
  // base dword i (leaf dwords, then lo/hi at kLohi = kBinQ) by lane i % 64
  for (int i = lane; i <= Y::kBinQ; i += 64) {
    uint32_t s = 0;
    if (i < Y::kBinQ) {
#pragma unroll 8
      for (int c = 0; c <= 2 * r; ++c) s += L.bins[c * Y::kPitch + i];
    } else {
#pragma unroll 8
      for (int c = 0; c <= 2 * r; ++c) s += *lohi_of<BQ>(L, c);
    }
    L.base[i] = s;
  }
  __builtin_amdgcn_wave_barrier();
}

// Move the scanned dwords from [q0, q0 + s0) to [q1, q1 + s1) (all multiples
// of 4): every column's lo gains the leaves of [q0, q1) (loses [q1, q0)) and
// its hi loses the leaves of [q0 + s0, q1 + s1) (gains [q1 + s1, q0 + s0));
// column leaf bytes are exact (at most 2r + 1 <= 255 values), so their digit
// sums are the counts.  Then the base's lo/hi is summed again from the
// columns.  All 64 lanes active.
template <int KC, int BQ>
__device__ __forceinline__ void retarget(const WaveLds& L, int ncols, int r2, int q0, int s0,
                                         int q1, int s1, int lane) {
  using Y = Layout<BQ>;
  const int la = q0 < q1 ? q0 : q1, lb = q0 < q1 ? q1 : q0;
  const int e0 = q0 + s0, e1 = q1 + s1;
  const int ha = e0 < e1 ? e0 : e1, hb = e0 < e1 ? e1 : e0;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int c = lane + 64 * k;
    if (c < ncols) {
      const uint32_t* col = L.bins + c * Y::kPitch;
      uint32_t lo = 0, hi = 0;
      for (int q = la; q < lb; q += 4) {
        const uint4 u = *(const uint4*)(col + q);
        lo = dsum(u.w, dsum(u.z, dsum(u.y, dsum(u.x, lo))));
      }
      for (int q = ha; q < hb; q += 4) {
        const uint4 u = *(const uint4*)(col + q);
        hi = dsum(u.w, dsum(u.z, dsum(u.y, dsum(u.x, hi))));
      }
      const uint32_t dlo = q1 > q0 ? lo : 0u - lo;
      const uint32_t dhi = e1 > e0 ? 0u - hi : hi;
      const uint32_t d = dlo + (dhi << 16);
      if (d) lds_add(lohi_of<BQ>(L, c), d);
    }
  }
  __builtin_amdgcn_wave_barrier();
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int c = lane + 64 * k;
    if (c <= r2) s += *lohi_of<BQ>(L, c);
  }
  s = wave_scan(s);
  if (lane == 63) L.base[Y::kLohi] = s;
  __builtin_amdgcn_wave_barrier();
}

// One pass over a row with the current range: every lane's leaf offset and
// whether its check passed; over the live lanes, the lanes whose order
// statistic lies below / above the scanned leaves.
struct RowOut {
  int off, lo;
  bool ok;
  uint64_t low, high;
};

template <int BQ, int SQ>
__device__ __forceinline__ RowOut row_medians(const WaveLds& L, int q0, int lane, int r2,
                                              int ncols, int n, int rank, bool live) {
  uint32_t wl;
  const vu<SQ> W = window_counts<BQ, SQ>(L, q0, lane, r2, ncols, wl);
  const int lo = (int)(wl & 0xffffu), hi = (int)(wl >> 16);
  const int win = n - lo - hi;
  const int kp = rank - lo;
  RowOut o;
  o.lo = lo;
  o.off = descend<SQ>(W, kp, win, o.ok);
  o.low = ballot(live && kp < 0);
  o.high = ballot(live && kp >= win);
  return o;
}

// Exact window counts of the 64 leaves in dwords [qs, qs + 16) with 16-bit
// fields, for rows where a leaf count passed 255 (a value repeated that often
// in one window: clamp-to-edge repeats a corner pixel (r+1)^2 times).
// `below` is each pixel's exact window count below these leaves.  Per lane:
// ok = its order statistic lies in these leaves, off its leaf offset, cnt the
// exact number of window values in these leaves.  The 16-bit counts of the
// wave's first window go to the pad dwords kSpare, kSpare + 1 of columns
// 0..15 (pair q in column q).  All 64 lanes active.
template <int BQ>
__device__ __forceinline__ void row16(const WaveLds& L, int qs, int lane, int r2, int rank,
                                      int below, int& off, bool& ok, int& cnt) {
  using Y = Layout<BQ>;
  // the first window's counts, summed again from its 2r + 1 columns
  if (lane < 32) {
    uint32_t acc = 0;
    const int q = qs + (lane >> 1), sh = (lane & 1) * 8;
    for (int c = 0; c <= r2; ++c) acc += (L.bins[c * Y::kPitch + q] >> sh) & 0x00ff00ffu;
    L.bins[(lane >> 1) * Y::kPitch + Y::kSpare + (lane & 1)] = acc;
  }
  __builtin_amdgcn_wave_barrier();
  const int ci = lane + r2;
  const int co = lane == 0 ? ci : lane - 1;
  const uint32_t* pi = L.bins + ci * Y::kPitch + qs;
  const uint32_t* po = L.bins + co * Y::kPitch + qs;
  // F[2q]: leaves 4q and 4q + 2, F[2q + 1]: leaves 4q + 1 and 4q + 3
  vu<32> F;
#pragma unroll
  for (int k = 0; k < 16; k += 4) {
    const uint4 a = *(const uint4*)(pi + k);
    const uint4 b = *(const uint4*)(po + k);
    const uint32_t av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = k + i;
      const uint2 b16 = *(const uint2*)(L.bins + q * Y::kPitch + Y::kSpare);
      F[2 * q] = b16.x + wave_scan((av[i] & 0x00ff00ffu) - (bv[i] & 0x00ff00ffu));
      F[2 * q + 1] =
          b16.y + wave_scan(((av[i] >> 8) & 0x00ff00ffu) - ((bv[i] >> 8) & 0x00ff00ffu));
    }
  }
  __builtin_amdgcn_wave_barrier();
  vu<16> t0;
#pragma unroll
  for (int q = 0; q < 16; ++q)
    t0[q] = (F[2 * q] & 0xffffu) + (F[2 * q] >> 16) + (F[2 * q + 1] & 0xffffu) +
            (F[2 * q + 1] >> 16);
  const vu<8> t1 = pairs<16>(t0);
  const vu<4> t2 = pairs<8>(t1);
  const vu<2> t3 = pairs<4>(t2);
  cnt = (int)(t3[0] + t3[1]);
  const int kp = rank - below;
  ok = kp >= 0 && kp < cnt;
  uint32_t k = (uint32_t)kp;
  const bool b1 = step(t3[0], k);
  const bool b2 = step(pick<2>(evens<4>(t2), b1), k);
  const bool b3 = step(pick<4>(evens<8>(t1), b1, b2), k);
  const bool b4 = step(pick<8>(evens<16>(t0), b1, b2, b3), k);
  vu<16> lo, hi;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    lo[q] = F[2 * q];
    hi[q] = F[2 * q + 1];
  }
  const uint32_t fl = pick<16>(lo, b1, b2, b3, b4), fh = pick<16>(hi, b1, b2, b3, b4);
  const bool b5 = step((fl & 0xffffu) + (fh & 0xffffu), k);
  const bool b6 = step(b5 ? fl >> 16 : fl & 0xffffu, k);
  off = (b1 ? 32 : 0) + (b2 ? 16 : 0) + (b3 ? 8 : 0) + (b4 ? 4 : 0) + (b5 ? 2 : 0) + (b6 ? 1 : 0);
}

// One wave's tile `tile` of the image `a` (tiles in launch order: short
// segments near the image's edges first (see WindowArgs), then the inner
// strips' segments, neighbouring strips together; volumes (D3): slice by
// slice, each in that order - 6 % faster at r = 3 and 5 than running the
// slices of one 2-D tile in turn);
// wv = the wave's index in its workgroup, uniform (its LDS area).  A volume's
// column holds the (2r + 1) x (2r + 1) values of its rows and slices.
template <typename T, bool ADAPT, int KC, int BQ, bool D3 = false>
__device__ __forceinline__ void window_tile(const WindowArgs& a, int64_t tile, int wv,
                                            uint8_t* lds) {
  using Y = Layout<BQ>;
  const int lane = threadIdx.x & 63;
  int strip, y0, y1;
  int z = 0;
  if constexpr (D3) {
    const int64_t per = window_tile_count(a);
    z = (int)(tile / per);
    tile %= per;
  }
  if (!window_tile_rows(a, tile, strip, y0, y1)) return;
  const T* __restrict__ src = (const T*)a.src;
  T* __restrict__ dst = (T*)a.dst + (D3 ? z * a.dss : 0);
  const int r = a.r, r2 = 2 * a.r, ncols = 64 + 2 * a.r;
  const int w = (int)a.w, h = (int)a.h;
  const int x0 = strip * 64;
  int gx[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int x = x0 - r + lane + 64 * k;
    gx[k] = x < 0 ? 0 : (x > w - 1 ? w - 1 : x);
  }

  WaveLds L;
  L.bins = (uint32_t*)(lds + (size_t)wv * a.wave_bytes);
  L.base = (uint32_t*)(lds + (size_t)wv * a.wave_bytes + window_base_offset(ncols, BQ));
  const int wave_dwords = a.wave_bytes / 4;

  y1 = y1 < h ? y1 : h;
  const bool live = x0 + lane < w;
  constexpr int maxv = sizeof(T) == 2 ? 65535 : 255;
  const int rank = (int)a.rank;

  // scanned range: dwords [q0, q0 + sq) of the leaves [bc, bc + 128);
  // adaptive trees scan 16 dwords placed on the medians, widening to all 32
  // for rows whose medians spread wider; the uniform tree scans both of its
  // 64-leaf subtrees, or (8-bit) only one of them from a row whose medians
  // lie well inside it until a median leaves it.  (16-bit: the medians of a
  // row at r = 10..31 rarely fit one subtree, and the second code path alone
  // measured 8 % slower; 8-bit low-key 8192^2 r = 8: 1.13 -> 0.89 ms.)
  constexpr bool kNarrowPlain = sizeof(T) == 1 && BQ == 32;
  int bc = 0, q0 = 0;
  bool wide = !ADAPT;  // adaptive trees start on 16 dwords
  auto place = [&](int m) {
    if (!ADAPT) {  // BQ / 16 64-leaf subtrees of the uniform tree, m in the middle half
      bc = (m - 2 * Y::kBinQ + 32) & ~63;
      bc = bc < 0 ? 0 : bc;
      q0 = 0;
      wide = true;
    } else if (wide) {
      bc = (m - 2 * Y::kBinQ) & ~15;
      bc = bc < 0 ? 0 : bc;
      q0 = 0;
    } else {  // 64 scanned leaves centred on m, in the middle of the 4 BQ leaves
      int bs = (m - 32 + 8) & ~15;
      bs = bs < 0 ? 0 : bs;
      bc = bs - (2 * Y::kBinQ - 32) < 0 ? 0 : bs - (2 * Y::kBinQ - 32);
      q0 = (bs - bc) >> 2;
    }
  };
  auto sq = [&]() { return wide ? Y::kBinQ : 16; };
  auto estimate = [&](int lane_of, int y) -> int {
    const int xc = x0 + lane_of < w ? x0 + lane_of : w - 1;
    return window_rank_exact<T, D3>(src, a.srs, a.w, a.h, xc, y, r, rank, L.bins, lane,
                                    D3 ? a.sss : 0, D3 ? a.d : 1, z);
  };
  auto build = [&](int y) {
    rebuild<T, KC, BQ, D3>(src, a.srs, h, r, gx, ncols, L, wave_dwords, y, bc, q0, sq(), lane,
                           D3 ? a.sss : 0, D3 ? a.d : 1, z);
  };
  // a row this strip cannot finish: flag the tiered kernel's tile holding it
  // (that tile is recomputed whole after this launch)
  auto flag_row = [&](int y) {
    const int64_t seg = (D3 ? (int64_t)z * a.fb_segs : 0) + y / a.fb_rows;
    if (lane == 0) a.need[seg * a.fb_strips + x0 / kBlock] = 1u;
  };

  place(estimate(32, y0));
  build(y0);
  int prev = -1;  // this lane's result in the previous row

  for (int y = y0; y < y1; ++y) {
    // raw values of the next row step (rows yo out, yi in), loaded before
    // they are needed (volumes: those of its first slice; each further
    // slice's are loaded while the one before is applied)
    const int yo = y - r < 0 ? 0 : (y - r > h - 1 ? h - 1 : y - r);
    const int yi = y + r + 1 > h - 1 ? h - 1 : y + r + 1;
    int vo[KC], vi[KC];
    auto load_slice = [&](int zz, int (&o)[KC], int (&i)[KC]) {
      const T* sz = src + (D3 ? clampi(zz, a.d - 1) * a.sss : 0);
      const T* ro = sz + (int64_t)yo * a.srs;
      const T* ri = sz + (int64_t)yi * a.srs;
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        o[k] = (int)ro[gx[k]];
        i[k] = (int)ri[gx[k]];
      }
    };
    load_slice(z - r, vo, vi);
    // passes over the row until every live pixel has its result: a range
    // that misses some medians moves (adaptive: first to all 128 leaves;
    // uniform: by one subtree) or is rebuilt around the exact median of the
    // first pixel still open; results already found stay
    int res = 0;
    bool have = false, done = true, moved = false;
    for (int tries = 0;; ++tries) {
      RowOut o;
      if (!wide)
        o = row_medians<BQ, 16>(L, q0, lane, r2, ncols, a.n, rank, live);
      else
        o = row_medians<BQ, BQ>(L, q0, lane, r2, ncols, a.n, rank, live);
      if (!have && o.ok) {
        res = bc + 4 * q0 + o.off;
        have = true;
      }
      uint64_t open = ballot(live && !have);
      if (!open) break;
      if (open & ~(o.low | o.high)) {
        // a leaf count passed 255: count the scanned leaves again with
        // 16-bit fields, 64 leaves at a time
        int below = o.lo;
        for (int qs = q0; qs < q0 + (!wide ? 16 : Y::kBinQ); qs += 16) {
          int off16, cnt16;
          bool ok16;
          row16<BQ>(L, qs, lane, r2, rank, below, off16, ok16, cnt16);
          if (!have && ok16) {
            res = bc + 4 * qs + off16;
            have = true;
          }
          below += cnt16;
        }
        open = ballot(live && !have);
        if (!open) break;
      }
      // a count that still disagrees, or too many passes: the tiered kernel
      // takes this row
      if ((open & ~(o.low | o.high)) || tries >= kMaxPasses) {
        done = false;
        break;
      }
      if (!wide) {  // scan all 128 leaves
        retarget<KC, BQ>(L, ncols, r2, q0, 16, 0, Y::kBinQ, lane);
        q0 = 0;
        wide = true;
        continue;
      }
      const uint64_t lo = o.low & open, hi = o.high & open;
      if (!ADAPT && tries == 0 && !(lo && hi)) {  // move the pair of subtrees by one
        const int nbc = bc + (lo ? -64 : 64);
        if (nbc >= 0 && nbc <= maxv) {
          bc = nbc;
          build(y);
          continue;
        }
      }
      // around the first open pixel's previous-row result (medians move
      // little from row to row), else its exact median
      const int fl = (int)__builtin_ctzll(open);
      const int pm = readlane(prev, fl);
      place(pm >= 0 && !moved ? pm : estimate(fl, y));
      moved = pm >= 0;
      build(y);
    }
    if (!done) {
      // leave the rest of the fallback tile to the tiered kernel and start
      // again at the next one
      flag_row(y);
      const int ny = (y / a.fb_rows + 1) * a.fb_rows;
      if (ny >= y1) return;
      y = ny - 1;
      prev = -1;
      place(estimate(32, ny));
      build(ny);
      continue;
    }
    if (live) dst[(int64_t)y * a.drs + x0 + lane] = (T)res;
    prev = live ? res : -1;
    if (y + 1 >= y1) break;
    const int off = res - (bc + 4 * q0);  // relative to the current scanned leaves

    // keep the medians away from the edges of the scanned leaves
    constexpr int kMargin = 8;
    bool rebuilt = false;
    if (ADAPT && wide) {
      // back to 16 scanned dwords once the row's medians fit them with margins
      int q1 = -1;
#pragma unroll
      for (int q = 0; q <= Y::kBinQ - 16; q += 4)
        if (q1 < 0 && !ballot(live && (off < 4 * q + kMargin || off >= 4 * q + 64 - kMargin)))
          q1 = q;
      if (q1 >= 0) {
        retarget<KC, BQ>(L, ncols, r2, 0, Y::kBinQ, q1, 16, lane);
        q0 = q1;
        wide = false;
      }
    } else if (ADAPT) {
      // (the shift tests only for rows with a median near an edge that can move)
      const int bs = bc + 4 * q0;
      if (ballot(live && ((bs > 0 && off < kMargin) || (bs + 64 <= maxv && off >= 64 - kMargin)))) {
        const bool near_lo = ballot(live && off < kMargin) != 0;
        const bool near_hi = ballot(live && off >= 64 - kMargin) != 0;
        // shift by 16 leaves when the far side keeps its margin afterwards
        const bool room_lo = ballot(live && off >= 64 - kMargin - 16) == 0;
        const bool room_hi = ballot(live && off < kMargin + 16) == 0;
        if (near_lo && room_lo && bs > 0) {
          if (q0 >= 4) {
            retarget<KC, BQ>(L, ncols, r2, q0, 16, q0 - 4, 16, lane);
            q0 -= 4;
          } else {
            place(bs + 32 - 16);
            build(y + 1);
            rebuilt = true;
          }
        } else if (near_hi && room_hi && bs + 64 <= maxv) {
          if (q0 + 4 <= Y::kBinQ - 16) {
            retarget<KC, BQ>(L, ncols, r2, q0, 16, q0 + 4, 16, lane);
            q0 += 4;
          } else {
            place(bs + 32 + 16);
            build(y + 1);
            rebuilt = true;
          }
        }
      }
    } else if (kNarrowPlain && !wide) {
      // one subtree scanned: it stays until a median leaves it (a pass that
      // misses scans both again)
    } else if (kNarrowPlain && (!ballot(live && (off < kMargin || off >= 64 - kMargin)) ||
                                !ballot(live && (off < 64 + kMargin || off >= 128 - kMargin)))) {
      // the row's medians lie well inside one subtree: scan only that one
      const int q1 = ballot(live && off >= 64) ? 16 : 0;
      retarget<KC, BQ>(L, ncols, r2, 0, Y::kBinQ, q1, 16, lane);
      q0 = q1;
      wide = false;
    } else {
      // move the pair of subtrees by one subtree
      const bool near_lo = ballot(live && off < kMargin) != 0;
      const bool near_hi = ballot(live && off >= 4 * Y::kBinQ - kMargin) != 0;
      const bool room_lo = ballot(live && off >= 4 * Y::kBinQ - 64 - kMargin) == 0;
      const bool room_hi = ballot(live && off < 64 + kMargin) == 0;
      if ((near_lo && room_lo && bc >= 64) || (near_hi && room_hi && bc + 4 * Y::kBinQ <= maxv)) {
        bc += near_lo ? -64 : 64;
        build(y + 1);
        rebuilt = true;
      }
    }
    if (rebuilt) continue;

    // row step y -> y + 1: remove row y - r, insert row y + r + 1 (clamped);
    // a removal and an insertion in one dword are one update
    const int s = sq();
    for (int dz = D3 ? -r : 0; dz <= (D3 ? r : 0); ++dz) {
    int no[KC], ni[KC];
    if (D3 && dz < r) load_slice(z + dz + 1, no, ni);
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int c = lane + 64 * k;
      if (c < ncols) {
        const Cls o = classify<BQ>(vo[k], bc, q0, s);
        const Cls i = classify<BQ>(vi[k], bc, q0, s);
        const bool same = i.q == o.q;
        const uint32_t di = same ? i.inc - o.inc : i.inc;
        const uint32_t dl = i.lh - o.lh;
        uint32_t* col = L.bins + c * Y::kPitch;
        lds_add(col + i.q, di);
        lds_add(col + (same ? Y::kSink : o.q), same ? 0u : 0u - o.inc);
        lds_add(lohi_of<BQ>(L, c), dl);
        if (c <= r2) {
          lds_add(L.base + i.q, di);
          lds_add(L.base + (same ? Y::kSink : o.q), same ? 0u : 0u - o.inc);
          lds_add(L.base + Y::kLohi, dl);
        }
      }
    }
    if (D3 && dz < r) {
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        vo[k] = no[k];
        vi[k] = ni[k];
      }
    }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Columns one lane holds: ceil((64 + 2r) / 64).
constexpr int kc_for(int r) { return (64 + 2 * r + 63) / 64; }

template <typename T, bool ADAPT, int KC, int WPG, int BQ, bool D3 = false>
__global__ __launch_bounds__(64 * WPG) void k_median_window(WindowArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  // the wave's index in the workgroup, as a value the compiler knows to be
  // uniform: everything derived from it (tile, rows, range) stays scalar
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  window_tile<T, ADAPT, KC, BQ, D3>(a, (int64_t)blockIdx.x * WPG + wv, wv, lds);
}

// Many images in one launch (uniform tree): workgroup g belongs to the first
// image whose workgroup range ends after g; each image's tiles start on a
// workgroup boundary, so the waves of a workgroup share one image (and its
// LDS layout).  The launch's LDS holds WPG waves of the largest image radius.
template <typename T, int KC, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_median_window_multi(
    const WindowImage* __restrict__ imgs, int n) {
  extern __shared__ __align__(16) uint8_t lds[];
  const int64_t g = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (imgs[mid].group_end > g)
      hi = mid;
    else
      lo = mid + 1;
  }
  const int64_t first = lo > 0 ? imgs[lo - 1].group_end : 0;
  const WindowArgs a = imgs[lo].args;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  window_tile<T, false, KC, 32>(a, (g - first) * WPG + wv, wv, lds);
}

template <typename T, bool ADAPT, int KC, int WPG, int BQ = 32, bool D3 = false>
hipError_t launch_k(const WindowArgs& a, hipStream_t stream) {
  const size_t lds = (size_t)WPG * a.wave_bytes;
  const void* kern = (const void*)k_median_window<T, ADAPT, KC, WPG, BQ, D3>;
  hipError_t e = ensure_dynamic_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int64_t grid = (window_tiles(a) + WPG - 1) / WPG;
  hipLaunchKernelGGL((k_median_window<T, ADAPT, KC, WPG, BQ, D3>), dim3((uint32_t)grid),
                     dim3(64 * WPG), lds, stream, a);
  return hipGetLastError();
}

template <typename T, bool ADAPT>
hipError_t launch_w(const WindowArgs& a, hipStream_t stream) {
  const int kc = kc_for(a.r);
  const int wpg = window_launch_wpg((int)sizeof(T), a.r, a.bq);
  if (a.bq == 64)  // (r <= 32: two columns per lane)
    return wpg == 4 ? launch_k<T, ADAPT, 2, 4, 64>(a, stream) : launch_k<T, ADAPT, 2, 1, 64>(a, stream);
  if (kc <= 2)
    return wpg == 4 ? launch_k<T, ADAPT, 2, 4>(a, stream) : launch_k<T, ADAPT, 2, 1>(a, stream);
  if (kc == 3) return wpg == 4 ? launch_k<T, ADAPT, 3, 4>(a, stream)
                               : launch_k<T, ADAPT, 3, 2>(a, stream);
  return wpg == 2 ? launch_k<T, ADAPT, 5, 2>(a, stream) : launch_k<T, ADAPT, 5, 1>(a, stream);
}

template <typename T, bool ADAPT>
hipError_t prime_w() {
  const void* ks[] = {(const void*)k_median_window<T, ADAPT, 2, 4, 32>,
                      (const void*)k_median_window<T, ADAPT, 2, 1, 32>,
                      (const void*)k_median_window<T, ADAPT, 3, 4, 32>,
                      (const void*)k_median_window<T, ADAPT, 3, 2, 32>,
                      (const void*)k_median_window<T, ADAPT, 5, 2, 32>,
                      (const void*)k_median_window<T, ADAPT, 5, 1, 32>};
  for (const void* k : ks) {
    const hipError_t e = ensure_dynamic_lds(k, kLdsLimit);
    if (e != hipSuccess) return e;
  }
  const void* k64[] = {(const void*)k_median_window<T, ADAPT, 2, 4, 64>,
                       (const void*)k_median_window<T, ADAPT, 2, 1, 64>};
  for (const void* k : k64) {
    const hipError_t e = ensure_dynamic_lds(k, kLdsLimit);
    if (e != hipSuccess) return e;
  }
  if constexpr (sizeof(T) == 2) {
    const hipError_t e =
        ensure_dynamic_lds((const void*)k_median_window<T, ADAPT, 2, 1, 32, true>, kLdsLimit);
    if (e != hipSuccess) return e;
    return ensure_dynamic_lds((const void*)k_median_window<T, ADAPT, 2, 1, 64, true>, kLdsLimit);
  }
  return hipSuccess;
}

}  // namespace

int64_t window_tiles(const WindowArgs& a) {
  return window_tile_count(a) * (a.dims == 3 ? a.d : 1);
}

// Waves per CU with workgroups of wpg waves at radius r (LDS is granted to a
// workgroup in blocks of 1,280 bytes).
static int waves_at(int wpg, int r, int bq) {
  const size_t per = ((size_t)wpg * window_wave_bytes(r, bq) + 1279) / 1280 * 1280;
  const int waves = (int)((size_t)kLdsLimit / per) * wpg;
  return waves < 32 ? (waves > 0 ? waves : 1) : 32;
}

int window_launch_wpg(int bytes, int r, int bq) {
  const int kc = kc_for(r);
  if (kc <= 2) {
    // one- or four-wave workgroups, whichever lets more waves share a CU
    // (16-bit X-ray-like 4096^2 r = 15: 11 against 8 waves, 0.47 -> 0.41 ms);
    // on a tie 8-bit launches, which have four times the waves, take four
    // (8-bit low-key 8192^2 r = 8: 0.94 -> 0.87 ms)
    const int w1 = waves_at(1, r, bq), w4 = waves_at(4, r, bq);
    return bytes == 1 ? (w4 >= w1 ? 4 : 1) : (w1 >= w4 ? 1 : 4);
  }
  const int wpg = window_waves_per_group(r);
  if (kc == 3) return wpg >= 4 ? 4 : 2;
  return wpg >= 2 ? 2 : 1;
}

int window_waves_per_cu(int bytes, int r, int bq) {
  return waves_at(window_launch_wpg(bytes, r, bq), r, bq);
}

int window_bq(int bytes, int r, bool adaptive) {
  // 16-bit windows of r <= 7: 256 grey levels per column, as their rows'
  // medians spread over more than 128 (X-ray-like 4096^2 r = 5: uniform tree
  // 0.69 against 1.73 ms, adaptive 0.82 against 1.71; r = 7 0.59 against
  // 0.69, adaptive 0.67 against 1.11); the adaptive tree at r = 1 keeps 128
  // (1.27 against 5.3 ms: its narrow ranges there miss more often)
  return bytes == 2 && r <= 7 && (!adaptive || r >= 2) ? 64 : 32;
}

int window_multi_waves(int bytes, int r_max) {
  return kc_for(r_max) > 2 ? 0 : bytes == 2 ? 1 : 4;
}

hipError_t launch_window_multi(const WindowImage* d_imgs, int n, int64_t groups, int bytes,
                               int r_max, hipStream_t stream) {
  if (n <= 0 || groups <= 0) return hipSuccess;
  if (kc_for(r_max) > 2 || groups > 0x7fffffffLL) return hipErrorInvalidValue;
  const int wpg = window_multi_waves(bytes, r_max);
  const size_t lds = (size_t)wpg * window_wave_bytes(r_max, 32);
  const void* kern = bytes == 2 ? (const void*)k_median_window_multi<uint16_t, 2, 1>
                                : (const void*)k_median_window_multi<uint8_t, 2, 4>;
  hipError_t e = ensure_dynamic_lds(kern, lds);
  if (e != hipSuccess) return e;
  if (bytes == 2)
    hipLaunchKernelGGL((k_median_window_multi<uint16_t, 2, 1>), dim3((uint32_t)groups), dim3(64),
                       lds, stream, d_imgs, n);
  else
    hipLaunchKernelGGL((k_median_window_multi<uint8_t, 2, 4>), dim3((uint32_t)groups),
                       dim3(256), lds, stream, d_imgs, n);
  return hipGetLastError();
}

size_t window_wave_bytes(int r, int bq) {
  const int ncols = 64 + 2 * r;
  // + base and a block of zeros (bq + 4 dwords each)
  return window_base_offset(ncols + 2, bq);
}

int window_waves_per_group(int r) {
  const size_t b = window_wave_bytes(r, 32);
  return 4 * b <= (size_t)kLdsLimit ? 4 : 2 * b <= (size_t)kLdsLimit ? 2 : 1;
}

hipError_t launch_window(const WindowArgs& a, int bytes, bool adaptive, hipStream_t stream) {
  if (a.dims == 3) {
    // 16-bit volumes, r <= 7: two columns per lane, 128 grey levels (r <= 3:
    // 256), one-wave workgroups (14 waves per CU at r = 7)
    if (bytes != 2 || kc_for(a.r) > 2 || window_launch_wpg(2, a.r, a.bq) != 1)
      return hipErrorInvalidValue;
    if (a.bq == 64)
      return adaptive ? launch_k<uint16_t, true, 2, 1, 64, true>(a, stream)
                      : launch_k<uint16_t, false, 2, 1, 64, true>(a, stream);
    if (a.bq != 32) return hipErrorInvalidValue;
    return adaptive ? launch_k<uint16_t, true, 2, 1, 32, true>(a, stream)
                    : launch_k<uint16_t, false, 2, 1, 32, true>(a, stream);
  }
  if (bytes == 1)
    return adaptive ? launch_w<uint8_t, true>(a, stream) : launch_w<uint8_t, false>(a, stream);
  return adaptive ? launch_w<uint16_t, true>(a, stream) : launch_w<uint16_t, false>(a, stream);
}

__global__ void k_clear_flags(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_clear_flags(uint32_t* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256 < 64 ? (n + 255) / 256 : 64;
  hipLaunchKernelGGL(k_clear_flags, dim3((uint32_t)blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t prime_window_lds() {
  hipError_t e = prime_w<uint8_t, true>();
  if (e == hipSuccess) e = prime_w<uint8_t, false>();
  if (e == hipSuccess) e = prime_w<uint16_t, true>();
  if (e == hipSuccess) e = prime_w<uint16_t, false>();
  if (e == hipSuccess)
    e = ensure_dynamic_lds((const void*)k_median_window_multi<uint8_t, 2, 4>, kLdsLimit);
  if (e == hipSuccess)
    e = ensure_dynamic_lds((const void*)k_median_window_multi<uint16_t, 2, 1>, kLdsLimit);
  return e;
}

}  // namespace hrrm
