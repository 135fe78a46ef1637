// Wave64 primitives and small helpers shared by the gfx950 kernels.
#pragma once
#include "hrrm_internal.h"

namespace hrrm {

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ uint32_t readlane_u(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4, 8 inside
// each 16-lane row, then lane 15 of a row added into the next row and lane 31
// into the upper half.  Lanes whose DPP source is outside the row keep 0.
// Must run with all 64 lanes active.
__device__ __forceinline__ uint32_t wave_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
  return v;
}

__host__ __device__ __forceinline__ int64_t clampi(int64_t v, int64_t hi) {
  return v < 0 ? 0 : (v > hi ? hi : v);
}

// Element offsets of the clamped window rows (z + dz, y + j) of one output
// pixel, one row per next(): j = -r..r within each slice dz = -zr..zr,
// slice-major (3-D), or j = -r, -r + 1, ... (2-D).  The offset moves on by a
// row (slice) stride only where the step stays inside the image, so
// clamp-to-edge repeats the edge row with no per-row 64-bit clamp or
// multiply.  Past the last window row the walk goes on with rows still
// clamped into the image (valid addresses).
template <bool D3>
struct RowWalk {
  int64_t off, top, srs, sss;  // current offset; offset of row j = -r in the current slice
  int j, dz, r;
  // the step j -> j + 1 moves down a row iff 0 <= j - jlo < jn (rows y + j
  // and y + j + 1 both inside 0..h-1); the same for slices with zlo, zn
  int jlo, jn, zlo, zn;
  __host__ __device__ __forceinline__ RowWalk(int64_t y, int64_t z, int64_t h, int64_t d,
                                              int64_t srs_, int64_t sss_, int r_, int zr)
      : srs(srs_), sss(sss_), j(-r_), dz(-zr), r(r_) {
    // bounds of the advancing steps, cut to +-(4r + 16) so they fit an int:
    // exact while j and dz stay within that range (a walk covers its window
    // plus at most one batch of rows past it)
    auto lim = [&](int64_t v) -> int {
      const int64_t m = 4 * (int64_t)r_ + 16;
      return (int)(v < -m ? -m : v > m ? m : v);
    };
    jlo = lim(-y);
    jn = lim(h - 2 - y) - jlo + 1;
    jn = jn < 0 ? 0 : jn;
    zlo = lim(-z);
    zn = lim(d - 2 - z) - zlo + 1;
    zn = zn < 0 ? 0 : zn;
    const int64_t zz = D3 ? clampi(z - zr, d - 1) : z;
    top = zz * sss + clampi(y - r_, h - 1) * srs;
    off = top;
  }
  __host__ __device__ __forceinline__ void next() {
    if (!D3 || j < r) {
      off += (uint32_t)(j - jlo) < (uint32_t)jn ? srs : 0;
      ++j;
    } else {
      j = -r;
      top += (uint32_t)(dz - zlo) < (uint32_t)zn ? sss : 0;
      ++dz;
      off = top;
    }
  }
};

__device__ __forceinline__ size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Workgroup tile from blockIdx: consecutive workgroups land on consecutive
// XCDs; remap so that each XCD works on a contiguous band of tiles (shared
// halos stay in that XCD's L2).
__host__ __device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, rem = nb & 7, xcd = bid & 7, i = bid >> 3;
  return xcd * q + (xcd < rem ? xcd : rem) + i;
}

}  // namespace hrrm
