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

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t hi) {
  return v < 0 ? 0 : (v > hi ? hi : v);
}

__device__ __forceinline__ size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Workgroup tile from blockIdx: consecutive workgroups land on consecutive
// XCDs; remap so that each XCD works on a contiguous band of tiles (shared
// halos stay in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, rem = nb & 7, xcd = bid & 7, i = bid >> 3;
  return xcd * q + (xcd < rem ? xcd : rem) + i;
}

}  // namespace hrrm
