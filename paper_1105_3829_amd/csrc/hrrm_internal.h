// Internal declarations shared by the HIP kernels and the host-side C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hrrm {

constexpr int kBlock = 256;          // threads per workgroup = output columns per strip
constexpr int kWaves = kBlock / 64;  // wave64
constexpr int kTierLevels = 4;       // tree levels held by one tier slot
constexpr int kTierNodes = (1 << kTierLevels) - 1;  // left-node counters per tier slot
constexpr int kDenseNodes = 255;     // left-node counters of a full 8-bit tree
constexpr int kHash = 128;           // slot hash-table entries (power of two)
constexpr int kMaxSlots = 64;        // tier slots per workgroup, slot 0 included
constexpr int kLdsLimit = 160 * 1024;
// Largest LDS budgets at which three, four or six workgroups share one CU.
// LDS is granted in blocks of 1,280 bytes (measured on MI355X: 53,536 bytes
// per workgroup let three in and 53,856 did not).
constexpr int kLdsThird = 53760;
constexpr int kLdsQuarter = 40960;
constexpr int kLdsSixth = 26880;

// Workgroups of the tiered kernel that share one CU at this LDS budget; past
// kLdsThird the build that runs them has registers for three waves per SIMD,
// and for four or six only when it counts no subtree wave-wide
// (max_groups = 0).
constexpr int tiered_per_cu(int lds_budget, int max_groups) {
  return lds_budget > kLdsLimit / 2   ? 1
         : lds_budget > kLdsThird     ? 2
         : lds_budget > kLdsQuarter   ? 3
         : max_groups > 0             ? 3
         : lds_budget > kLdsSixth     ? 4
                                      : 6;
}
constexpr int kRawWindow = 81;       // (2r+1)^D up to this: missing subtrees counted raw

// Bytes of one wave's scratch area in the tiered kernel: the column vectors
// of a subtree for the wave's 64 + 2r + 1 columns (16 bytes each), or the
// raw-count histograms (8 x 64 dwords) plus one staged window row of
// 64 + 2r 16-bit values, whichever is larger; 16-byte aligned.
__host__ __device__ constexpr size_t wave_scratch_bytes(int r) {
  const size_t cols = (size_t)(64 + 2 * r + 1) * 16;
  const size_t raw = 8 * 64 * 4 + (size_t)(64 + 2 * r) * 2;
  return ((cols > raw ? cols : raw) + 15) & ~(size_t)15;
}

// Adaptive topology node.  Internal nodes are numbered 0..2^d-2 (root 0).
// A child >= 0 is an internal node; a child < 0 is the leaf holding grey value
// (-child - 1).  The left child covers [lo, split-1], the right [split, hi].
struct TopoNode {
  int32_t split, left, right, pad;
};

// Everything one launch of the median kernel needs.  Strides in elements.
struct MedianArgs {
  const void* src;
  void* dst;
  int64_t w, h, d;
  int64_t srs, sss, drs, dss;
  int64_t rank;       // K, 0-based
  int32_t r;
  int32_t bits;       // 8 or 16
  int32_t stop;       // levels to descend (bits - drop_levels; adaptive: large)
  int32_t seg_rows;   // output rows per workgroup
  int32_t strips, segs;
  int32_t ncols, cp;  // columns held per strip, padded byte pitch of a counter row
  int32_t nslots;     // tier slots incl. slot 0 (tiered storage)
  int32_t min_group;  // smallest lane group counted cooperatively
  int32_t max_groups; // cooperative groups per level before falling back to direct sums
  int32_t raw_window; // windows of at most this many values count a missing subtree raw
  int32_t mfma;       // 1: window counts on the matrix cores (8-bit 2-D, column counts
                      // <= 127); 0 = DPP-scan and per-lane counts
  int32_t wslots;     // > 0: slots per wave of wave-private deeper subtrees (uniform 2-D)
  int32_t wpitch;     // columns per wave-private slot (>= 64 + 2r + 1)
  int32_t pad1;
  const TopoNode* topo;  // adaptive topology (device), else null
  // non-null: recompute only the tiles whose flag is set (flag index = the
  // tile's workgroup index, 2-D), clearing each flag it consumes
  uint32_t* need;
};

// One image of a persistent batched launch: its launch arguments, element size
// and the exclusive end of its range in the batch's tile index space.
struct BatchImage {
  MedianArgs args;
  int64_t tile_end;
  int32_t bytes;
  int32_t pad;
};

// Tile shape / strategy of one launch.
struct TileConfig {
  int32_t seg_rows;
  int32_t nslots;     // 0 = as many as fit the LDS budget
  int32_t min_group;
  int32_t max_groups;
  int32_t lds_budget; // bytes of LDS one workgroup may use
  int32_t tiered_u8;  // 1 = tiered storage for u8 as well
  int32_t raw_window; // windows of at most this many values count deeper tiers raw
  int32_t wave_slots; // 1 = deeper subtrees in wave-private slots (uniform 2-D)
  int32_t window_rows; // > 0: 2-D grey-level-window kernel, strip segments of this many rows
};

// One launch of the grey-level-window kernel (2-D): strips of 64 output
// columns x seg_rows rows, one wave each.  A strip segment that cannot finish
// sets the flags of the tiered kernel's tiles (fb_strips x fb_rows geometry)
// covering its remaining rows in `need`.
struct WindowArgs {
  const void* src;
  void* dst;
  int64_t w, h, srs, drs;
  int64_t d, sss, dss;  // volumes: slices and slice strides (images: d = 1)
  int64_t rank;
  int32_t r, n;  // radius, window size (2r+1)^dims
  int32_t dims;  // 2, or 3: cube windows, tiles of every slice
  int32_t seg_rows, strips, segs;
  // Tiles near the image's edges, whose windows are dominated by a repeated
  // edge column or row (so that their medians stray from their neighbours'),
  // run first, in short segments of border_rows rows: the first and last
  // strip over all rows (side_tiles tiles), then the other strips' rows
  // [0, top_end) (top_tiles tiles) and [bot_start, h); the rest of those
  // strips follows, rows [top_end, tail_start) in segments of seg_rows rows,
  // then rows [tail_start, bot_start) in segments of tail_rows rows (the
  // launch's last generation of waves, shorter so that it ends together).
  int32_t border_rows, border_tiles, side_tiles, top_tiles, top_end, bot_start;
  int32_t tail_start, tail_rows;
  int32_t wave_bytes;  // LDS bytes of one wave
  int32_t bq;          // dwords of leaf counters per column: 32 or 64 (uniform tree)
  uint32_t* need;
  int32_t fb_strips, fb_rows, fb_segs;
};

// One image of a multi-image window launch: its arguments and the exclusive
// end of its workgroups in the launch's grid.
struct WindowImage {
  WindowArgs args;
  int64_t group_end;
};

// LDS bytes of one wave of a window launch at radius r with bq dwords of leaf
// counters per column (32: 128 grey levels, 64: 256).
size_t window_wave_bytes(int r, int bq);
// Leaf dwords per column of a window launch (element size `bytes`, radius r).
int window_bq(int bytes, int r, bool adaptive);
// Waves per workgroup of a single window launch (element size `bytes`,
// radius r), and the waves of that launch that fit a CU.
int window_launch_wpg(int bytes, int r, int bq);
int window_waves_per_cu(int bytes, int r, int bq);
int64_t window_tiles(const WindowArgs& a);
// Waves per workgroup of a multi-image window launch of `bytes`-byte images
// whose largest radius is r_max; 0 when no such launch exists (r_max > 32).
int window_multi_waves(int bytes, int r_max);
hipError_t launch_window_multi(const WindowImage* d_imgs, int n, int64_t groups, int bytes,
                               int r_max, hipStream_t stream);
int window_waves_per_group(int r);
// adaptive = scanned range placed on the medians (64 leaves); else the uniform
// tree's pairs of 64-leaf subtrees (128 leaves)
hipError_t launch_window(const WindowArgs& a, int bytes, bool adaptive, hipStream_t stream);
hipError_t prime_window_lds();
// Zero n tile flags on `stream` with a fill kernel (no memset node in graphs).
hipError_t launch_clear_flags(uint32_t* p, int64_t n, hipStream_t stream);

// Launch the fused median kernel.  dims = 2 or 3; full = update every node of
// the window tree at every pixel (8-bit dense storage only).  Returns
// hipSuccess or the launch error.
hipError_t launch_median(const MedianArgs& a, int bytes, int dims, bool adaptive, bool tiered,
                         bool full, hipStream_t stream);

// Raise `kernel`'s dynamic-LDS limit on the current device to at least
// `bytes`.  The attribute is set only when a launch needs more than every
// earlier one of that kernel on that device, so steady-state launches (and
// launches under stream capture) make no attribute call.
hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes);

// Raise the dynamic-LDS limit of every build of the tiered, batched, dense and
// topology kernels to the most any launch can ask for, on the current device,
// so that no later launch makes an attribute call (hrrm_ctx_reserve).
hipError_t prime_tiered_lds();
hipError_t prime_dense_lds();
hipError_t prime_topology_lds();

// LDS bytes a launch with these parameters needs.
size_t median_lds_bytes(int bytes, bool adaptive, bool tiered, int ncols, int cp, int nslots);

// Tiered-kernel LDS bytes besides the slots, for radius r and element size
// `bytes` (1 or 2); adaptive trees add tiered_topo_bytes(nslots) for the held
// subtrees' topology.
size_t tiered_meta_bytes(int r, int bytes);
// LDS bytes of a launch with wave-private slots: slot 0 (cp columns), the
// tier state, and per wave its scratch plus `wslots` slots of `wpitch` columns.
size_t wps_lds_bytes(int r, int cp, int wslots, int wpitch);
size_t tiered_topo_bytes(int nslots);

// Persistent batched launch (zeroes *d_counter first, then runs `grid`
// workgroups over all tiles of the images in d_imgs; d_hdr[0] = image count).
// launch_batched_prepare sets the kernel's LDS limit; call it before capture.
// light = the build without matrix-core counts (images with max_groups 0),
// four workgroups per CU.
hipError_t launch_batched_prepare(size_t lds, bool light);
hipError_t launch_batched(const BatchImage* d_imgs, const int32_t* d_hdr, uint32_t* d_counter,
                          int grid, size_t lds, bool light, hipStream_t stream);

// Adaptive topology pre-pass (Sec. III-C).  Builds `topo` (2^bits - 1 nodes)
// from the input's global histogram mixed 1:1 with the histogram of its
// clamp-to-edge box mean over the same window, or, when `est` is given, with
// the histogram of that w x h estimate image (row stride est_rs; 2-D).  ws
// must hold topology_workspace_bytes(bits, pixels) bytes.
size_t topology_workspace_bytes(int bits, int64_t pixels);
hipError_t launch_topology(const MedianArgs& a, int bytes, int dims, void* ws, TopoNode* topo,
                           hipStream_t stream, const void* est = nullptr, int64_t est_rs = 0);

}  // namespace hrrm
