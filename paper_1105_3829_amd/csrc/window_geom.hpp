// Tile geometry of the grey-level-window kernel (2-D): which strip and rows
// each tile (one wave) covers, and how the host lays the tiles out.  Shared
// by the kernel, the launch set-up and a host test of the decomposition.
#pragma once

#include <stdint.h>

#include "hrrm_internal.h"

namespace hrrm {

// Number of tiles of a launch.
__host__ __device__ inline int64_t window_tile_count(const WindowArgs& a) {
  const int64_t inner = a.strips > 2 ? a.strips - 2 : 0;
  if (!inner) return a.border_tiles;
  return (int64_t)a.border_tiles + inner * ((a.tail_start - a.top_end + a.seg_rows - 1) / a.seg_rows) +
         inner * ((a.bot_start - a.tail_start + a.tail_rows - 1) / a.tail_rows);
}

// Strip and rows [y0, y1) of tile `tile` (tiles in launch order: the edge
// tiles in short segments first, see WindowArgs, then the inner strips'
// segments, neighbouring strips together); false past the last tile.
__host__ __device__ inline bool window_tile_rows(const WindowArgs& a, int64_t tile, int& strip,
                                                 int& y0, int& y1) {
  const int inner = a.strips > 2 ? a.strips - 2 : 0;
  const int64_t mid_tiles =
      inner ? (int64_t)inner * ((a.tail_start - a.top_end + a.seg_rows - 1) / a.seg_rows) : 0;
  const int64_t tail_tiles =
      inner ? (int64_t)inner * ((a.bot_start - a.tail_start + a.tail_rows - 1) / a.tail_rows) : 0;
  if (tile >= (int64_t)a.border_tiles + mid_tiles + tail_tiles) return false;
  if (tile < a.side_tiles) {
    const int sides = a.strips > 1 ? 2 : 1;
    strip = (int)(tile % sides) ? a.strips - 1 : 0;
    y0 = (int)(tile / sides) * a.border_rows;
    y1 = y0 + a.border_rows;
  } else if (tile < a.side_tiles + a.top_tiles) {
    const int j = (int)(tile - a.side_tiles);
    strip = 1 + j % inner;
    y0 = (j / inner) * a.border_rows;
    y1 = y0 + a.border_rows < a.top_end ? y0 + a.border_rows : a.top_end;
  } else if (tile < a.border_tiles) {
    const int j = (int)(tile - a.side_tiles - a.top_tiles);
    strip = 1 + j % inner;
    y0 = a.bot_start + (j / inner) * a.border_rows;
    y1 = y0 + a.border_rows;
  } else if (tile < a.border_tiles + mid_tiles) {
    const int64_t j = tile - a.border_tiles;
    strip = 1 + (int)(j % inner);
    y0 = a.top_end + (int)(j / inner) * a.seg_rows;
    y1 = y0 + a.seg_rows < a.tail_start ? y0 + a.seg_rows : a.tail_start;
  } else {
    const int64_t j = tile - a.border_tiles - mid_tiles;
    strip = 1 + (int)(j % inner);
    y0 = a.tail_start + (int)(j / inner) * a.tail_rows;
    y1 = y0 + a.tail_rows < a.bot_start ? y0 + a.tail_rows : a.bot_start;
  }
  y1 = y1 < a.h ? y1 : (int)a.h;
  return true;
}

// Tile layout of an image of w x h pixels with segments of `seg` rows.
// slots = waves the GPU holds at once; alone = the image has the GPU to
// itself: segments are shortened until it fills two generations of waves,
// and (r <= 32) the inner strips' last generation runs in half-height
// segments, so that the launch's last waves end together.
inline void window_geometry(WindowArgs& wa, int64_t w, int64_t h, int64_t seg, int64_t slots,
                            bool alone, int r) {
  wa.strips = (int32_t)((w + 63) / 64);
  if (alone && seg > 8 && (int64_t)wa.strips * ((h + seg - 1) / seg) < 2 * slots) {
    int64_t s = (int64_t)wa.strips * h / (2 * slots);
    s = s < seg ? s : seg;
    seg = s > 8 ? s : 8;
  }
  wa.seg_rows = (int32_t)(seg < 1 ? 1 : (seg < h ? seg : h));
  wa.segs = (int32_t)((h + wa.seg_rows - 1) / wa.seg_rows);
  wa.border_rows = wa.seg_rows < 8 ? wa.seg_rows : 8;
  const int64_t br = wa.border_rows, inner = wa.strips > 2 ? wa.strips - 2 : 0;
  const int64_t top_end = h < wa.seg_rows ? h : wa.seg_rows;
  const int64_t bot_start = top_end > h - wa.seg_rows ? top_end : h - wa.seg_rows;
  wa.top_end = (int32_t)top_end;
  wa.bot_start = (int32_t)bot_start;
  wa.tail_rows = wa.seg_rows / 2 > 1 ? wa.seg_rows / 2 : 1;
  int64_t tail_start = bot_start;
  if (alone && inner > 0 && wa.seg_rows >= 16 && r <= 32) {
    const int64_t tail_segs = (slots + inner - 1) / inner;
    tail_start = bot_start - tail_segs * wa.tail_rows;
    tail_start = tail_start > top_end ? tail_start : top_end;
  }
  wa.tail_start = (int32_t)tail_start;
  wa.side_tiles = (int32_t)((wa.strips > 1 ? 2 : 1) * ((h + br - 1) / br));
  wa.top_tiles = (int32_t)(inner * ((top_end + br - 1) / br));
  wa.border_tiles = (int32_t)(wa.side_tiles + wa.top_tiles + inner * ((h - bot_start + br - 1) / br));
}

}  // namespace hrrm
