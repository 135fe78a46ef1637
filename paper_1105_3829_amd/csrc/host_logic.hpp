// Host-only logic of the library that involves no device: argument checks of
// the image entry points, the first-fit arena of the request loop and its
// admission rule.  Header-only and free of HIP so that it can be built and
// exercised (also under AddressSanitizer/UBSan) by a plain host compiler.
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <vector>

#include "hrrm.h"

namespace hrrm {

// Largest accepted size, stride or byte extent (2^46 bytes: far above any
// device memory, far below int64 overflow of the products formed here).
constexpr int64_t kMaxExtent = (int64_t)1 << 46;

// Checks one image or volume description.  Returns HRRM_OK or an error code and
// points *why at a static message.  Sizes and strides are in elements; every
// product is formed with overflow checks, after the range checks.
inline int check_image_args(const void* src, const void* dst, int dtype, int64_t w, int64_t h,
                            int64_t d, int64_t srs, int64_t sss, int64_t drs, int64_t dss, int r,
                            int dims, const char** why) {
  *why = "";
  if (dtype != HRRM_U8 && dtype != HRRM_U16) return (*why = "unknown dtype", HRRM_EINVAL);
  if (w < 0 || h < 0 || d < 0) return (*why = "negative image size", HRRM_EINVAL);
  if (r < 0) return (*why = "negative radius", HRRM_EINVAL);
  if (r > (dims == 2 ? HRRM_MAX_R_2D : HRRM_MAX_R_3D))
    return (*why = "radius above the supported maximum", HRRM_EUNSUPPORTED);
  if (w == 0 || h == 0 || d == 0) return HRRM_OK;  // nothing to do
  if (!src || !dst) return (*why = "null image pointer", HRRM_EINVAL);
  if (w > kMaxExtent || h > kMaxExtent || d > kMaxExtent || srs > kMaxExtent ||
      drs > kMaxExtent || (dims == 3 && (sss > kMaxExtent || dss > kMaxExtent)))
    return (*why = "image dimensions out of range", HRRM_EINVAL);
  if (srs < w || drs < w) return (*why = "row stride smaller than width", HRRM_EINVAL);
  const int64_t bytes = dtype == HRRM_U8 ? 1 : 2;
  if (bytes == 2 && ((((uintptr_t)src) | ((uintptr_t)dst)) & 1))
    return (*why = "uint16 buffer not 2-byte aligned", HRRM_EINVAL);
  // extent in elements: (d-1) * slice stride + (h-1) * row stride + w
  int64_t ext[2];
  const int64_t rs[2] = {srs, drs}, ss[2] = {sss, dss};
  for (int i = 0; i < 2; ++i) {
    int64_t rows = 0, slices = 0, plane = 0;
    if (__builtin_mul_overflow(h - 1, rs[i], &rows) || __builtin_add_overflow(rows, w, &ext[i]))
      return (*why = "image extent out of range", HRRM_EINVAL);
    if (dims == 3) {
      if (__builtin_mul_overflow(rs[i], h, &plane) || ss[i] < plane)
        return (*why = "slice stride smaller than row_stride * height", HRRM_EINVAL);
      if (__builtin_mul_overflow(d - 1, ss[i], &slices) ||
          __builtin_add_overflow(slices, ext[i], &ext[i]))
        return (*why = "image extent out of range", HRRM_EINVAL);
    }
    if (ext[i] > kMaxExtent / bytes) return (*why = "image extent out of range", HRRM_EINVAL);
  }
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
  const uintptr_t an = (uintptr_t)(ext[0] * bytes), bn = (uintptr_t)(ext[1] * bytes);
  if (a < b + bn && b < a + an) return (*why = "src and dst overlap", HRRM_EINVAL);
  return HRRM_OK;
}

// First-fit sub-allocator over the offsets of one device arena; sizes are
// rounded up to `align` bytes and adjacent free ranges coalesce.
class Arena {
 public:
  static constexpr size_t kAlign = 256;
  static size_t round_up(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }

  void reset(size_t n) {
    free_.clear();
    if (n) free_[0] = n;
    used_ = 0;
    size_ = n;
  }
  bool alloc(size_t n, size_t* off) {
    n = round_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t base = it->first, rest = it->second - n;
        free_.erase(it);
        if (rest) free_[base + n] = rest;
        *off = base;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = round_up(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  size_t free_ranges() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, size_ = 0;
};

// One admission round of the request loop.  `need[i]` = (input bytes, output
// bytes) of the i-th queued request, in arrival order.  Requests are admitted
// in order while fewer than `slots` are admitted; a request whose buffers do
// not fit is passed, and at most `bypass` such passes are made before the
// round stops (so a large request is not starved by a stream of small ones).
// Returns the admitted queue positions with their (input, output) offsets.
struct Admitted {
  size_t index, off_in, off_out;
};
inline std::vector<Admitted> plan_admission(Arena& arena,
                                            const std::vector<std::pair<size_t, size_t>>& need,
                                            int slots, int bypass) {
  std::vector<Admitted> out;
  int passed = 0;
  for (size_t i = 0; i < need.size() && (int)out.size() < slots; ++i) {
    size_t oi = 0, oo = 0;
    if (!arena.alloc(need[i].first, &oi)) {
      if (++passed > bypass) break;
      continue;
    }
    if (!arena.alloc(need[i].second, &oo)) {
      arena.release(oi, need[i].first);
      if (++passed > bypass) break;
      continue;
    }
    out.push_back(Admitted{i, oi, oo});
  }
  return out;
}

// One entry line of the tile-table cache file written by hrrm_save_tuning:
// {"bytes": .., "dims": .., "r": .., "adaptive": .., "seg_rows": .., ...}.
struct TuningLine {
  int bytes, dims, r, adaptive;
  int32_t seg_rows, nslots, min_group, max_groups, lds_budget, tiered_u8, raw_window, wave_slots;
  int32_t window_rows;
  double ms;
};

// Value of "name": in `line` (a number), or false when the key is absent.
inline bool tuning_field(const char* line, const char* name, double* out) {
  char key[64];
  const size_t n = strlen(name);
  if (n + 4 > sizeof key) return false;
  key[0] = '"';
  memcpy(key + 1, name, n);
  key[n + 1] = '"';
  key[n + 2] = ':';
  key[n + 3] = 0;
  const char* p = strstr(line, key);
  if (!p) return false;
  char* end = nullptr;
  *out = strtod(p + n + 3, &end);
  return end != p + n + 3;
}

// Parses one cache line; false for lines that are not entries or whose values
// lie outside what a launch accepts (slot count, LDS budget, flags).
inline bool parse_tuning_line(const char* line, TuningLine* e, int max_slots, int lds_limit) {
  static const char* const names[14] = {"bytes",      "dims",       "r",          "adaptive",
                                        "seg_rows",   "nslots",     "min_group",  "max_groups",
                                        "lds_budget", "tiered_u8",  "ms",         "raw_window",
                                        "wave_slots", "window_rows"};
  double v[14];
  for (int i = 0; i < 11; ++i)
    if (!tuning_field(line, names[i], &v[i])) return false;
  if (!tuning_field(line, names[11], &v[11])) v[11] = 49;
  if (!tuning_field(line, names[12], &v[12])) v[12] = 0;
  if (!tuning_field(line, names[13], &v[13])) v[13] = 0;
  for (int i = 0; i < 14; ++i)
    if (!(v[i] >= -1e9 && v[i] <= 1e9)) return false;  // also rejects NaN
  *e = TuningLine{(int)v[0],      (int)v[1],      (int)v[2],     (int)v[3],     (int32_t)v[4],
                  (int32_t)v[5],  (int32_t)v[6],  (int32_t)v[7], (int32_t)v[8], (int32_t)v[9],
                  (int32_t)v[11], (int32_t)v[12], (int32_t)v[13], v[10]};
  return (e->bytes == 1 || e->bytes == 2) && (e->dims == 2 || e->dims == 3) && e->r >= 0 &&
         e->r <= (e->dims == 2 ? HRRM_MAX_R_2D : HRRM_MAX_R_3D) &&
         (e->adaptive == 0 || e->adaptive == 1) && e->seg_rows >= 1 && e->nslots >= 0 &&
         e->nslots <= max_slots && e->min_group >= 1 && e->max_groups >= 0 &&
         e->lds_budget >= 16 * 1024 && e->lds_budget <= lds_limit && e->raw_window >= 0 &&
         (e->wave_slots == 0 || e->wave_slots == 1) && e->window_rows >= 0 &&
         e->window_rows <= (1 << 20);
}

}  // namespace hrrm
