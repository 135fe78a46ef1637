// Tile autotuner and tile-table cache (hrrm_autotune / hrrm_load_tuning).
//
// For one key (dtype, dims = 2, r, variant) the tuner times candidate tile
// configurations on a sample image - the caller's, or a synthetic one drawn on
// the device - by coordinate descent over the segment height, the LDS budget
// (tier slots and workgroups per CU), the cooperative-group policy, the window
// size below which deeper tiers are counted raw and, for 8-bit data, dense
// versus tiered storage.  Every candidate's output is
// compared with the default configuration's on the device; a candidate that
// differs would be a defect and is never kept.  The best configuration goes
// into the context's tile table (used by every later call, batched launches
// included) and, if asked, into a JSON cache file (one entry per line).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hrrm.h"
#include "hrrm_ctx.h"
#include "hrrm_internal.h"
#include "host_logic.hpp"

namespace hrrm {

namespace {

// Synthetic sample: 8-bit uniform values, or 12-bit values near 2000 (sum of
// four hashed uniforms, roughly normal) plus a smooth ramp - the shape of the
// X-ray-like workload - for 16-bit data.
__global__ void k_fill(void* p, int bytes, int64_t w, int64_t h, uint32_t seed) {
  const int64_t n = w * h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i * 2654435761u ^ seed;
    uint32_t s = 0;
    for (int k = 0; k < 4; ++k) {
      x ^= x >> 15;
      x *= 2246822519u;
      x ^= x >> 13;
      x *= 3266489917u;
      x ^= x >> 16;
      s += x & 0xffu;
    }
    if (bytes == 1) {
      ((uint8_t*)p)[i] = (uint8_t)(x >> 8);
    } else {
      const int64_t xx = i % w, yy = i / w;
      int v = 2000 + ((int)s - 510) + (int)(150 * (xx + yy) / (w + h)) - 75;
      v = v < 0 ? 0 : (v > 4095 ? 4095 : v);
      ((uint16_t*)p)[i] = (uint16_t)v;
    }
  }
}

__global__ void k_diff(const uint8_t* a, const uint8_t* b, size_t n, unsigned int* bad) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    if (a[i] != b[i]) {
      atomicAdd(bad, 1u);
      return;
    }
}

struct Buf {
  void* p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

int save_tuning(const Context* c, const char* path) {
  FILE* f = fopen(path, "w");
  if (!f) return fail(HRRM_EINVAL, "cannot write %s", path);
  fprintf(f, "{\"version\": 1, \"entries\": [\n");
  for (size_t i = 0; i < c->tuned.size(); ++i) {
    const TunedEntry& e = c->tuned[i];
    fprintf(f,
            " {\"bytes\": %d, \"dims\": %d, \"r\": %d, \"adaptive\": %d, \"seg_rows\": %d, "
            "\"nslots\": %d, \"min_group\": %d, \"max_groups\": %d, \"lds_budget\": %d, "
            "\"tiered_u8\": %d, \"raw_window\": %d, \"wave_slots\": %d, \"window_rows\": %d, "
            "\"ms\": %.5f}%s\n",
            e.bytes, e.dims, e.r, e.adaptive, e.cfg.seg_rows, e.cfg.nslots, e.cfg.min_group,
            e.cfg.max_groups, e.cfg.lds_budget, e.cfg.tiered_u8, e.cfg.raw_window,
            e.cfg.wave_slots, e.cfg.window_rows, e.ms, i + 1 < c->tuned.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  return HRRM_OK;
}

int load_tuning(Context* c, const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return fail(HRRM_EINVAL, "cannot read %s", path);
  char line[1024];
  std::vector<TunedEntry> got;
  while (fgets(line, sizeof line, f)) {
    TuningLine t;
    if (!parse_tuning_line(line, &t, kMaxSlots, kLdsLimit)) continue;
    got.push_back(TunedEntry{t.bytes, t.dims, t.r, t.adaptive,
                             TileConfig{t.seg_rows, t.nslots, t.min_group, t.max_groups,
                                        t.lds_budget, t.tiered_u8, t.raw_window, t.wave_slots,
                                        t.window_rows},
                             t.ms});
  }
  fclose(f);
  for (const TunedEntry& e : got) {
    auto& v = c->tuned;
    v.erase(std::remove_if(v.begin(), v.end(), [&](const TunedEntry& o) {
              return o.bytes == e.bytes && o.dims == e.dims && o.r == e.r &&
                     o.adaptive == e.adaptive;
            }), v.end());
    v.push_back(e);
  }
  return HRRM_OK;
}

int autotune(Context* c, const void* d_sample, int dtype, int r, int variant, int64_t w,
             int64_t h, int64_t stride, const char* cache_path, int32_t* best_out) {
  const int bytes = dtype == HRRM_U8 ? 1 : 2;
  const bool adaptive = variant == HRRM_ADAPTIVE;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
  // the caller's sample (if any) must be complete: drain the device first
  if ((e = hipDeviceSynchronize()) != hipSuccess) return fail_hip(e, "hipDeviceSynchronize");
  Buf img, o_ref, o_try, bad;
  const size_t nbytes = (size_t)w * h * bytes;
  if (hipMalloc(&o_ref.p, nbytes) != hipSuccess || hipMalloc(&o_try.p, nbytes) != hipSuccess ||
      hipMalloc(&bad.p, sizeof(unsigned int)) != hipSuccess)
    return fail(HRRM_ENOMEM, "tune buffers");
  hipStream_t s = nullptr;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
    return fail_hip(e, "tune stream");
  const void* src = d_sample;
  int64_t srs = stride;
  if (!src) {
    if ((e = hipMalloc(&img.p, nbytes)) != hipSuccess) {
      (void)hipStreamDestroy(s);
      return fail(HRRM_ENOMEM, "tune sample");
    }
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, img.p, bytes, w, h, 12345u);
    src = img.p;
    srs = w;
  }
  hipEvent_t ea = nullptr, eb = nullptr;
  (void)hipEventCreate(&ea);
  (void)hipEventCreate(&eb);
  const int64_t k0 = ((int64_t)(2 * r + 1) * (2 * r + 1) - 1) / 2;
  auto run = [&](const TileConfig& t, void* out) {
    return run_filter(c, src, out, dtype, w, h, 1, srs, 0, w, 0, r, k0, 0, variant, 2, s, &t);
  };
  auto time_cfg = [&](const TileConfig& t, double* ms) -> int {
    int rc = run(t, o_try.p);  // warm-up (and the output checked below)
    if (rc != HRRM_OK) return rc;
    (void)hipMemsetAsync(bad.p, 0, sizeof(unsigned int), s);
    hipLaunchKernelGGL(k_diff, dim3(1024), dim3(256), 0, s, (const uint8_t*)o_ref.p,
                       (const uint8_t*)o_try.p, nbytes, (unsigned int*)bad.p);
    unsigned int nbad = 0;
    (void)hipMemcpyAsync(&nbad, bad.p, sizeof nbad, hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    if (nbad) return fail(HRRM_EDEVICE, "tile configuration changed the output");
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(ea, s);
      rc = run(t, o_try.p);
      (void)hipEventRecord(eb, s);
      (void)hipEventSynchronize(eb);
      float m = 0.f;
      (void)hipEventElapsedTime(&m, ea, eb);
      best = std::min(best, m);
      if (rc != HRRM_OK) return rc;
    }
    *ms = best;
    return HRRM_OK;
  };
  TileConfig cur = default_tile(bytes, 2, r, adaptive, w, h, 1);
  int rc = run(cur, o_ref.p);
  (void)hipStreamSynchronize(s);
  double cur_ms = 0;
  if (rc == HRRM_OK) rc = time_cfg(cur, &cur_ms);
  int tried = 1;
  if (rc == HRRM_OK) {
    const bool tiered_kernel = bytes == 2 || cur.tiered_u8 != 0;
    std::vector<std::pair<int, std::vector<int>>> axes = {
        {0, {16, 32, 64, 128, 256}},  // seg_rows
        // lds_budget: six, four, three workgroups per CU up to kLdsSixth,
        // kLdsQuarter, kLdsThird (the first two only without wave-wide
        // counts), two up to 80 KB
        {4, {kLdsSixth, kLdsQuarter, kLdsThird, 64 * 1024, 80 * 1024, 112 * 1024, 160 * 1024}},
    };
    if (tiered_kernel || adaptive) axes.push_back({3, {0, 1, 2, 4, 8, 64}});  // max_groups
    else axes.push_back({2, {1, 2, 4, 8}});                               // min_group
    if (bytes == 1) axes.push_back({5, {0, 1}});                          // tiered_u8
    axes.push_back({6, {0, 9, 27, 49, 81}});                              // raw_window
    if (!adaptive) axes.push_back({7, {0, 1}});                           // wave_slots
    axes.push_back({8, {0, 32, 64, 128}});                                // window_rows
    for (int pass = 0; pass < 2; ++pass) {
      for (auto& ax : axes) {
        for (int v : ax.second) {
          TileConfig t = cur;
          int32_t* f[9] = {&t.seg_rows,   &t.nslots,     &t.min_group,  &t.max_groups,
                           &t.lds_budget, &t.tiered_u8,  &t.raw_window, &t.wave_slots,
                           &t.window_rows};
          if (*f[ax.first] == v) continue;
          *f[ax.first] = v;
          if (ax.first == 5 && v == 1 && t.max_groups > 8) t.max_groups = 1;
          double ms = 0;
          ++tried;
          int trc = time_cfg(t, &ms);
          if (trc == HRRM_EDEVICE) {
            rc = trc;
            break;
          }
          if (trc == HRRM_OK && ms < cur_ms * 0.98) {
            cur = t;
            cur_ms = ms;
          }
        }
        if (rc != HRRM_OK) break;
      }
      if (rc != HRRM_OK) break;
    }
  }
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  (void)hipStreamDestroy(s);
  if (rc != HRRM_OK) return rc;
  auto& v = c->tuned;
  v.erase(std::remove_if(v.begin(), v.end(), [&](const TunedEntry& o) {
            return o.bytes == bytes && o.dims == 2 && o.r == r && o.adaptive == (int)adaptive;
          }), v.end());
  v.push_back(TunedEntry{bytes, 2, r, (int)adaptive, cur, cur_ms});
  if (best_out) *best_out = tried;
  if (cache_path) return save_tuning(c, cache_path);
  return HRRM_OK;
}

}  // namespace hrrm

using namespace hrrm;

extern "C" {

int hrrm_autotune(hrrm_ctx ctx, const void* d_sample, hrrm_dtype dtype, int32_t r,
                  hrrm_variant variant, int64_t width, int64_t height, int64_t row_stride,
                  const char* cache_path, int32_t* tried) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c) return fail(HRRM_EINVAL, "null context");
  if ((dtype != HRRM_U8 && dtype != HRRM_U16) || (variant != HRRM_PLAIN && variant != HRRM_ADAPTIVE))
    return fail(HRRM_EINVAL, "bad dtype or variant");
  if (r < 0 || r > HRRM_MAX_R_2D) return fail(HRRM_EINVAL, "radius %d", r);
  if (width <= 0 || height <= 0 || width > (1 << 16) || height > (1 << 16))
    return fail(HRRM_EINVAL, "sample size");
  if (d_sample && row_stride < width) return fail(HRRM_EINVAL, "row stride smaller than width");
  return autotune(c, d_sample, dtype, r, variant, width, height, row_stride, cache_path, tried);
}

int hrrm_load_tuning(hrrm_ctx ctx, const char* cache_path) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c || !cache_path) return fail(HRRM_EINVAL, "null argument");
  return load_tuning(c, cache_path);
}

int hrrm_save_tuning(hrrm_ctx ctx, const char* cache_path) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c || !cache_path) return fail(HRRM_EINVAL, "null argument");
  return save_tuning(c, cache_path);
}

}  // extern "C"
