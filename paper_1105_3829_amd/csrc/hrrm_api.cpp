// Host side of the C ABI declared in include/hrrm.h: argument validation,
// contexts and their device workspaces, tile configuration, kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hrrm.h"
#include "hrrm_ctx.h"
#include "hrrm_internal.h"
#include "window_geom.hpp"
#include "host_logic.hpp"

namespace hrrm {

namespace {
thread_local std::string g_err;

// Tile flags of hrrm_rank2d_noalloc: a fixed device array (one copy per GPU,
// held until the process ends).  Host code never uses the array's name as an
// address: its device address on each GPU comes from hipGetSymbolAddress,
// taken once per device when a context is created there.
static __device__ __align__(256) uint32_t scratch[HRRM_NOALLOC_MAX_TILES];
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 256;
uint32_t* g_scratch_ptr[kMaxDevices];
}  // namespace

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int fail_hip(hipError_t e, const char* what) {
  return fail(HRRM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

// Device address of `scratch` on the current device `dev` (looked up once).
int scratch_address(int dev, uint32_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(HRRM_EUNSUPPORTED, "device index %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = (uint32_t*)p;
  }
  *out = g_scratch_ptr[dev];
  return HRRM_OK;
}


const char* last_error() { return g_err.c_str(); }

// ---- kernel attributes ---------------------------------------------------

hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes) {
  struct Entry {
    const void* kernel;
    int device;
    size_t bytes;
  };
  static std::mutex mu;
  static std::vector<Entry> set;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  for (auto& s : set) {
    if (s.kernel == kernel && s.device == dev) {
      if (s.bytes >= bytes) return hipSuccess;
      e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e == hipSuccess) s.bytes = bytes;
      return e;
    }
  }
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) set.push_back({kernel, dev, bytes});
  return e;
}

// ---- tile table ------------------------------------------------------------

TileConfig default_tile(int bytes, int dims, int r, bool adaptive, int64_t w, int64_t h,
                        int64_t d, bool fill_gpu) {
  TileConfig t{};
  t.tiered_u8 = 1;  // the radix-16 tiered kernel is also the faster one for 8-bit data
  t.min_group = 2;
  t.nslots = 0;
  t.lds_budget = 80 * 1024;  // two workgroups per CU
  // 16-bit windows of at most 49 values (r <= 3 in 2-D, r = 1 in 3-D; and
  // below, uniform 2-D r <= 5 and 3-D r = 2) count their deeper tiers from
  // the raw values; 8-bit trees are shallow enough that held subtrees win
  t.raw_window = bytes == 2 ? 49 : 0;
  const int64_t strips = (w + kBlock - 1) / kBlock;
  int64_t rows;
  if (dims == 2) {
    // Measured on MI355X (4096^2 16-bit and 8192^2 8-bit images, r = 1..127):
    // counting a tier for all 64 pixels of a wave at once (matrix cores, or
    // prefix sums past 127-value columns) pays off for more distinct subtrees
    // per wave the wider the window; narrow windows sum per lane.  Small
    // 16-bit windows count their deeper tiers raw and run six workgroups per
    // CU; 8-bit trees run three or four per CU on fewer slots (smooth images
    // need few); other 16-bit windows run two per CU with short segments up
    // to r = 63; from r = 64 smooth images need more slots than 80 KB holds
    // (the churn grows with the segment) and run one workgroup per CU with
    // the whole 160 KB and tall segments (4x faster at r = 100).  Images
    // whose medians change fast along rows (edges, noise) would rather keep
    // more workgroups per CU there, or more slots for 8-bit trees; the
    // autotuner picks per workload.
    if (bytes == 2)
      t.max_groups = r <= 7 ? 0 : r <= 15 ? 1 : r <= 31 ? 4 : 64;
    else
      t.max_groups = r <= 8 ? 0 : 64;
    if (bytes == 2 && adaptive && r >= 10) {
      // adaptive 16-bit trees spread a row's medians over many more deep
      // subtrees than the uniform tree (narrow weight-balanced splits), so
      // from r = 10 they take the whole LDS for slots: C1 r = 15 22.6 ->
      // 10.9 ms, r = 100 142 -> 57 ms
      t.lds_budget = kLdsLimit;
      t.max_groups = r <= 31 ? 1 : 64;
      rows = r <= 31 ? 48 : 16;
    } else if (bytes == 2) {
      if (r >= 64) {
        t.lds_budget = kLdsLimit;
        rows = 128;
      } else if (r <= 5 && !adaptive) {
        // windows of at most 121 values: every deeper tier counted raw, so
        // slot 0 is the only slot in use and six workgroups share a CU
        t.lds_budget = kLdsSixth;
        t.raw_window = (2 * r + 1) * (2 * r + 1);
        rows = r <= 1 ? 16 : 8;
      } else {
        rows = r <= 5 ? 64 : r <= 31 ? 48 : 24;
      }
    } else {
      // 8-bit trees need at most 17 slots: three workgroups per CU, four
      // where no subtree is counted wave-wide (the build without the matrix
      // cores has the registers for it); adaptive trees too (low-key
      // 8192^2 r = 64: 7.8 -> 6.6 ms against 80 KB budgets, r = 100 8.6 ->
      // 7.4)
      t.lds_budget = t.max_groups == 0 ? kLdsQuarter : kLdsThird;
      rows = t.max_groups == 0 ? 128 : 171;
    }
  } else if (!adaptive || r <= 2) {
    // measured on a 512 x 512 x 256 16-bit volume, r = 1..7: 16-bit cubes of
    // up to 125 values count every deeper tier raw at six workgroups per CU
    // (at r = 2 the medians spread over more deep subtrees than even 160 KB
    // of slots hold well); adaptive trees take the same tiles up to r = 2
    // (r = 1 26.9 -> 14.4 ms, r = 2 60.3 -> 32.0) but not at r = 5 (165
    // against 172 ms)
    t.max_groups = r <= 3 ? 0 : 2;
    rows = r == 2 ? 256 : r <= 3 ? 64 : 256;
    if (r <= 2 && bytes == 2) {
      t.lds_budget = kLdsSixth;
      t.raw_window = (2 * r + 1) * (2 * r + 1) * (2 * r + 1);
      rows = 8;
    } else if (r <= 1) {
      t.lds_budget = kLdsThird;
      rows = 16;
    }
  } else {
    // adaptive volumes: more distinct subtrees per row, so shorter segments
    // (fewer rows walking the same slots) and per-lane sums past one group
    const int span = 2 * r + 1;
    t.max_groups = 1;
    rows = std::max<int64_t>(std::max<int64_t>(16, span), (strips * h * d) / 2048);
  }
  // 2-D: the grey-level-window kernel where it measured faster than the
  // tiered kernel (MI355X):
  //   8-bit uniform tree r = 1..24 (low-key 8192^2: r = 1 1.03 against
  //   1.21 ms, r = 16 1.49 against 1.57, r = 24 1.54 against 1.59; uniform
  //   noise 4096^2 r = 2 0.61 against 0.98); past r = 24 the window counts
  //   of a dense grey level overflow their bytes (low-key r = 28: 2.16
  //   against 1.61);
  //   8-bit adaptive r = 1..32 (low-key r = 1 0.80, r = 32 3.5 against the
  //   topology-tree's 6.4 ms; r = 64 9.9 against 7.8);
  //   16-bit uniform tree from r = 4 (X-ray-like 4096^2, 256 grey levels
  //   per column up to r = 7: r = 4 0.93 against 1.44 ms, r = 5 0.69
  //   against 1.79, r = 7 0.59 against 1.38; 128 from r = 8: r = 15 0.42
  //   against 1.41; at r <= 3 a row's medians spread over more than 256
  //   grey levels: r = 3 2.05 against 1.07), and 16-bit adaptive at every r
  //   (r = 5 1.88 against 11 ms)
  t.window_rows = 0;
  if (dims == 2 && r >= 1 &&
      (bytes == 1 ? r <= (adaptive ? 32 : 24) : (adaptive || r >= 4)))
    // segments: 16-bit r <= 16 in 32 rows (C1 r = 15 0.43 against 0.44 ms at
    // 64, r = 10 0.54 against 0.55); longer ones share each build among more
    // rows where a build reads 2r + 1 rows (C1 r = 31 at 64 rows against 32:
    // 0.59 -> 0.57 ms, adaptive 0.49 -> 0.45; r = 50 at 128 against 64:
    // 1.16 -> 1.13, r = 100 2.70 -> 2.50) and for 8-bit windows (low-key
    // 8192^2 at 64 rows against 32: r = 1 1.01 -> 0.99 ms, r = 2 0.78 ->
    // 0.74, r = 4 0.78 -> 0.76, r = 8 0.84 -> 0.80, r = 16 1.08 -> 0.99,
    // r = 24 1.24 -> 1.11)
    t.window_rows = r > 40 ? 128 : (r > 16 || bytes == 1) ? 64 : 32;
  // 16-bit volumes from r = 2: the window kernel over every slice
  // (X-ray-like 512 x 512 x 256 with 1 % impulses, 256 grey levels per
  // column up to r = 3; uniform tree r = 2 7.2 against 12.3 ms, r = 3 6.0
  // against 14.6, r = 5 6.4 against 17.1, r = 7 7.8 against 22.5; adaptive
  // r = 2 7.9 against 32.2, r = 5 6.1 against 166); at r = 1 the medians of
  // 27-value cubes spread wider than a pass covers (40 against 5.4 ms)
  if (dims == 3 && bytes == 2 && r >= 2) t.window_rows = r <= 2 ? 16 : 32;
  // an image filtered on its own keeps at least two tiles per workgroup slot
  // of the GPU (256 CUs, 1 to 6 workgroups each) when it allows it; in a
  // batch the other images fill the GPU
  const int64_t want = 2 * 256 * (int64_t)tiered_per_cu(t.lds_budget, t.max_groups);
  const int64_t fill = (strips * h * d + want - 1) / want;
  if (fill_gpu && strips * ((h + rows - 1) / rows) * d < want)
    rows = std::max<int64_t>(8, std::min(rows, fill));
  rows = std::min<int64_t>(rows, 512);
  t.seg_rows = (int32_t)std::max<int64_t>(1, std::min<int64_t>(rows, h));
  return t;
}

TileConfig Context::tile_for(int bytes, int dims, int r, bool adaptive, int64_t w, int64_t h,
                             int64_t d, bool fill_gpu) const {
  TileConfig t = default_tile(bytes, dims, r, adaptive, w, h, d, fill_gpu);
  for (const auto& e : tuned) {
    if (e.bytes == bytes && e.dims == dims && e.r == r && e.adaptive == (int)adaptive) {
      TileConfig u = e.cfg;
      // a tuned segment height is a target; never exceed the image
      u.seg_rows = (int32_t)std::max<int64_t>(1, std::min<int64_t>(u.seg_rows, h));
      return u;
    }
  }
  return t;
}

// ---- validation --------------------------------------------------------------

int validate(const void* src, const void* dst, int dtype, int64_t w, int64_t h, int64_t d,
             int64_t srs, int64_t sss, int64_t drs, int64_t dss, int r, int dims) {
  const char* why = "";
  const int rc = check_image_args(src, dst, dtype, w, h, d, srs, sss, drs, dss, r, dims, &why);
  if (rc == HRRM_EUNSUPPORTED)
    return fail(rc, "%s (radius %d, at most %d for %d-D)", why, r,
                dims == 2 ? HRRM_MAX_R_2D : HRRM_MAX_R_3D, dims);
  if (rc != HRRM_OK) return fail(rc, "%s", why);
  return HRRM_OK;
}

// Variants each entry point accepts: the full window update exists for 8-bit
// data only (a 16-bit window tree has 65535 nodes per pixel).
int check_variant(int variant, int dtype) {
  if (variant != HRRM_PLAIN && variant != HRRM_ADAPTIVE && variant != HRRM_FULL_UPDATE)
    return fail(HRRM_EINVAL, "unknown variant %d", variant);
  if (variant == HRRM_FULL_UPDATE && dtype == HRRM_U16)
    return fail(HRRM_EUNSUPPORTED, "the full window update is implemented for 8-bit data only");
  return HRRM_OK;
}

// ---- launch ------------------------------------------------------------------

// Launch arguments of the tiered / dense kernels for tile configuration t;
// fails when the tile does not fit one launch or the LDS.
static int tiered_args(const TileConfig& t0, int bytes, int dims, bool adaptive, bool full,
                       const void* src, void* dst, int64_t w, int64_t h, int64_t d, int64_t srs,
                       int64_t sss, int64_t drs, int64_t dss, int r, int64_t rank, int drop,
                       MedianArgs& a, bool& tiered) {
  const int bits = 8 * bytes;
  TileConfig t = t0;
  if (t.seg_rows <= 0) t.seg_rows = 1;
  t.seg_rows = (int32_t)std::min<int64_t>(t.seg_rows, h);
  // the full update needs every node of every column: dense storage
  tiered = !full && (bytes == 2 || t.tiered_u8 != 0);

  a = MedianArgs{};
  a.src = src;
  a.dst = dst;
  a.w = w;
  a.h = h;
  a.d = dims == 3 ? d : 1;
  a.srs = srs;
  a.sss = dims == 3 ? sss : 0;
  a.drs = drs;
  a.dss = dims == 3 ? dss : 0;
  a.rank = rank;
  a.r = r;
  a.bits = bits;
  a.stop = adaptive ? 1 << 30 : bits - drop;
  a.seg_rows = t.seg_rows;
  a.strips = (int32_t)((w + kBlock - 1) / kBlock);
  a.segs = (int32_t)((h + t.seg_rows - 1) / t.seg_rows);
  a.ncols = kBlock + 2 * r + 1;
  a.cp = (a.ncols + 3) & ~3;
  a.min_group = std::max(1, t.min_group);
  a.max_groups = std::max(0, t.max_groups);
  a.raw_window = std::max(0, t.raw_window);
  // window counts on the matrix cores only for 8-bit 2-D windows of 2r + 1
  // <= 127 rows (column counts as signed bytes): the one case where they
  // measured clearly faster than the DPP-scan and per-lane counts (MI355X,
  // tiered kernel, 8-bit low-key 8192^2 r = 16: 1.57 against 1.94 ms,
  // r = 32: 1.63 against 2.30; 16-bit X-ray-like 4096^2 r = 15 to 50 and
  // 16-bit volumes r = 3 to 7 within 0 to 9 %)
  a.mfma = dims == 2 && bytes == 1 && 2 * r + 1 <= 127 ? 1 : 0;
  a.topo = nullptr;
  a.need = nullptr;

  const int64_t grid = (int64_t)a.strips * a.segs * a.d;
  if (grid > 0x7fffffff) return fail(HRRM_EUNSUPPORTED, "image too large for one launch");

  a.wslots = 0;
  a.wpitch = 0;
  if (tiered && t.wave_slots && !adaptive && dims == 2) {
    // wave-private slots: slot 0 shared, the rest of the budget split into
    // per-wave slots of 64 + 2r + 1 columns
    a.nslots = 1;
    a.wpitch = (64 + 2 * r + 1 + 3) & ~3;
    const size_t budget = (size_t)std::min(std::max(t.lds_budget, 16 * 1024), kLdsLimit);
    const size_t base = wps_lds_bytes(r, a.cp, 0, a.wpitch);
    const size_t per = (size_t)kWaves * a.wpitch * 16;
    int ws = budget > base ? (int)((budget - base) / per) : 0;
    if (t.nslots > 0) ws = std::min(ws, t.nslots);
    a.wslots = std::max(1, std::min(ws, 64));
  } else if (tiered) {
    const size_t meta = median_lds_bytes(bytes, adaptive, true, a.ncols, a.cp, 0);
    // one 16-byte tier vector per column, plus (adaptive) the subtree's topology
    const size_t slot_bytes = (size_t)a.cp * 16 + (adaptive ? tiered_topo_bytes(1) : 0);
    const size_t budget = (size_t)std::min(std::max(t.lds_budget, 16 * 1024), kLdsLimit);
    int fit = budget > meta ? (int)((budget - meta) / slot_bytes) : 0;
    int ns = t.nslots > 0 ? t.nslots : fit;
    ns = std::min(ns, std::max(fit, 1));
    ns = std::min(ns, kMaxSlots);
    if (ns < 1) ns = 1;
    a.nslots = ns;
  } else {
    a.nslots = 1;
  }
  const size_t lds = a.wslots > 0 ? wps_lds_bytes(r, a.cp, a.wslots, a.wpitch)
                                  : median_lds_bytes(bytes, adaptive, tiered, a.ncols, a.cp,
                                                     a.nslots);
  if (lds > (size_t)kLdsLimit)
    return fail(HRRM_EUNSUPPORTED, "radius %d needs %zu bytes of LDS per workgroup", r, lds);
  return HRRM_OK;
}

// Arguments of the grey-level-window launch of one 2-D image or 16-bit volume
// (segments of t.window_rows rows) and of the tiered kernel's pass (uniform
// tree) over the tiles the window kernel flags; neither `need` pointer is set.
int window_setup(Context* ctx, const TileConfig& t, const void* src, void* dst, int bytes,
                 int64_t w, int64_t h, int64_t srs, int64_t drs, int r, int64_t rank,
                 bool adaptive, WindowArgs& wa, MedianArgs& fa, bool alone, int dims,
                 int64_t d, int64_t sss, int64_t dss) {
  if (dims == 3 && (bytes != 2 || r > HRRM_MAX_R_3D))
    return fail(HRRM_EUNSUPPORTED, "window kernel volumes: 16-bit, r <= %d", HRRM_MAX_R_3D);
  if (dims != 3) d = 1, sss = 0, dss = 0;
  // rows the window kernel cannot finish are rare and come alone: short
  // fallback tiles
  TileConfig ft = ctx->tile_for(bytes, dims, r, false, w, h, d);
  ft.window_rows = 0;
  ft.seg_rows = 16;
  bool tiered = true;
  int rc = tiered_args(ft, bytes, dims, false, false, src, dst, w, h, d, srs, sss, drs, dss, r,
                       rank, 0, fa, tiered);
  if (rc != HRRM_OK) return rc;
  wa = WindowArgs{};
  wa.src = src;
  wa.dst = dst;
  wa.w = w;
  wa.h = h;
  wa.srs = srs;
  wa.drs = drs;
  wa.d = d;
  wa.sss = sss;
  wa.dss = dss;
  wa.dims = dims;
  wa.rank = rank;
  wa.r = r;
  const int span = 2 * r + 1;
  wa.n = dims == 3 ? span * span * span : span * span;
  // waves the GPU holds at once (segment sizing of an image launched alone;
  // a volume's slices give every launch tiles enough)
  // (volumes: 256 grey levels up to r = 3, r = 3 9.3 -> 6.0 ms; from r = 4
  // the 128-level columns' occupancy wins, r = 4 6.5 against 7.2, r = 5 6.4
  // against 9.6)
  wa.bq = dims == 3 ? (r <= 3 ? 64 : 32) : window_bq(bytes, r, adaptive);
  const int64_t slots = (int64_t)ctx->cu_count() * window_waves_per_cu(bytes, r, wa.bq);
  window_geometry(wa, w, h, t.window_rows, slots, alone && dims == 2, r);
  wa.wave_bytes = (int32_t)window_wave_bytes(r, wa.bq);
  wa.fb_strips = fa.strips;
  wa.fb_rows = fa.seg_rows;
  wa.fb_segs = fa.segs;
  if (window_tile_count(wa) * d > 0x7fffffffLL)
    return fail(HRRM_EUNSUPPORTED, "image too large for one launch");
  return HRRM_OK;
}

// 2-D grey-level-window kernel, then the tiered kernel (uniform tree) over the
// tiles the window kernel flagged.
static int run_window(Context* ctx, const TileConfig& t, const void* src, void* dst, int bytes,
                      int64_t w, int64_t h, int64_t srs, int64_t drs, int r, int64_t rank,
                      bool adaptive, hipStream_t stream, uint32_t* need_buf, int dims = 2,
                      int64_t d = 1, int64_t sss = 0, int64_t dss = 0) {
  WindowArgs wa;
  MedianArgs fa;
  int rc = window_setup(ctx, t, src, dst, bytes, w, h, srs, drs, r, rank, adaptive, wa, fa, true,
                        dims, d, sss, dss);
  if (rc != HRRM_OK) return rc;
  const int64_t tiles = (int64_t)fa.strips * fa.segs * fa.d;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
  if (!need_buf) {
    rc = ctx->ensure_need(tiles, stream, &need_buf);
    if (rc != HRRM_OK) return rc;
  } else {
    // a fixed flag array: its flags start clear only by clearing them here
    if (tiles > HRRM_NOALLOC_MAX_TILES)
      return fail(HRRM_EUNSUPPORTED, "%lld tiles, more than the %d flags of the fixed array",
                  (long long)tiles, HRRM_NOALLOC_MAX_TILES);
    e = launch_clear_flags(need_buf, tiles, stream);
    if (e != hipSuccess) return fail_hip(e, "tile flag clear");
  }
  wa.need = need_buf;
  fa.need = need_buf;
  e = launch_window(wa, bytes, adaptive, stream);
  if (e != hipSuccess) return fail_hip(e, "window kernel launch");
  e = launch_median(fa, bytes, dims, false, true, false, stream);
  if (e != hipSuccess) return fail_hip(e, "median kernel launch");
  return HRRM_OK;
}

int run_filter(Context* ctx, const void* src, void* dst, int dtype, int64_t w, int64_t h,
               int64_t d, int64_t srs, int64_t sss, int64_t drs, int64_t dss, int r,
               int64_t rank, int drop, int variant, int dims, hipStream_t stream,
               const TileConfig* force, const void* est, int64_t est_rs) {
  const int bytes = dtype == HRRM_U8 ? 1 : 2;
  const bool adaptive = variant == HRRM_ADAPTIVE;
  const bool full = variant == HRRM_FULL_UPDATE;  // 8-bit only, checked by the callers
  const TileConfig t = force ? *force : ctx->tile_for(bytes, dims, r, adaptive, w, h, d);
  if (dims == 2 && drop == 0 && !full && est == nullptr && t.window_rows > 0)
    return run_window(ctx, t, src, dst, bytes, w, h, srs, drs, r, rank, adaptive, stream,
                      nullptr);
  if (dims == 3 && bytes == 2 && !full && t.window_rows > 0 && r >= 1)
    return run_window(ctx, t, src, dst, bytes, w, h, srs, drs, r, rank, adaptive, stream,
                      nullptr, 3, d, sss, dss);

  MedianArgs a;
  bool tiered = true;
  int rc = tiered_args(t, bytes, dims, adaptive, full, src, dst, w, h, d, srs, sss, drs, dss, r,
                       rank, drop, a, tiered);
  if (rc != HRRM_OK) return rc;

  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
  if (adaptive) {
    rc = ctx->ensure_topology(bytes, w * h * a.d, stream);
    if (rc != HRRM_OK) return rc;
    a.topo = (const TopoNode*)ctx->topo;
    e = launch_topology(a, bytes, dims, ctx->topo_ws, (TopoNode*)ctx->topo, stream, est, est_rs);
    if (e != hipSuccess) return fail_hip(e, "adaptive topology launch");
  }
  e = launch_median(a, bytes, dims, adaptive, tiered, full, stream);
  if (e != hipSuccess) return fail_hip(e, "median kernel launch");
  return HRRM_OK;
}

// hrrm_rank2d_noalloc: the window kernel with the fixed flag array, or the
// tiered kernel (uniform tree), which uses no device memory of its own.
int run_noalloc(Context* ctx, const void* src, void* dst, int dtype, int64_t w, int64_t h,
                int64_t srs, int64_t drs, int r, int64_t rank, int variant, hipStream_t stream) {
  const int bytes = dtype == HRRM_U8 ? 1 : 2;
  const bool adaptive = variant == HRRM_ADAPTIVE;
  TileConfig t = ctx->tile_for(bytes, 2, r, adaptive, w, h, 1);
  if (adaptive && t.window_rows <= 0) t.window_rows = r <= 24 ? 32 : 64;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
  if (t.window_rows > 0) {
    uint32_t* flags = nullptr;
    const int rc = scratch_address(ctx->device, &flags);
    if (rc != HRRM_OK) return rc;
    return run_window(ctx, t, src, dst, bytes, w, h, srs, drs, r, rank, adaptive, stream, flags);
  }
  MedianArgs a;
  bool tiered = true;
  int rc = tiered_args(t, bytes, 2, false, false, src, dst, w, h, 1, srs, 0, drs, 0, r, rank, 0,
                       a, tiered);
  if (rc != HRRM_OK) return rc;
  e = launch_median(a, bytes, 2, false, tiered, false, stream);
  if (e != hipSuccess) return fail_hip(e, "median kernel launch");
  return HRRM_OK;
}

int Context::cu_count() {
  if (cus <= 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        n <= 0)
      n = 256;
    cus = n;
  }
  return cus;
}

int Context::ensure_need(int64_t tiles, hipStream_t stream, uint32_t** out) {
  NeedBuf* mine = nullptr;
  NeedBuf* shared = nullptr;
  for (auto& b : needs) {
    if (b.stream == stream) mine = &b;
    if (b.stream == nullptr) shared = &b;
  }
  if (mine && mine->count >= (size_t)tiles) {
    *out = mine->p;
    return HRRM_OK;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (stream && hipStreamIsCapturing(stream, &cs) == hipSuccess &&
      cs != hipStreamCaptureStatusNone) {
    if (!mine && shared && shared->count >= (size_t)tiles) {
      *out = shared->p;
      return HRRM_OK;
    }
    return fail(HRRM_ENOMEM, "tile flag buffer too small under stream capture "
                             "(call hrrm_ctx_reserve before capturing)");
  }
  if (!mine) {
    needs.push_back(NeedBuf{stream, nullptr, 0});
    mine = &needs.back();
  }
  if (mine->p) (void)hipFree(mine->p);
  mine->p = nullptr;
  mine->count = 0;
  hipError_t e = hipMalloc(&mine->p, (size_t)tiles * sizeof(uint32_t));
  if (e != hipSuccess) return fail(HRRM_ENOMEM, "tile flag buffer: %s", hipGetErrorString(e));
  // every flag starts clear; the tiered kernel clears each flag it consumes
  e = hipMemsetAsync(mine->p, 0, (size_t)tiles * sizeof(uint32_t), stream);
  if (e != hipSuccess) return fail_hip(e, "tile flag buffer clear");
  if (!stream) {
    e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return fail_hip(e, "tile flag buffer clear");
  }
  mine->count = (size_t)tiles;
  *out = mine->p;
  return HRRM_OK;
}

// ---- context -----------------------------------------------------------------

int Context::ensure_topology(int bytes, int64_t pixels, hipStream_t stream) {
  const int bits = 8 * bytes;
  const size_t need_ws = topology_workspace_bytes(bits, pixels);
  const size_t need_topo = sizeof(TopoNode) << bits;  // nodes + root entry
  if (need_ws <= topo_ws_bytes && need_topo <= topo_bytes) return HRRM_OK;
  // growing allocates (and hipFree waits for the device): not allowed while
  // the stream is being captured into a graph
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (stream && hipStreamIsCapturing(stream, &cs) == hipSuccess &&
      cs != hipStreamCaptureStatusNone)
    return fail(HRRM_ENOMEM, "adaptive workspace too small under stream capture "
                             "(call hrrm_ctx_reserve before capturing)");
  if (need_ws > topo_ws_bytes) {
    if (topo_ws) (void)hipFree(topo_ws);
    topo_ws = nullptr;
    topo_ws_bytes = 0;
    hipError_t e = hipMalloc(&topo_ws, need_ws);
    if (e != hipSuccess) return fail(HRRM_ENOMEM, "topology workspace: %s", hipGetErrorString(e));
    topo_ws_bytes = need_ws;
  }
  if (need_topo > topo_bytes) {
    if (topo) (void)hipFree(topo);
    topo = nullptr;
    topo_bytes = 0;
    hipError_t e = hipMalloc(&topo, need_topo);
    if (e != hipSuccess) return fail(HRRM_ENOMEM, "topology table: %s", hipGetErrorString(e));
    topo_bytes = need_topo;
  }
  return HRRM_OK;
}

Context::~Context() {
  (void)hipSetDevice(device);
  if (topo_ws) (void)hipFree(topo_ws);
  if (topo) (void)hipFree(topo);
  for (auto& b : needs)
    if (b.p) (void)hipFree(b.p);
  release_batch();
}

}  // namespace hrrm

using namespace hrrm;

extern "C" {

const char* hrrm_last_error(void) { return last_error(); }

const char* hrrm_version(void) { return "hrrm-mi355x 0.1 (gfx950)"; }

int hrrm_ctx_create(int device, hrrm_ctx* out) {
  clear_error();
  if (!out) return fail(HRRM_EINVAL, "null output handle");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return fail_hip(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(HRRM_EINVAL, "device %d out of range (%d)", device, n);
  Context* c = new (std::nothrow) Context();
  if (!c) return fail(HRRM_ENOMEM, "out of host memory");
  c->device = device;
  {
    // the fixed flag array's address on this device, once per device
    int prev = 0;
    e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    if (e != hipSuccess) {
      delete c;
      return fail_hip(e, "hipSetDevice");
    }
    uint32_t* p = nullptr;
    const int rc = scratch_address(device, &p);
    (void)hipSetDevice(prev);
    if (rc != HRRM_OK) {
      delete c;
      return rc;
    }
  }
  if (const char* tc = getenv("HRRM_TUNE_CACHE")) {
    if (FILE* f = fopen(tc, "r")) {
      fclose(f);
      (void)load_tuning(c, tc);
    }
  }
  *out = reinterpret_cast<hrrm_ctx>(c);
  return HRRM_OK;
}

int hrrm_ctx_destroy(hrrm_ctx ctx) {
  clear_error();
  delete reinterpret_cast<Context*>(ctx);
  return HRRM_OK;
}

int hrrm_ctx_reserve(hrrm_ctx ctx, hrrm_dtype dtype, int64_t max_pixels, int32_t max_r,
                     hrrm_variant variant) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c) return fail(HRRM_EINVAL, "null context");
  if (dtype != HRRM_U8 && dtype != HRRM_U16) return fail(HRRM_EINVAL, "unknown dtype");
  if (max_pixels < 0 || max_r < 0) return fail(HRRM_EINVAL, "negative size");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
  // every kernel's LDS limit once, so later (captured) calls set no attribute
  e = prime_tiered_lds();
  if (e == hipSuccess) e = prime_dense_lds();
  if (e == hipSuccess) e = prime_topology_lds();
  if (e == hipSuccess) e = prime_window_lds();
  if (e != hipSuccess) return fail_hip(e, "kernel LDS limits");
  {
    // flags of the tiered kernel's tiles for any 2-D image of max_pixels
    // with segments of at least 8 rows (the defaults): ceil(w / 256) *
    // ceil(h / 8) <= P / 2048 + w / 256 + h / 8 + 1
    const int64_t tiles = max_pixels / 2048 + max_pixels / 256 + max_pixels / 8 + 2;
    uint32_t* buf = nullptr;
    const int rc = c->ensure_need(tiles, nullptr, &buf);
    if (rc != HRRM_OK) return rc;
  }
  if (variant == HRRM_ADAPTIVE)
    return c->ensure_topology(dtype == HRRM_U8 ? 1 : 2, max_pixels, nullptr);
  return HRRM_OK;
}

int hrrm_median2d(hrrm_ctx ctx, const void* d_src, void* d_dst, hrrm_dtype dtype, int64_t width,
                  int64_t height, int64_t src_row_stride, int64_t dst_row_stride, int32_t r,
                  hrrm_variant variant, void* hip_stream) {
  return hrrm_rank2d(ctx, d_src, d_dst, dtype, width, height, src_row_stride, dst_row_stride, r,
                     ((int64_t)(2 * r + 1) * (2 * r + 1) - 1) / 2, 0, variant, hip_stream);
}

int hrrm_rank2d(hrrm_ctx ctx, const void* d_src, void* d_dst, hrrm_dtype dtype, int64_t width,
                int64_t height, int64_t src_row_stride, int64_t dst_row_stride, int32_t r,
                int64_t rank, int32_t drop_levels, hrrm_variant variant, void* hip_stream) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c) return fail(HRRM_EINVAL, "null context");
  int rc = check_variant(variant, dtype);
  if (rc != HRRM_OK) return rc;
  rc = validate(d_src, d_dst, dtype, width, height, 1, src_row_stride, 0, dst_row_stride, 0, r, 2);
  if (rc != HRRM_OK) return rc;
  const int64_t n = (int64_t)(2 * r + 1) * (2 * r + 1);
  if (rank < 0 || rank >= n) return fail(HRRM_EINVAL, "rank %lld outside 0..%lld", (long long)rank,
                                         (long long)(n - 1));
  const int bits = dtype == HRRM_U8 ? 8 : 16;
  if (drop_levels < 0 || drop_levels > bits)
    return fail(HRRM_EINVAL, "drop_levels %d outside 0..%d", drop_levels, bits);
  if (drop_levels != 0 && variant == HRRM_ADAPTIVE)
    return fail(HRRM_EINVAL, "reduced precision needs the uniform (PLAIN) tree");
  if (width == 0 || height == 0) return HRRM_OK;
  return run_filter(c, d_src, d_dst, dtype, width, height, 1, src_row_stride, 0, dst_row_stride,
                    0, r, rank, drop_levels, variant, 2, (hipStream_t)hip_stream, nullptr);
}

int hrrm_rank2d_noalloc(hrrm_ctx ctx, const void* d_src, void* d_dst, hrrm_dtype dtype,
                        int64_t width, int64_t height, int64_t src_row_stride,
                        int64_t dst_row_stride, int32_t r, int64_t rank, hrrm_variant variant,
                        void* hip_stream) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c) return fail(HRRM_EINVAL, "null context");
  int rc = check_variant(variant, dtype);
  if (rc != HRRM_OK) return rc;
  if (variant == HRRM_FULL_UPDATE)
    return fail(HRRM_EUNSUPPORTED, "the allocation-free form takes PLAIN or ADAPTIVE");
  rc = validate(d_src, d_dst, dtype, width, height, 1, src_row_stride, 0, dst_row_stride, 0, r, 2);
  if (rc != HRRM_OK) return rc;
  const int64_t n = (int64_t)(2 * r + 1) * (2 * r + 1);
  if (rank < 0 || rank >= n) return fail(HRRM_EINVAL, "rank %lld outside 0..%lld", (long long)rank,
                                         (long long)(n - 1));
  if (width == 0 || height == 0) return HRRM_OK;
  return run_noalloc(c, d_src, d_dst, dtype, width, height, src_row_stride, dst_row_stride, r,
                     rank, variant, (hipStream_t)hip_stream);
}

int hrrm_median2d_video(hrrm_ctx ctx, const void* d_src, void* d_dst, const void* d_estimate,
                        hrrm_dtype dtype, int64_t width, int64_t height, int64_t src_row_stride,
                        int64_t dst_row_stride, int64_t est_row_stride, int32_t r,
                        void* hip_stream) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c) return fail(HRRM_EINVAL, "null context");
  int rc = validate(d_src, d_dst, dtype, width, height, 1, src_row_stride, 0, dst_row_stride, 0,
                    r, 2);
  if (rc != HRRM_OK) return rc;
  if (width == 0 || height == 0) return HRRM_OK;
  if (d_estimate) {
    if (est_row_stride < width) return fail(HRRM_EINVAL, "estimate row stride smaller than width");
    if (dtype == HRRM_U16 && (((uintptr_t)d_estimate) & 1))
      return fail(HRRM_EINVAL, "uint16 estimate not 2-byte aligned");
  }
  return run_filter(c, d_src, d_dst, dtype, width, height, 1, src_row_stride, 0, dst_row_stride,
                    0, r, ((int64_t)(2 * r + 1) * (2 * r + 1) - 1) / 2, 0, HRRM_ADAPTIVE, 2,
                    (hipStream_t)hip_stream, nullptr, d_estimate, est_row_stride);
}

int hrrm_median3d(hrrm_ctx ctx, const void* d_src, void* d_dst, hrrm_dtype dtype, int64_t width,
                  int64_t height, int64_t depth, int64_t src_row_stride, int64_t src_slice_stride,
                  int64_t dst_row_stride, int64_t dst_slice_stride, int32_t r,
                  hrrm_variant variant, void* hip_stream) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c) return fail(HRRM_EINVAL, "null context");
  int rc = check_variant(variant, dtype);
  if (rc != HRRM_OK) return rc;
  rc = validate(d_src, d_dst, dtype, width, height, depth, src_row_stride, src_slice_stride,
                dst_row_stride, dst_slice_stride, r, 3);
  if (rc != HRRM_OK) return rc;
  if (width == 0 || height == 0 || depth == 0) return HRRM_OK;
  const int64_t s = 2 * r + 1;
  return run_filter(c, d_src, d_dst, dtype, width, height, depth, src_row_stride,
                    src_slice_stride, dst_row_stride, dst_slice_stride, r, (s * s * s - 1) / 2, 0,
                    variant, 3, (hipStream_t)hip_stream, nullptr);
}

static bool tile_ok(const hrrm_tile_config* c) {
  return c->seg_rows >= 1 && c->nslots >= 0 && c->nslots <= kMaxSlots && c->min_group >= 1 &&
         c->min_group <= 65 && c->max_groups >= 0 && c->lds_budget >= 16 * 1024 &&
         c->lds_budget <= kLdsLimit && (c->tiered_u8 == 0 || c->tiered_u8 == 1) &&
         c->raw_window >= 0 && (c->wave_slots == 0 || c->wave_slots == 1) &&
         c->window_rows >= 0 && c->window_rows <= (1 << 20);
}

int hrrm_set_tile_config(hrrm_ctx ctx, hrrm_dtype dtype, int32_t dims, int32_t r,
                         hrrm_variant variant, const hrrm_tile_config* cfg) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c) return fail(HRRM_EINVAL, "null context");
  if ((dtype != HRRM_U8 && dtype != HRRM_U16) || (dims != 2 && dims != 3) || r < 0 ||
      (variant != HRRM_PLAIN && variant != HRRM_ADAPTIVE))
    return fail(HRRM_EINVAL, "bad tile key");
  if (cfg && !tile_ok(cfg)) return fail(HRRM_EINVAL, "tile configuration out of range");
  const int bytes = dtype == HRRM_U8 ? 1 : 2;
  const int ad = variant == HRRM_ADAPTIVE;
  auto& v = c->tuned;
  v.erase(std::remove_if(v.begin(), v.end(), [&](const TunedEntry& e) {
            return e.bytes == bytes && e.dims == dims && e.r == r && e.adaptive == ad;
          }), v.end());
  if (cfg) {
    TunedEntry e{bytes, dims, r, ad, TileConfig{cfg->seg_rows, cfg->nslots, cfg->min_group,
                                                cfg->max_groups, cfg->lds_budget, cfg->tiered_u8,
                                                cfg->raw_window, cfg->wave_slots,
                                                cfg->window_rows},
                 0.0};
    v.push_back(e);
  }
  return HRRM_OK;
}

int hrrm_get_tile_config(hrrm_ctx ctx, hrrm_dtype dtype, int32_t dims, int32_t r,
                         hrrm_variant variant, int64_t width, int64_t height, int64_t depth,
                         hrrm_tile_config* out) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c || !out) return fail(HRRM_EINVAL, "null argument");
  if ((dtype != HRRM_U8 && dtype != HRRM_U16) || (dims != 2 && dims != 3) || r < 0)
    return fail(HRRM_EINVAL, "bad tile key");
  const TileConfig t = c->tile_for(dtype == HRRM_U8 ? 1 : 2, dims, r, variant == HRRM_ADAPTIVE,
                                   width, height, dims == 3 ? depth : 1);
  *out = hrrm_tile_config{t.seg_rows, t.nslots, t.min_group, t.max_groups, t.lds_budget,
                          t.tiered_u8, t.raw_window, t.wave_slots, t.window_rows};
  return HRRM_OK;
}

}  // extern "C"
