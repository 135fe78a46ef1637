// Host side of the persistent batched launch (hrrm_median2d_batched).
//
// Many uneven 2-D images (8- or 16-bit, any radius up to the batch limit) are
// filtered by ONE launch of a persistent kernel whose workgroups pull tiles of
// all images from a device work counter.  Per image the tile shape comes from
// the context's tile table; the LDS of the launch is fixed, so each image gets
// as many tier slots as fit next to its radius-dependent state.
//
// The launch (counter reset + persistent kernel) is captured once per stream
// into a HIP graph and replayed; a batch only uploads its descriptors (into a
// device buffer owned by that stream's entry) before the replay.  The counter
// is reset by a kernel node, not a memset node.
//
// Images whose tile configuration picks the grey-level-window kernel (and
// whose radius fits its two-column build, r <= 32) are not part of the
// persistent launch: they run as one multi-image window launch per element
// type, followed by one tiered pass per image over the tiles the window
// kernel flagged, all before the graph on the same stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "hrrm.h"
#include "hrrm_ctx.h"
#include "hrrm_internal.h"

namespace hrrm {

namespace {
constexpr int kBatchCap = 4096;           // images per batch
// dynamic LDS per workgroup: with the kernel's few static bytes two (heavy
// class) or four (light class) workgroups fit a CU
constexpr size_t kBatchLds = 80 * 1024 - 256;
constexpr size_t kBatchLightLds = kLdsQuarter - 256;
constexpr int kBatchMaxR = 127;
constexpr int kMinPacked = 8;  // small images a persistent launch needs to pay off
}  // namespace

// Device buffer of one stream: the light and heavy classes' 8 work counters at
// bytes 0 and 32, their image counts at bytes 64 and 68, their descriptors in
// two fixed regions (the captured launches keep their pointers).
constexpr size_t kDescOffset = 256;
constexpr size_t kClassBytes = sizeof(BatchImage) * kBatchCap;
// then the window launches' descriptors (both element types, kBatchCap in all)
constexpr size_t kWinOffset = (kDescOffset + 2 * kClassBytes + 255) & ~(size_t)255;
constexpr size_t kBatchBytes = kWinOffset + sizeof(WindowImage) * kBatchCap;

BatchStream* Context::batch_for(hipStream_t s) {
  for (auto& b : batch)
    if (b.stream == s) return &b;
  BatchStream b{};
  b.stream = s;
  bool ok = hipMalloc(&b.d_buf, kBatchBytes) == hipSuccess;
  for (int k = 0; ok && k < kStages; ++k)
    ok = hipHostMalloc(&b.h_stage[k], kBatchBytes, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&b.staged[k], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    if (b.d_buf) (void)hipFree(b.d_buf);
    for (int k = 0; k < kStages; ++k) {
      if (b.h_stage[k]) (void)hipHostFree(b.h_stage[k]);
      if (b.staged[k]) (void)hipEventDestroy(b.staged[k]);
    }
    return nullptr;
  }
  batch.push_back(b);
  return &batch.back();
}

void Context::release_batch() {
  for (auto& b : batch) {
    for (int k = 0; k < kStages; ++k)
      if (b.pending[k]) (void)hipEventSynchronize(b.staged[k]);
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    for (int k = 0; k < kStages; ++k) {
      if (b.staged[k]) (void)hipEventDestroy(b.staged[k]);
      if (b.h_stage[k]) (void)hipHostFree(b.h_stage[k]);
    }
    if (b.d_buf) (void)hipFree(b.d_buf);
  }
  batch.clear();
}

int batched_grid(int device, bool light) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return cus * (light ? 4 : 2);
}

int run_batched(Context* ctx, const hrrm_image* images, int count, hipStream_t stream,
                bool use_graph) {
  // light class: 16-bit images whose windows are counted raw below tier 1
  // (no subtree counted wave-wide, only slot 0 in use); heavy class: the rest
  std::vector<BatchImage> descs, light;
  descs.reserve(count);
  // window-kernel images by element type (u8, u16), with their fallback passes
  std::vector<WindowImage> wins[2];
  std::vector<MedianArgs> fbs[2];
  int win_rmax[2] = {0, 0};
  int64_t need_tiles = 0;
  int64_t tiles = 0;
  // window images per element type: a batch too small for two generations
  // of waves gets shorter segments (its latency is one segment's time)
  int64_t win_rows[2] = {0, 0};
  int win_r[2] = {0, 0};
  int64_t tier_rows = 0;  // the same for the persistent launch (256-column strips)
  // images whose own launch fills the GPU run alone (one launch per image
  // gains nothing from packing them, and loses the single launch's shorter
  // last segments); the rest are packed
  std::vector<char> solo(count, 0);
  int tier_n = 0;
  const int64_t cus = ctx->cu_count();
  for (int i = 0; i < count; ++i) {
    const hrrm_image& im = images[i];
    if ((im.dtype != HRRM_U8 && im.dtype != HRRM_U16) || im.width <= 0 || im.height <= 0 ||
        im.r < 0 || im.r > kBatchMaxR)
      continue;  // (rejected below)
    const int bytes = im.dtype == HRRM_U8 ? 1 : 2;
    const TileConfig t = ctx->tile_for(bytes, 2, im.r, false, im.width, im.height, 1, false);
    if (t.window_rows > 0 && window_bq(bytes, im.r, false) != 32) {
      solo[i] = 1;  // (the multi-image launch holds 128 grey levels per column)
      continue;
    }
    if (t.window_rows > 0 && window_multi_waves(bytes, im.r) > 0) {
      const int64_t own = (im.width + 63) / 64 * ((im.height + t.window_rows - 1) / t.window_rows);
      if (own >= cus * window_waves_per_cu(bytes, im.r, 32)) {
        solo[i] = 1;
        continue;
      }
      win_rows[bytes - 1] += (im.width + 63) / 64 * im.height;
      win_r[bytes - 1] = std::max(win_r[bytes - 1], im.r);
    } else {
      const int64_t seg = std::max(1, t.seg_rows);
      const int64_t own = (im.width + kBlock - 1) / kBlock * ((im.height + seg - 1) / seg);
      if (own >= cus * tiered_per_cu(t.lds_budget, t.max_groups)) {
        solo[i] = 1;
        continue;
      }
      tier_rows += (im.width + kBlock - 1) / kBlock * im.height;
      ++tier_n;
      solo[i] = 2;  // packed unless the batch has too few such images
    }
  }
  // the persistent launch pays for its fixed cost (descriptor upload, two
  // persistent grids) only with several small images: fewer run alone
  // (batches of C4-like requests, 1-2 small images of this class: 0.46 ms
  // against 0.27 ms alone for one)
  for (int i = 0; i < count; ++i) solo[i] = solo[i] == 2 ? (tier_n < kMinPacked ? 1 : 0) : solo[i];
  if (tier_n < kMinPacked) tier_rows = 0;
  std::vector<int> solos;
  // two tiles per workgroup of the persistent launch (two per CU)
  const int64_t tier_seg = std::max<int64_t>(8, tier_rows / (4 * (int64_t)ctx->cu_count()));
  int64_t win_seg[2];
  for (int c = 0; c < 2; ++c) {
    const int64_t slots = (int64_t)ctx->cu_count() * window_waves_per_cu(c + 1, win_r[c], 32);
    win_seg[c] = std::max<int64_t>(8, win_rows[c] / (2 * slots));
  }
  for (int i = 0; i < count; ++i) {
    const hrrm_image& im = images[i];
    int rc = validate(im.src, im.dst, im.dtype, im.width, im.height, 1, im.src_row_stride, 0,
                      im.dst_row_stride, 0, im.r, 2);
    if (rc != HRRM_OK) return fail(rc, "image %d: %s", i, hrrm_last_error());
    if (im.r > kBatchMaxR) return fail(HRRM_EUNSUPPORTED, "image %d: radius %d", i, im.r);
    if (im.width == 0 || im.height == 0) continue;
    if (solo[i]) {
      solos.push_back(i);
      continue;
    }
    const int bytes = im.dtype == HRRM_U8 ? 1 : 2;
    TileConfig t = ctx->tile_for(bytes, 2, im.r, false, im.width, im.height, 1, false);
    if (t.window_rows > 0 && window_multi_waves(bytes, im.r) > 0) {
      t.window_rows = (int32_t)std::min<int64_t>(t.window_rows, win_seg[bytes - 1]);
      WindowImage wi{};
      MedianArgs fa;
      const int64_t n = (int64_t)(2 * im.r + 1) * (2 * im.r + 1);
      int rc = window_setup(ctx, t, im.src, im.dst, bytes, im.width, im.height, im.src_row_stride,
                            im.dst_row_stride, im.r, (n - 1) / 2, false, wi.args, fa, false);
      if (rc != HRRM_OK) return fail(rc, "image %d: %s", i, hrrm_last_error());
      // the flag offset for now; the pointer once the flag buffer is known
      wi.args.need = nullptr;
      fa.need = (uint32_t*)(uintptr_t)need_tiles;
      need_tiles += (int64_t)fa.strips * fa.segs;
      wins[bytes - 1].push_back(wi);
      fbs[bytes - 1].push_back(fa);
      win_rmax[bytes - 1] = std::max(win_rmax[bytes - 1], im.r);
      continue;
    }
    BatchImage b{};
    MedianArgs& a = b.args;
    a.src = im.src;
    a.dst = im.dst;
    a.w = im.width;
    a.h = im.height;
    a.d = 1;
    a.srs = im.src_row_stride;
    a.drs = im.dst_row_stride;
    a.r = im.r;
    a.rank = ((int64_t)(2 * im.r + 1) * (2 * im.r + 1) - 1) / 2;
    a.bits = 8 * bytes;
    a.stop = a.bits;
    // the batch runs two workgroups per CU; a tile tuned for the whole LDS of
    // a CU (wide 16-bit windows) gets short segments instead, as slots churn
    // more the more rows a segment walks
    // (and segments of at most 128 rows: many short images share the GPU)
    // (and, in a batch too small for two tiles per workgroup, shorter still)
    const int64_t seg = std::min<int64_t>(
        tier_seg, (size_t)t.lds_budget > kBatchLds ? (im.r <= 63 ? 24 : 8)
                                                    : std::min<int64_t>(t.seg_rows, 128));
    a.seg_rows = (int32_t)std::max<int64_t>(1, std::min<int64_t>(seg, im.height));
    a.strips = (int32_t)((im.width + kBlock - 1) / kBlock);
    a.segs = (int32_t)((im.height + a.seg_rows - 1) / a.seg_rows);
    a.ncols = kBlock + 2 * im.r + 1;
    a.cp = (a.ncols + 3) & ~3;
    a.min_group = std::max(1, t.min_group);
    a.max_groups = std::max(0, t.max_groups);
    a.raw_window = std::max(0, t.raw_window);
    a.mfma = bytes == 1 && 2 * im.r + 1 <= 127;  // as for a single 2-D launch
    const size_t meta = tiered_meta_bytes(im.r, bytes) + 16;
    const size_t slot_bytes = (size_t)a.cp * 16;
    const int64_t span = 2 * im.r + 1;
    const int ns_light =
        kBatchLightLds > meta ? (int)((kBatchLightLds - meta) / slot_bytes) : 0;
    // (8-bit trees stay heavy: images of mixed content want more slots than
    // the light LDS holds)
    const bool is_light = bytes == 2 && a.max_groups == 0 && ns_light >= 1 &&
                          span * span <= a.raw_window;
    int ns = is_light ? ns_light : kBatchLds > meta ? (int)((kBatchLds - meta) / slot_bytes) : 0;
    if (t.nslots > 0) ns = std::min(ns, t.nslots);
    ns = std::min(ns, kMaxSlots);
    if (ns < 1) return fail(HRRM_EUNSUPPORTED, "image %d: radius %d does not fit a batch", i, im.r);
    a.nslots = ns;
    tiles += (int64_t)a.strips * a.segs;
    if (tiles > 0x7fffffff) return fail(HRRM_EUNSUPPORTED, "batch has too many tiles");
    b.bytes = bytes;
    (is_light ? light : descs).push_back(b);
  }
  // the images that run alone first (their flag buffer use ends, stream-ordered,
  // before the packed window launch takes the same buffer)
  for (int i : solos) {
    const hrrm_image& im = images[i];
    const int rc = run_filter(ctx, im.src, im.dst, im.dtype, im.width, im.height, 1,
                              im.src_row_stride, 0, im.dst_row_stride, 0, im.r,
                              ((int64_t)(2 * im.r + 1) * (2 * im.r + 1) - 1) / 2, 0, HRRM_PLAIN, 2,
                              stream, nullptr);
    if (rc != HRRM_OK) return fail(rc, "image %d: %s", i, hrrm_last_error());
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
  const bool any_win = !wins[0].empty() || !wins[1].empty();
  if (descs.empty() && light.empty() && !any_win) return HRRM_OK;
  uint32_t* need_buf = nullptr;
  int64_t groups[2] = {0, 0};
  if (any_win) {
    int rc = ctx->ensure_need(need_tiles, stream, &need_buf);
    if (rc != HRRM_OK) return rc;
    for (int c = 0; c < 2; ++c) {
      // larger images first: their many workgroups start early, small ones
      // fill the tail
      std::vector<size_t> order(wins[c].size());
      for (size_t k = 0; k < order.size(); ++k) order[k] = k;
      std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
        return wins[c][x].args.w * wins[c][x].args.h > wins[c][y].args.w * wins[c][y].args.h;
      });
      std::vector<WindowImage> sorted;
      sorted.reserve(order.size());
      const int wpg = window_multi_waves(c + 1, win_rmax[c]);
      for (size_t k : order) {
        WindowImage wi = wins[c][k];
        MedianArgs& fa = fbs[c][k];
        fa.need = need_buf + (uintptr_t)fa.need;
        wi.args.need = fa.need;
        groups[c] += (window_tiles(wi.args) + wpg - 1) / wpg;
        wi.group_end = groups[c];
        sorted.push_back(wi);
      }
      wins[c].swap(sorted);
      if (groups[c] > 0x7fffffffLL) return fail(HRRM_EUNSUPPORTED, "batch has too many tiles");
    }
  }
  // per class, longest work first: expensive images (16-bit, larger windows)
  // at the front of every chunk's range shortens the tail of the launch
  for (auto* v : {&light, &descs}) {
    std::stable_sort(v->begin(), v->end(), [](const BatchImage& x, const BatchImage& y) {
      const double cx = (double)x.args.w * x.args.h * (x.bytes == 2 ? 3.0 : 1.0) *
                        (1.0 + x.args.r / 16.0);
      const double cy = (double)y.args.w * y.args.h * (y.bytes == 2 ? 3.0 : 1.0) *
                        (1.0 + y.args.r / 16.0);
      return cx > cy;
    });
    tiles = 0;
    for (auto& d : *v) {
      tiles += (int64_t)d.args.strips * d.args.segs;
      d.tile_end = tiles;
    }
  }
  BatchStream* bs = ctx->batch_for(stream);
  if (!bs) return fail(HRRM_ENOMEM, "batch descriptor buffers");
  // uploaded from the pinned staging copy once the previous upload from it
  // has completed
  char* base = (char*)bs->d_buf;
  uint32_t* d_counter[2] = {(uint32_t*)base, (uint32_t*)(base + 32)};
  int32_t* d_hdr[2] = {(int32_t*)(base + 64), (int32_t*)(base + 68)};
  const BatchImage* d_imgs[2] = {(const BatchImage*)(base + kDescOffset),
                                 (const BatchImage*)(base + kDescOffset + kClassBytes)};
  // the staging copies are used in turn, so the host waits only for the
  // upload of kStages batches ago on this stream (a wait for the last one
  // would wait for everything enqueued before it)
  const int sk = bs->next;
  bs->next = (bs->next + 1) % kStages;
  if (bs->pending[sk]) {
    e = hipEventSynchronize(bs->staged[sk]);
    if (e != hipSuccess) return fail_hip(e, "batch staging wait");
    bs->pending[sk] = false;
  }
  const int32_t n[2] = {(int32_t)light.size(), (int32_t)descs.size()};
  char* stage = (char*)bs->h_stage[sk];
  std::memcpy(stage + 64, n, sizeof n);
  std::memcpy(stage + kDescOffset, light.data(), sizeof(BatchImage) * light.size());
  std::memcpy(stage + kDescOffset + kClassBytes, descs.data(), sizeof(BatchImage) * descs.size());
  std::memcpy(stage + kWinOffset, wins[0].data(), sizeof(WindowImage) * wins[0].size());
  std::memcpy(stage + kWinOffset + sizeof(WindowImage) * wins[0].size(), wins[1].data(),
              sizeof(WindowImage) * wins[1].size());
  e = hipMemcpyAsync(base + 64, stage + 64, kDescOffset - 64 + sizeof(BatchImage) * light.size(),
                     hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && !descs.empty())
    e = hipMemcpyAsync(base + kDescOffset + kClassBytes, stage + kDescOffset + kClassBytes,
                       sizeof(BatchImage) * descs.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && any_win)
    e = hipMemcpyAsync(base + kWinOffset, stage + kWinOffset,
                       sizeof(WindowImage) * (wins[0].size() + wins[1].size()),
                       hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return fail_hip(e, "batch descriptor upload");
  e = hipEventRecord(bs->staged[sk], stream);
  if (e != hipSuccess) return fail_hip(e, "batch staging event");
  bs->pending[sk] = true;
  if (any_win) {
    const WindowImage* d_win = (const WindowImage*)(base + kWinOffset);
    for (int c = 1; c >= 0; --c) {  // 16-bit images first: the longer work
      const WindowImage* d = d_win + (c == 1 ? wins[0].size() : 0);
      e = launch_window_multi(d, (int)wins[c].size(), groups[c], c + 1, win_rmax[c], stream);
      if (e != hipSuccess) return fail_hip(e, "window kernel launch (batch)");
    }
    for (int c = 1; c >= 0; --c)
      for (const MedianArgs& fa : fbs[c]) {
        e = launch_median(fa, c + 1, 2, false, true, false, stream);
        if (e != hipSuccess) return fail_hip(e, "median kernel launch (batch fallback)");
      }
    if (descs.empty() && light.empty()) return HRRM_OK;
  }
  const size_t lds[2] = {kBatchLightLds, kBatchLds};
  const int grid[2] = {batched_grid(ctx->device, true), batched_grid(ctx->device, false)};
  // both launches run every time (an empty class ends at once), so the
  // captured graph fits every batch
  auto launch_both = [&]() -> hipError_t {
    for (int c = 0; c < 2; ++c) {
      hipError_t le = launch_batched(d_imgs[c], d_hdr[c], d_counter[c], grid[c], lds[c], c == 0,
                                     stream);
      if (le != hipSuccess) return le;
    }
    return hipSuccess;
  };
  auto prepare_both = [&]() -> hipError_t {
    hipError_t pe = launch_batched_prepare(lds[0], true);
    return pe != hipSuccess ? pe : launch_batched_prepare(lds[1], false);
  };
  if (!use_graph || stream == nullptr) {
    e = prepare_both();
    if (e != hipSuccess) return fail_hip(e, "batched kernel attribute");
    e = launch_both();
    if (e != hipSuccess) return fail_hip(e, "batched launch");
    return HRRM_OK;
  }
  if (!bs->exec) {
    // configure the kernels once outside capture, then capture the launches
    e = prepare_both();
    if (e != hipSuccess) return fail_hip(e, "batched kernel attribute");
    e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail_hip(e, "hipStreamBeginCapture");
    hipError_t le = launch_both();
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(stream, &g);
    if (le != hipSuccess) return fail_hip(le, "batched launch (capture)");
    if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail_hip(e, "hipGraphInstantiate");
    }
    bs->graph = g;
    bs->exec = x;
  }
  e = hipGraphLaunch(bs->exec, stream);
  if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
  return HRRM_OK;
}

}  // namespace hrrm

using namespace hrrm;

extern "C" {

int32_t hrrm_batch_capacity(void) { return kBatchCap; }

int hrrm_median2d_batched(hrrm_ctx ctx, const hrrm_image* images, int32_t count,
                          void* hip_stream) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c) return fail(HRRM_EINVAL, "null context");
  if (count < 0 || count > kBatchCap)
    return fail(HRRM_EINVAL, "batch count %d outside 0..%d", count, kBatchCap);
  if (count > 0 && !images) return fail(HRRM_EINVAL, "null image array");
  return run_batched(c, images, count, (hipStream_t)hip_stream, true);
}

}  // extern "C"
