// Context object behind the opaque hrrm_ctx handle.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "hrrm.h"
#include "hrrm_internal.h"

namespace hrrm {

struct TunedEntry {
  int bytes, dims, r, adaptive;
  TileConfig cfg;
  double ms;
};

// Per-stream state of batched launches: descriptor buffer, work counter and
// the captured graph of the launch.
constexpr int kStages = 4;  // pinned staging copies per stream, used in turn
struct BatchStream {
  hipStream_t stream;
  void* d_buf;                 // work counters, image counts, descriptor regions
  void* h_stage[kStages];      // pinned staging copies of d_buf's upload
  hipEvent_t staged[kStages];  // recorded after each upload; its copy is reused after it
  bool pending[kStages];
  int next;                    // staging copy of the next batch
  hipGraph_t graph;
  hipGraphExec_t exec;
};

struct Context {
  int device = 0;
  int cus = 0;  // compute units of the device (0: not yet queried)
  int cu_count();
  // adaptive topology workspace (histograms, prefix sums, box sums, frontier)
  void* topo_ws = nullptr;
  size_t topo_ws_bytes = 0;
  void* topo = nullptr;  // TopoNode[2^bits], last entry holds the root index
  size_t topo_bytes = 0;
  std::vector<TunedEntry> tuned;
  // flags of the tiered kernel's tiles that the grey-level-window kernel
  // could not finish (all clear between calls), one buffer per stream so that
  // calls running at the same time on different streams do not share flags;
  // stream == nullptr: the buffer hrrm_ctx_reserve sizes, also taken by calls
  // captured on a stream that has no buffer yet
  struct NeedBuf {
    hipStream_t stream;
    uint32_t* p;
    size_t count;
  };
  std::vector<NeedBuf> needs;

  // batched launches (persistent kernel), one entry per stream used
  std::vector<BatchStream> batch;

  // fill_gpu: the image runs on its own, so small images get shorter segments
  TileConfig tile_for(int bytes, int dims, int r, bool adaptive, int64_t w, int64_t h, int64_t d,
                      bool fill_gpu = true) const;
  // grow the adaptive workspace to `pixels` (refused while `stream` is being
  // captured); a grown workspace replaces the old one after hipFree, which
  // waits for the device
  int ensure_topology(int bytes, int64_t pixels, hipStream_t stream);
  // the tile flag buffer of `stream`, grown to `tiles` flags (growing is
  // refused under capture); *out receives it
  int ensure_need(int64_t tiles, hipStream_t stream, uint32_t** out);
  void release_batch();
  BatchStream* batch_for(hipStream_t s);
  ~Context();
};

int fail(int code, const char* fmt, ...);
int fail_hip(hipError_t e, const char* what);
void clear_error();
TileConfig default_tile(int bytes, int dims, int r, bool adaptive, int64_t w, int64_t h, int64_t d,
                        bool fill_gpu = true);
int validate(const void* src, const void* dst, int dtype, int64_t w, int64_t h, int64_t d,
             int64_t srs, int64_t sss, int64_t drs, int64_t dss, int r, int dims);
int load_tuning(Context* c, const char* path);
int save_tuning(const Context* c, const char* path);
int run_batched(Context* ctx, const hrrm_image* images, int count, hipStream_t stream,
                bool use_graph);
// alone: the image has the GPU to itself (segments shortened until it fills
// the GPU, and the launch's last generation of waves in half-height
// segments); in a batch the other images fill it
// (volumes: d slices of slice strides sss / dss, cube windows)
int window_setup(Context* ctx, const TileConfig& t, const void* src, void* dst, int bytes,
                 int64_t w, int64_t h, int64_t srs, int64_t drs, int r, int64_t rank,
                 bool adaptive, WindowArgs& wa, MedianArgs& fa, bool alone, int dims = 2,
                 int64_t d = 1, int64_t sss = 0, int64_t dss = 0);
// est / est_rs: optional estimate image for the adaptive topology (2-D)
int run_filter(Context* ctx, const void* src, void* dst, int dtype, int64_t w, int64_t h,
               int64_t d, int64_t srs, int64_t sss, int64_t drs, int64_t dss, int r,
               int64_t rank, int drop, int variant, int dims, hipStream_t stream,
               const TileConfig* force, const void* est = nullptr, int64_t est_rs = 0);

}  // namespace hrrm
