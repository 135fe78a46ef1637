// Context object behind the opaque hrrm_ctx handle.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "hrrm_internal.h"

namespace hrrm {

struct TunedEntry {
  int bytes, dims, r, adaptive;
  TileConfig cfg;
  double ms;
};

struct Context {
  int device = 0;
  // adaptive topology workspace (histograms, prefix sums, box sums, frontier)
  void* topo_ws = nullptr;
  size_t topo_ws_bytes = 0;
  void* topo = nullptr;  // TopoNode[2^bits], last entry holds the root index
  size_t topo_bytes = 0;
  bool capture_locked = false;
  std::vector<TunedEntry> tuned;

  // batched launches (persistent kernel)
  void* batch_desc = nullptr;   // device descriptor ring
  void* batch_host = nullptr;   // pinned staging copy
  void* batch_ctrl = nullptr;   // device work counters
  int batch_cap = 0;
  hipGraphExec_t batch_exec = nullptr;
  hipGraph_t batch_graph = nullptr;
  hipStream_t batch_stream = nullptr;
  int batch_grid = 0;

  TileConfig tile_for(int bytes, int dims, int r, bool adaptive, int64_t w, int64_t h,
                      int64_t d) const;
  int ensure_topology(int bytes, int64_t pixels);
  void release_batch();
  ~Context();
};

int fail(int code, const char* fmt, ...);
int fail_hip(hipError_t e, const char* what);
void clear_error();
TileConfig default_tile(int bytes, int dims, int r, bool adaptive, int64_t w, int64_t h, int64_t d);
int validate(const void* src, const void* dst, int dtype, int64_t w, int64_t h, int64_t d,
             int64_t srs, int64_t sss, int64_t drs, int64_t dss, int r, int dims);
int run_filter(Context* ctx, const void* src, void* dst, int dtype, int64_t w, int64_t h,
               int64_t d, int64_t srs, int64_t sss, int64_t drs, int64_t dss, int r,
               int64_t rank, int drop, int variant, int dims, hipStream_t stream,
               const TileConfig* force);

}  // namespace hrrm
