/*
 * hrrm.h - C ABI of the MI355X (gfx950) hierarchical recursive running median.
 *
 * The operation is the running median (and, more generally, the running k-th
 * order statistic) of Alekseychuk, "Hierarchical Recursive Running Median":
 * for every pixel p of a 2-D image (or voxel of a 3-D volume) the output is the
 * K-th smallest (0-based) of the N = (2r+1)^D input values in the window
 * centred on p (Sec. II, definition of the median; Sec. III, the
 * get_order_statistic procedure and its percentile K).  The median is
 * K = (N-1)/2; N is always odd.  Borders are clamp-to-edge: window positions
 * outside the image take the nearest edge pixel, with multiplicity, so every
 * window holds exactly N values.
 *
 * The result is computed with the paper's method - per-column interval-
 * occurrence trees (Sec. III, Sec. III-A, Sec. III-B) updated recursively as the
 * window moves down one row, window counts built on demand from the column
 * trees, and a descent through the tree one level at a time - in hand-written
 * HIP kernels.  The output is bit-identical to any correct median filter.
 *
 * Conventions shared by every entry point:
 *  - Pixel buffers are DEVICE pointers (hipMalloc / torch CUDA tensors), owned
 *    by the caller.  The library keeps no pointer after the enqueued work ends.
 *  - Strides are in ELEMENTS (as torch.Tensor.stride()); x is fastest.
 *  - Work is enqueued on `hip_stream` (a hipStream_t; NULL = default stream)
 *    and is asynchronous: calls never synchronise the host.
 *  - Arguments are validated on the host before anything is enqueued; a
 *    rejected call enqueues nothing.  Errors are returned as negative status
 *    codes, with a message in hrrm_last_error() (thread-local).  Calls never
 *    throw across the ABI and never abort.
 *  - A zero-sized image is a successful no-op.  r >= image size is valid.
 *  - src and dst must not overlap.
 */
#ifndef HRRM_H
#define HRRM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define HRRM_OK 0
#define HRRM_EINVAL (-1)       /* bad argument (null pointer, bad size, overlap ...) */
#define HRRM_ENOMEM (-2)       /* device memory for a workspace could not be obtained */
#define HRRM_EUNSUPPORTED (-3) /* valid request outside what the library supports */
#define HRRM_EDEVICE (-4)      /* a HIP runtime call failed */
#define HRRM_EAGAIN (-5)       /* try again later (serving queue full / not finished) */

typedef enum { HRRM_U8 = 1, HRRM_U16 = 2 } hrrm_dtype;

/* Tree topology and window-update form.  PLAIN: the uniform
 * interval-occurrences tree (Sec. III), each split halves its interval,
 * height = bit depth, window counts built on demand for the nodes the descent
 * visits.  ADAPTIVE: a tree shaped by an estimate of where the medians lie
 * (Sec. III-C), so that the descent skips the levels above them.  2-D images
 * (8-bit up to r = 32, 16-bit at every r): per strip of 64 columns, a 64-leaf
 * range placed on the previous rows' medians, reached by two short paths
 * ("below" / "above") from the root.  Volumes and wider 8-bit windows: split
 * so that both children are visited about equally often, estimated from the
 * 1:1 mix of the input's global histogram and the global histogram of its
 * running (box) mean; frequent grey values get short paths.  FULL_UPDATE: the uniform tree with the
 * unconditional update of the entire window tree at every pixel (Sec. III:
 * strictly constant work per pixel, one update per node), 8-bit data only
 * (EUNSUPPORTED for 16-bit).  All give identical output. */
typedef enum { HRRM_PLAIN = 0, HRRM_ADAPTIVE = 1, HRRM_FULL_UPDATE = 2 } hrrm_variant;

/* Largest supported radius.  2-D: column counts are bytes (<= 2r+1 <= 255).
 * 3-D: a column holds (2r+1)^2 values, also kept in a byte. */
#define HRRM_MAX_R_2D 127
#define HRRM_MAX_R_3D 7

typedef struct hrrm_ctx_s* hrrm_ctx;

/* Thread-local message for the last failed call on this thread ("" if none). */
const char* hrrm_last_error(void);

/* Library version string. */
const char* hrrm_version(void);

/* Create a context bound to HIP device `device`.  The context owns device
 * workspaces (adaptive-topology histograms and tables) and the tile
 * configuration table; it is not thread-safe (one context per host thread, or
 * external locking).  Adaptive calls (HRRM_ADAPTIVE, hrrm_median2d_video) of
 * one context share its topology workspace: enqueue them on one stream, or
 * order them; other calls of a context may run on any streams concurrently.
 * *out receives the handle. */
int hrrm_ctx_create(int device, hrrm_ctx* out);

/* Destroy a context and free its workspaces.  The caller must make sure no
 * enqueued work of this context is still running.  NULL is a no-op. */
int hrrm_ctx_destroy(hrrm_ctx ctx);

/* Pre-size the workspaces so later calls up to these sizes allocate nothing
 * (required before capturing adaptive calls into a HIP graph: a call that
 * would have to grow a workspace while its stream is being captured fails
 * with ENOMEM), and raise every kernel's LDS limit on the context's device
 * once, so later calls make no function-attribute call either.  max_pixels
 * counts pixels (2-D) or voxels (3-D). */
int hrrm_ctx_reserve(hrrm_ctx ctx, hrrm_dtype dtype, int64_t max_pixels, int32_t max_r,
                     hrrm_variant variant);

/* Running median over (2r+1) x (2r+1) windows (Sec. III).
 *   d_src, d_dst : device buffers of `dtype` elements; row y of the image
 *                  starts at element y * src_row_stride (dst_row_stride).
 *   width, height: image size in pixels (>= 0).
 *   r            : radius, 0 <= r <= HRRM_MAX_R_2D (window 2r+1).
 * Errors: EINVAL (null pointer with non-zero size, negative size or r,
 * stride < width, misaligned u16 pointer, overlapping buffers, unknown dtype or
 * variant), EUNSUPPORTED (r > HRRM_MAX_R_2D; FULL_UPDATE with 16-bit data),
 * ENOMEM, EDEVICE. */
int hrrm_median2d(hrrm_ctx ctx, const void* d_src, void* d_dst, hrrm_dtype dtype, int64_t width,
                  int64_t height, int64_t src_row_stride, int64_t dst_row_stride, int32_t r,
                  hrrm_variant variant, void* hip_stream);

/* Running median over (2r+1)^3 cubes of a volume (Sec. III, closing remark on
 * the N-dimensional extension).  Element (x, y, z) is at
 * z * slice_stride + y * row_stride + x.  0 <= r <= HRRM_MAX_R_3D.
 * Errors as hrrm_median2d, plus EINVAL if a slice stride is smaller than
 * row_stride * height. */
int hrrm_median3d(hrrm_ctx ctx, const void* d_src, void* d_dst, hrrm_dtype dtype, int64_t width,
                  int64_t height, int64_t depth, int64_t src_row_stride, int64_t src_slice_stride,
                  int64_t dst_row_stride, int64_t dst_slice_stride, int32_t r,
                  hrrm_variant variant, void* hip_stream);

/* Running median of one frame of an image sequence with the adaptive tree
 * (Sec. III-C: for video, the median distribution of the previous frame can
 * stand for where the order-statistic descents go).  The topology is built
 * from the 1:1 mix of this frame's global histogram and the global histogram
 * of d_estimate - typically the previous frame's median output, left on the
 * device - instead of the running-mean histogram; d_estimate = NULL falls back
 * to the running mean (first frame).  d_estimate is a width x height image of
 * `dtype` with row stride est_row_stride (elements); it may alias d_dst (it is
 * read completely before the frame's output is written, in stream order).
 * Output is identical to hrrm_median2d.  Errors as hrrm_median2d, plus EINVAL
 * for est_row_stride < width or a misaligned 16-bit estimate. */
int hrrm_median2d_video(hrrm_ctx ctx, const void* d_src, void* d_dst, const void* d_estimate,
                        hrrm_dtype dtype, int64_t width, int64_t height, int64_t src_row_stride,
                        int64_t dst_row_stride, int64_t est_row_stride, int32_t r,
                        void* hip_stream);

/* Running k-th order statistic, 0 <= rank < (2r+1)^2 (Sec. III,
 * get_order_statistic with K = rank; Sec. VI names order statistics other
 * than the median as a use of the same descent).
 * rank = 0 is the running minimum, (2r+1)^2-1 the running maximum.
 * drop_levels (PLAIN only, 0..bit depth) stops the descent that many levels
 * above the leaves and returns the lower bound of the last node reached
 * (Sec. III-D, variable precision): the exact result with its drop_levels low
 * bits cleared, error < 2^drop_levels grey values.  ADAPTIVE requires
 * drop_levels == 0 (its nodes are not aligned blocks). */
int hrrm_rank2d(hrrm_ctx ctx, const void* d_src, void* d_dst, hrrm_dtype dtype, int64_t width,
                int64_t height, int64_t src_row_stride, int64_t dst_row_stride, int32_t r,
                int64_t rank, int32_t drop_levels, hrrm_variant variant, void* hip_stream);

/* ---- Allocation-free form ------------------------------------------------- */

/* Largest number of tile flags hrrm_rank2d_noalloc keeps: one per 256-column x
 * 16-row tile of the image, ceil(width / 256) * ceil(height / 16). */
#define HRRM_NOALLOC_MAX_TILES 65536

/* hrrm_rank2d (drop_levels = 0, PLAIN or ADAPTIVE) for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It calls no hipMalloc, hipFree or other
 * allocating routine.  The grey-level-window kernel's tile flags (the only
 * device memory the 2-D path uses beyond the caller's buffers and LDS) live in
 * a fixed array of HRRM_NOALLOC_MAX_TILES flags per GPU, held from the
 * context's creation until the process ends, and are cleared by a small
 * kernel at the start of every call that uses them.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (different
 * streams or host threads, any context) race and must be ordered by the
 * caller.  ADAPTIVE always takes the window kernel here (the adaptive tiered
 * kernel needs a topology workspace).  Output equals hrrm_rank2d's.
 * Errors as hrrm_rank2d, plus EUNSUPPORTED for an image with more than
 * HRRM_NOALLOC_MAX_TILES tiles or for FULL_UPDATE. */
int hrrm_rank2d_noalloc(hrrm_ctx ctx, const void* d_src, void* d_dst, hrrm_dtype dtype,
                        int64_t width, int64_t height, int64_t src_row_stride,
                        int64_t dst_row_stride, int32_t r, int64_t rank, hrrm_variant variant,
                        void* hip_stream);

/* ---- Batched launch (many uneven images in one persistent kernel) --------- */

/* One image of a batch.  Pointers are device pointers; strides in elements. */
typedef struct {
  const void* src;
  void* dst;
  int64_t width, height;
  int64_t src_row_stride, dst_row_stride;
  int32_t dtype; /* hrrm_dtype */
  int32_t r;
} hrrm_image;

/* Filter `count` independent 2-D images (PLAIN median) with a few launches
 * for the whole batch: images whose tile configuration picks the
 * grey-level-window kernel (r <= 32) run as one multi-image launch per
 * element type (each image's strips in one grid) followed by one pass per
 * image over the tiles that launch flagged; all others run in ONE persistent
 * launch whose workgroups pull tiles of all images from a device work counter.
 * The tile shape of each image comes from the context's tile table (see
 * hrrm_autotune).  `images` is a HOST array; it is copied into device
 * descriptor buffers owned by the context.  The persistent launch is captured
 * once per (context, stream) into a HIP graph and replayed for later batches.
 * Errors: as hrrm_median2d for any image; EINVAL if count < 0 or
 * count > hrrm_batch_capacity(). */
int hrrm_median2d_batched(hrrm_ctx ctx, const hrrm_image* images, int32_t count,
                          void* hip_stream);

/* Largest `count` hrrm_median2d_batched accepts. */
int32_t hrrm_batch_capacity(void);

/* ---- Tile configuration / autotuning ------------------------------------- */

/* Launch shape and strategy of the fused kernel for one (dtype, dims, r,
 * variant).  Every configuration gives bit-identical output; they differ in
 * speed only.
 *   seg_rows   : output rows one workgroup produces (its column trees are built
 *                once per segment: 2r+1 rows, then updated row by row)
 *   nslots     : tier slots per workgroup for trees deeper than one tier
 *                (0 = as many as lds_budget allows)
 *   min_group  : smallest group of lanes sharing a tree node whose window count
 *                is formed cooperatively (prefix sum over the wave); smaller
 *                groups sum their 2r+1 column counters directly
 *   max_groups : cooperative groups per level before the rest count directly
 *   lds_budget : LDS bytes one workgroup may use (caps nslots; sets occupancy)
 *   tiered_u8  : 1 = 8-bit data uses tiered storage (the default), 0 = dense
 *   raw_window : windows of at most this many values ((2r+1)^D) count the
 *                deeper tiers of the tree directly from the window's values
 *                instead of holding them in slots
 *   wave_slots : 1 = (uniform 2-D trees) the workgroup shares only the first
 *                tier's slot; each wave holds its own slots of deeper subtrees
 *                for the 64 + 2r + 1 columns its windows cover (nslots then
 *                caps the slots per wave); 0 = every slot shared
 *   window_rows: > 0 = (2-D full precision, and 16-bit volumes) the
 *                grey-level-window kernel: each wave holds the leaves of 128
 *                (16-bit 2-D r <= 7: 256) consecutive grey levels per column
 *                of a 64-column strip (a volume's column: its rows and
 *                slices) and skips the tree levels above them (Sec. III;
 *                adaptive: placed on the medians, Sec. III-C), strip
 *                segments of window_rows rows; the rows a
 *                strip cannot finish (byte overflow of a leaf count, medians
 *                spread wider than the scanned leaves) are recomputed by the
 *                tiered kernel with the uniform tree's default configuration.
 *                0 = the tiered kernel alone */
typedef struct {
  int32_t seg_rows, nslots, min_group, max_groups, lds_budget, tiered_u8, raw_window;
  int32_t wave_slots, window_rows;
} hrrm_tile_config;

/* Set (cfg != NULL) or clear (cfg == NULL) the context's tile configuration
 * for one key.  EINVAL for out-of-range fields. */
int hrrm_set_tile_config(hrrm_ctx ctx, hrrm_dtype dtype, int32_t dims, int32_t r,
                         hrrm_variant variant, const hrrm_tile_config* cfg);

/* The configuration a call of this shape would use now. */
int hrrm_get_tile_config(hrrm_ctx ctx, hrrm_dtype dtype, int32_t dims, int32_t r,
                         hrrm_variant variant, int64_t width, int64_t height, int64_t depth,
                         hrrm_tile_config* out);

/* Autotune the 2-D tile configuration of one key (dtype, r, variant): time
 * candidate configurations (segment height, LDS budget, cooperative-group
 * policy, 8-bit storage) on a sample image by coordinate descent and keep the
 * fastest in the context's tile table, which every later call (batched
 * launches included) uses.  d_sample: a DEVICE image of width x height with
 * row_stride (elements) to tune on, or NULL for a synthetic sample drawn on
 * the device (uniform 8-bit values; 12-bit X-ray-like values for 16-bit).
 * Every candidate's output is checked against the default configuration's on
 * the device; EDEVICE if one ever differs.  Synchronises the device.  If
 * cache_path is not NULL the whole tile table is written there (JSON, one
 * entry per line).  *tried (may be NULL) receives the number of candidates
 * timed.  A context created while the environment variable HRRM_TUNE_CACHE
 * names a readable file starts from that table. */
int hrrm_autotune(hrrm_ctx ctx, const void* d_sample, hrrm_dtype dtype, int32_t r,
                  hrrm_variant variant, int64_t width, int64_t height, int64_t row_stride,
                  const char* cache_path, int32_t* tried);

/* Merge / write the context's tile table from / to a JSON cache file. */
int hrrm_load_tuning(hrrm_ctx ctx, const char* cache_path);
int hrrm_save_tuning(hrrm_ctx ctx, const char* cache_path);

/* ---- Serving: continuous-batching request loop ---------------------------- */

typedef struct hrrm_server_s* hrrm_server;

typedef struct {
  const void* src;        /* HOST pointer to the input (copied on admission; pinned memory with
                             packed rows, src_row_stride == width, uploads at full link speed) */
  int64_t width, height;  /* pixels */
  int64_t src_row_stride; /* elements */
  int32_t dtype;          /* hrrm_dtype */
  int32_t r;
} hrrm_request;

typedef struct {
  void* d_dst;            /* device buffer with the output (row stride = width), owned by
                             the server until hrrm_server_release */
  int64_t width, height;
  int32_t dtype;
  int32_t status;         /* HRRM_OK, or the error that failed the request */
  double t_submit;        /* seconds on the server clock */
  double t_admit;
  double t_done;
} hrrm_result;

/* Server flags. */
#define HRRM_SERVER_PER_IMAGE 1u /* launch each admitted image on its own (comparison mode)
                                    instead of one persistent batched launch per batch */

/* Start a server on the context's device (the server copies the context's tile
 * table and drives its own context from a worker thread; the caller's context
 * stays usable).  device_mem_budget bytes of device memory are allocated once
 * and hold the inputs and outputs of admitted requests; max_inflight bounds
 * the admitted, unreleased requests; max_queue bounds the host queue of
 * not-yet-admitted requests.  Requests are filtered with the PLAIN median.
 * Errors: EINVAL, ENOMEM (budget not allocatable), EDEVICE. */
int hrrm_server_create(hrrm_ctx ctx, size_t device_mem_budget, int32_t max_inflight,
                       int32_t max_queue, uint32_t flags, hrrm_server* out);

/* Queue a request (non-blocking; the input is read on admission, so it must
 * stay valid until hrrm_server_poll reports the ticket done).  EAGAIN if the
 * queue is full, EINVAL for a malformed request, ENOMEM if it can never fit the
 * memory budget. */
int hrrm_server_submit(hrrm_server srv, const hrrm_request* req, uint64_t* ticket);

/* HRRM_OK with *res filled once the ticket is done; EAGAIN before. */
int hrrm_server_poll(hrrm_server srv, uint64_t ticket, hrrm_result* res);

/* Report up to `max` done tickets not reported before, in completion order:
 * tickets[i] and results[i] are filled; returns the number reported (>= 0).
 * A ticket is reported once (by drain; poll may still be used on it). */
int hrrm_server_drain(hrrm_server srv, uint64_t* tickets, hrrm_result* results, int32_t max);

/* Give the output buffer of a done ticket back to the server. */
int hrrm_server_release(hrrm_server srv, uint64_t ticket);

/* Cancel a queued (not yet admitted) request: OK if cancelled, EAGAIN if it
 * was already admitted. */
int hrrm_server_cancel(hrrm_server srv, uint64_t ticket);

/* Server clock (seconds), the clock of the t_* stamps. */
double hrrm_server_now(hrrm_server srv);

/* Stop the server (waits for admitted work) and free everything it holds. */
int hrrm_server_destroy(hrrm_server srv);

#ifdef __cplusplus
}
#endif

#endif /* HRRM_H */
