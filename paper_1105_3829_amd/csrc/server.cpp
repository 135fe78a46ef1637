// Continuous-batching request loop (hrrm_server_*).
//
// submit() queues a request on the host.  A worker thread, bound to the
// context's device, repeatedly
//   1. retires finished batches (event query), stamping completion times and
//      returning their input memory;
//   2. admits queued requests in arrival order while the device-memory budget
//      and the in-flight limit allow (a request that does not fit may be
//      passed by at most kBypass later, smaller ones), allocating input and
//      output buffers from one pre-allocated device arena and uploading the
//      input on a copy stream;
//   3. launches everything admitted since the last launch as one batch - one
//      persistent batched launch (or, in the comparison mode, one launch per
//      image) - alternating between two compute streams, so a batch that
//      arrives while another runs starts on the device as soon as workgroups
//      free up.
// Only the bookkeeping shared with the API calls (requests, queue, arena)
// runs under the server's lock; uploads, launches and event queries do not,
// so a submit() never waits behind a large batch being launched.
// Output buffers stay owned by the server until release().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hrrm.h"
#include "hrrm_ctx.h"
#include "host_logic.hpp"

namespace hrrm {

namespace {

constexpr int kBypass = 8;
constexpr int kStreams = 2;

size_t round_up(size_t n) { return Arena::round_up(n); }

enum class St { Queued, Admitted, Done };

struct Item {
  hrrm_request req;
  St st;
  int status;
  double t_submit, t_admit, t_done;
  size_t off_in, off_out, in_bytes, out_bytes;
};

struct Running {
  hipEvent_t ev;
  std::vector<uint64_t> tickets;
};

// An admitted request as the worker needs it outside the lock: its ticket,
// its image in the arena and where its input comes from.
struct Staged {
  uint64_t tk;
  hrrm_image im;
  char* dev_in;  // im.src, writable
  const void* src;
  int64_t src_row_stride;
  size_t in_bytes;
};

}  // namespace

struct Server {
  Context* ctx = nullptr;  // the server's own context (tile table copied from the caller's)
  size_t budget = 0;
  int max_inflight = 0, max_queue = 0;
  int mode = 0;  // 0: persistent batched launch, 1: one launch per image
  char* base = nullptr;
  Arena arena;
  hipStream_t copy = nullptr;
  hipStream_t comp[kStreams] = {nullptr, nullptr};
  int next_stream = 0;
  std::mutex mu;
  // under mu (shared with the API calls)
  std::unordered_map<uint64_t, Item> items;
  std::deque<uint64_t> queue;
  std::deque<uint64_t> finished;  // done tickets not yet reported by drain()
  int inflight = 0;
  // the worker's own (uploads issued, not yet launched; batches on the device)
  std::vector<Staged> staged;
  std::vector<Running> running;
  uint64_t next_ticket = 1;
  std::atomic<bool> stop{false};
  std::thread worker;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  bool step();  // one pass of the loop; true if anything happened
  void finish(const std::vector<uint64_t>& tks, int status, bool release_input);  // under mu
  void loop();
};

static size_t bpp(int dtype) { return dtype == HRRM_U8 ? 1 : 2; }

// Marks the tickets done with `status` at the current time (under mu).
void Server::finish(const std::vector<uint64_t>& tks, int status, bool release_input) {
  const double t = now();
  for (uint64_t tk : tks) {
    auto it = items.find(tk);
    if (it == items.end()) continue;
    Item& r = it->second;
    if (r.status == HRRM_OK) r.status = status;
    r.st = St::Done;
    r.t_done = t;
    if (release_input) arena.release(r.off_in, r.in_bytes);
    finished.push_back(tk);
  }
}

// One pass of the worker.  Only the bookkeeping shared with the API calls
// (items, queue, arena, finished) runs under mu; the event queries, uploads
// and launches do not, so submit() and drain() never wait behind them.
bool Server::step() {
  bool did = false;
  // 1. retire finished batches
  std::vector<uint64_t> done;
  for (size_t i = 0; i < running.size();) {
    if (hipEventQuery(running[i].ev) == hipSuccess) {
      done.insert(done.end(), running[i].tickets.begin(), running[i].tickets.end());
      (void)hipEventDestroy(running[i].ev);
      running.erase(running.begin() + i);
    } else {
      ++i;
    }
  }
  // 2. admission (the rule itself is host_logic.hpp's plan_admission)
  std::vector<Staged> admitted;
  {
    std::lock_guard<std::mutex> g(mu);
    if (!done.empty()) {
      finish(done, HRRM_OK, true);
      did = true;
    }
    if (!queue.empty() && inflight < max_inflight) {
      std::vector<std::pair<size_t, size_t>> need;
      need.reserve(queue.size());
      for (uint64_t tk : queue) {
        const Item& r = items[tk];
        need.emplace_back(r.in_bytes, r.out_bytes);
      }
      const std::vector<Admitted> plan =
          plan_admission(arena, need, max_inflight - inflight, kBypass);
      std::vector<bool> taken(queue.size(), false);
      const double t = now();
      for (const Admitted& p : plan) {
        const uint64_t tk = queue[p.index];
        Item& r = items[tk];
        taken[p.index] = true;
        r.off_in = p.off_in;
        r.off_out = p.off_out;
        r.st = St::Admitted;
        r.t_admit = t;
        ++inflight;
        hrrm_image im{};
        im.src = base + r.off_in;
        im.dst = base + r.off_out;
        im.width = r.req.width;
        im.height = r.req.height;
        im.src_row_stride = r.req.width;
        im.dst_row_stride = r.req.width;
        im.dtype = r.req.dtype;
        im.r = r.req.r;
        admitted.push_back(
            Staged{tk, im, base + r.off_in, r.req.src, r.req.src_row_stride, r.in_bytes});
      }
      if (!plan.empty()) {
        std::deque<uint64_t> rest;
        for (size_t i = 0; i < queue.size(); ++i)
          if (!taken[i]) rest.push_back(queue[i]);
        queue.swap(rest);
        did = true;
      }
    }
  }
  // uploads on the copy stream: packed rows as one linear copy (full link
  // speed from pinned memory); strided rows as a 2-D copy, which the runtime
  // performs far more slowly
  std::vector<uint64_t> failed;
  for (const Staged& a : admitted) {
    const size_t b = bpp(a.im.dtype);
    const hipError_t e =
        a.src_row_stride == a.im.width
            ? hipMemcpyAsync(a.dev_in, a.src, a.in_bytes, hipMemcpyHostToDevice, copy)
            : hipMemcpy2DAsync(a.dev_in, (size_t)a.im.width * b, a.src,
                               (size_t)a.src_row_stride * b, (size_t)a.im.width * b,
                               (size_t)a.im.height, hipMemcpyHostToDevice, copy);
    if (e != hipSuccess)
      failed.push_back(a.tk);  // the request fails; its input buffer is returned at once
    else
      staged.push_back(a);
  }
  if (!failed.empty()) {
    std::lock_guard<std::mutex> g(mu);
    finish(failed, HRRM_EDEVICE, true);
  }
  // 3. launch what was admitted
  if (!staged.empty() && (int)running.size() < kStreams) {
    const int s = next_stream;
    next_stream = (next_stream + 1) % kStreams;
    hipEvent_t up = nullptr, ev = nullptr;
    bool ok = hipEventCreateWithFlags(&up, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
              hipEventRecord(up, copy) == hipSuccess &&
              hipStreamWaitEvent(comp[s], up, 0) == hipSuccess;
    int rc = ok ? HRRM_OK : HRRM_EDEVICE;
    std::vector<hrrm_image> imgs;
    std::vector<uint64_t> tks;
    imgs.reserve(staged.size());
    tks.reserve(staged.size());
    for (const Staged& a : staged) {
      imgs.push_back(a.im);
      tks.push_back(a.tk);
    }
    staged.clear();
    if (rc == HRRM_OK) {
      if (mode == 0) {
        for (size_t i = 0; i < imgs.size() && rc == HRRM_OK; i += hrrm_batch_capacity()) {
          const int n = (int)std::min<size_t>(imgs.size() - i, hrrm_batch_capacity());
          rc = run_batched(ctx, imgs.data() + i, n, comp[s], true);
        }
      } else {
        for (size_t i = 0; i < imgs.size() && rc == HRRM_OK; ++i) {
          const hrrm_image& im = imgs[i];
          rc = run_filter(ctx, im.src, im.dst, im.dtype, im.width, im.height, 1,
                          im.src_row_stride, 0, im.dst_row_stride, 0, im.r,
                          ((int64_t)(2 * im.r + 1) * (2 * im.r + 1) - 1) / 2, 0, HRRM_PLAIN, 2,
                          comp[s], nullptr);
        }
      }
    }
    if (ok && hipEventRecord(ev, comp[s]) != hipSuccess) ok = false;
    if (up) (void)hipEventDestroy(up);
    if (rc != HRRM_OK || !ok) {
      // the batch failed to launch: its requests finish with the error once
      // their uploads are complete
      (void)hipStreamSynchronize(copy);
      (void)hipStreamSynchronize(comp[s]);
      if (ev) (void)hipEventDestroy(ev);
      std::lock_guard<std::mutex> g(mu);
      finish(tks, rc != HRRM_OK ? rc : HRRM_EDEVICE, true);
    } else {
      running.push_back(Running{ev, std::move(tks)});
    }
    did = true;
  }
  return did;
}

void Server::loop() {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    const bool did = step();
    bool idle;
    {
      std::lock_guard<std::mutex> g(mu);
      idle = queue.empty();
    }
    idle = idle && staged.empty() && running.empty();
    if (stop.load() && idle) break;
    if (!did) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

}  // namespace hrrm

using namespace hrrm;

extern "C" {

int hrrm_server_create(hrrm_ctx ctx, size_t device_mem_budget, int32_t max_inflight,
                       int32_t max_queue, uint32_t flags, hrrm_server* out) {
  clear_error();
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!c || !out) return fail(HRRM_EINVAL, "null argument");
  *out = nullptr;
  if (device_mem_budget < (1u << 20) || max_inflight < 1 || max_queue < 1)
    return fail(HRRM_EINVAL, "budget below 1 MiB or non-positive limits");
  if (flags & ~(uint32_t)HRRM_SERVER_PER_IMAGE) return fail(HRRM_EINVAL, "unknown flags");
  Server* s = new (std::nothrow) Server();
  if (!s) return fail(HRRM_ENOMEM, "out of host memory");
  // the worker thread drives its own context, so the caller's stays usable
  s->ctx = new (std::nothrow) Context();
  if (!s->ctx) {
    delete s;
    return fail(HRRM_ENOMEM, "out of host memory");
  }
  s->ctx->device = c->device;
  s->ctx->tuned = c->tuned;
  s->budget = device_mem_budget;
  s->max_inflight = max_inflight;
  s->max_queue = max_queue;
  s->mode = (flags & HRRM_SERVER_PER_IMAGE) ? 1 : 0;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipMalloc((void**)&s->base, device_mem_budget);
  if (e != hipSuccess) {
    delete s->ctx;
    delete s;
    return fail(HRRM_ENOMEM, "server arena of %zu bytes: %s", device_mem_budget,
                hipGetErrorString(e));
  }
  s->arena.reset(device_mem_budget);
  bool ok = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i < kStreams && ok; ++i)
    ok = hipStreamCreateWithFlags(&s->comp[i], hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    for (int i = 0; i < kStreams; ++i)
      if (s->comp[i]) (void)hipStreamDestroy(s->comp[i]);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    (void)hipFree(s->base);
    delete s->ctx;
    delete s;
    return fail(HRRM_EDEVICE, "server streams");
  }
  s->worker = std::thread([s] { s->loop(); });
  *out = reinterpret_cast<hrrm_server>(s);
  return HRRM_OK;
}

int hrrm_server_submit(hrrm_server srv, const hrrm_request* req, uint64_t* ticket) {
  clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s || !req || !ticket) return fail(HRRM_EINVAL, "null argument");
  if (req->dtype != HRRM_U8 && req->dtype != HRRM_U16) return fail(HRRM_EINVAL, "bad dtype");
  if (req->width <= 0 || req->height <= 0 || !req->src || req->src_row_stride < req->width)
    return fail(HRRM_EINVAL, "bad request geometry");
  if (req->r < 0) return fail(HRRM_EINVAL, "negative radius");
  if (req->r > HRRM_MAX_R_2D) return fail(HRRM_EUNSUPPORTED, "radius %d", req->r);
  const size_t n = (size_t)req->width * (size_t)req->height * bpp(req->dtype);
  if (round_up(n) * 2 > s->budget) return fail(HRRM_ENOMEM, "request larger than the budget");
  std::lock_guard<std::mutex> g(s->mu);
  if ((int)s->queue.size() >= s->max_queue) return fail(HRRM_EAGAIN, "queue full");
  Item it{};
  it.req = *req;
  it.st = St::Queued;
  it.status = HRRM_OK;
  it.t_submit = s->now();
  it.in_bytes = n;
  it.out_bytes = n;
  const uint64_t t = s->next_ticket++;
  s->items.emplace(t, it);
  s->queue.push_back(t);
  *ticket = t;
  return HRRM_OK;
}

int hrrm_server_poll(hrrm_server srv, uint64_t ticket, hrrm_result* res) {
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s || !res) return fail(HRRM_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->items.find(ticket);
  if (it == s->items.end()) return fail(HRRM_EINVAL, "unknown ticket");
  const Item& r = it->second;
  if (r.st != St::Done) return HRRM_EAGAIN;
  res->d_dst = s->base + r.off_out;
  res->width = r.req.width;
  res->height = r.req.height;
  res->dtype = r.req.dtype;
  res->status = r.status;
  res->t_submit = r.t_submit;
  res->t_admit = r.t_admit;
  res->t_done = r.t_done;
  return HRRM_OK;
}

int hrrm_server_drain(hrrm_server srv, uint64_t* tickets, hrrm_result* results, int32_t max) {
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s || !tickets || !results || max < 0) return fail(HRRM_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  int n = 0;
  while (n < max && !s->finished.empty()) {
    const uint64_t t = s->finished.front();
    s->finished.pop_front();
    auto it = s->items.find(t);
    if (it == s->items.end()) continue;  // already released after a poll
    const Item& r = it->second;
    tickets[n] = t;
    hrrm_result& res = results[n];
    res.d_dst = s->base + r.off_out;
    res.width = r.req.width;
    res.height = r.req.height;
    res.dtype = r.req.dtype;
    res.status = r.status;
    res.t_submit = r.t_submit;
    res.t_admit = r.t_admit;
    res.t_done = r.t_done;
    ++n;
  }
  return n;
}

int hrrm_server_release(hrrm_server srv, uint64_t ticket) {
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s) return fail(HRRM_EINVAL, "null server");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->items.find(ticket);
  if (it == s->items.end()) return fail(HRRM_EINVAL, "unknown ticket");
  if (it->second.st != St::Done) return fail(HRRM_EAGAIN, "ticket not done");
  s->arena.release(it->second.off_out, it->second.out_bytes);
  --s->inflight;
  s->items.erase(it);
  return HRRM_OK;
}

int hrrm_server_cancel(hrrm_server srv, uint64_t ticket) {
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s) return fail(HRRM_EINVAL, "null server");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->items.find(ticket);
  if (it == s->items.end()) return fail(HRRM_EINVAL, "unknown ticket");
  if (it->second.st != St::Queued) return fail(HRRM_EAGAIN, "already admitted");
  s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
  s->items.erase(it);
  return HRRM_OK;
}

double hrrm_server_now(hrrm_server srv) {
  Server* s = reinterpret_cast<Server*>(srv);
  return s ? s->now() : 0.0;
}

int hrrm_server_destroy(hrrm_server srv) {
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s) return HRRM_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->queue.clear();  // not-yet-admitted requests are dropped
  }
  s->stop = true;
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->ctx->device);
  for (int i = 0; i < kStreams; ++i) (void)hipStreamSynchronize(s->comp[i]);
  (void)hipStreamSynchronize(s->copy);
  delete s->ctx;  // frees the batch state of the server streams
  for (int i = 0; i < kStreams; ++i) (void)hipStreamDestroy(s->comp[i]);
  (void)hipStreamDestroy(s->copy);
  (void)hipFree(s->base);
  delete s;
  return HRRM_OK;
}

}  // extern "C"
