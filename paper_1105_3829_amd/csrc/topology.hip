// Adaptive interval-occurrences tree: topology pre-pass (Sec. III-C).
//
// The adaptive tree splits a node's grey-value interval so that both children
// are visited about equally often.  Visits come from value insertions and
// removals (distributed like the input, i.e. its global histogram) and from
// order-statistic descents (distributed like the output, estimated here by the
// global histogram of the running box mean over the same window - the O(1)
// first approximation the paper names - or, for a frame of a sequence, by the
// global histogram of a caller-supplied estimate such as the previous frame's
// median, the paper's suggestion for video).  The two histograms are mixed 1:1 and
// every node is split where the mixed weight of its interval is halved
// (ties to the smaller split).  Where the mixed weight of an interval is zero
// the interval is halved by width, as in the uniform tree.
//
// Node numbering: an internal node with split point s (left child [lo, s-1],
// right child [s, hi]) is entry s-1 of the table - every split point of a tree
// over the integers is used by exactly one node - and the last entry's `split`
// holds the root's index.  The table is built one tree level per launch.
// Below depth 2*bits splits are by width, so the tree is at most 3*bits deep.
#include "hrrm_internal.h"

namespace hrrm {
namespace {

constexpr int kTB = 256;

struct Ws {
  uint32_t* hist_src;
  uint32_t* hist_mean;
  uint64_t* prefix;  // (2^bits + 1) entries
  int4* front[2];    // frontier of the current / next level: lo, hi, parent, side
  uint32_t* ctrl;    // rotating frontier counts
  uint32_t* box[2];  // box-sum planes
};

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

Ws carve(void* base, int bits, int64_t pixels) {
  Ws w;
  char* p = (char*)base;
  const size_t nb = (size_t)1 << bits;
  w.hist_src = (uint32_t*)p;
  p += al(nb * 4);
  w.hist_mean = (uint32_t*)p;
  p += al(nb * 4);
  w.prefix = (uint64_t*)p;
  p += al((nb + 1) * 8);
  w.front[0] = (int4*)p;
  p += al(nb / 2 * sizeof(int4));
  w.front[1] = (int4*)p;
  p += al(nb / 2 * sizeof(int4));
  w.ctrl = (uint32_t*)p;
  p += al(16);
  w.box[0] = (uint32_t*)p;
  p += al((size_t)pixels * 4);
  w.box[1] = (uint32_t*)p;
  return w;
}

__global__ void k_zero(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Workgroup-private histograms: 16-bit bins in LDS (2^bits x 2 bytes, 128 KB
// for 16-bit data), one workgroup per block of at most 65535 values so no bin
// overflows, updated with dword atomics on the bin's half (no carry: a bin
// never exceeds 65535), then the non-zero bins are added to the global
// histogram.  This keeps the device-wide atomics off the hot bins of compact
// distributions.
__device__ __forceinline__ void lds_bin_add(uint32_t* lh, uint32_t v) {
  atomicAdd(&lh[v >> 1], 1u << ((v & 1) * 16));
}

__device__ __forceinline__ void lds_hist_flush(const uint32_t* lh, uint32_t* hist, int nbins) {
  for (int i = threadIdx.x; i < nbins / 2; i += kTB) {
    const uint32_t p = lh[i];
    if (p & 0xffffu) atomicAdd(&hist[2 * i], p & 0xffffu);
    if (p >> 16) atomicAdd(&hist[2 * i + 1], p >> 16);
  }
}

constexpr int64_t kHistBlock = 65535;  // values per workgroup (16-bit bins)

template <typename T>
__global__ __launch_bounds__(kTB) void k_hist(MedianArgs a, uint32_t* hist) {
  extern __shared__ uint32_t lh[];
  const int nbins = 1 << (8 * sizeof(T));
  const T* src = (const T*)a.src;
  for (int i = threadIdx.x; i < nbins / 2; i += kTB) lh[i] = 0;
  __syncthreads();
  const int64_t n = a.w * a.h * a.d;
  const int64_t b0 = (int64_t)blockIdx.x * kHistBlock;
  const int64_t b1 = b0 + kHistBlock < n ? b0 + kHistBlock : n;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kTB) {
    const int64_t x = i % a.w, t = i / a.w, y = t % a.h, z = t / a.h;
    lds_bin_add(lh, src[z * a.sss + y * a.srs + x]);
  }
  __syncthreads();
  lds_hist_flush(lh, hist, nbins);
}

__device__ __forceinline__ int64_t cl(int64_t v, int64_t hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// Clamp-to-edge box sums of width 2r+1 along one axis.  Each thread runs a
// sliding sum over `seg` consecutive positions of one line.  Lines are the
// other two coordinates; consecutive threads take consecutive lines.  In the
// last pass (HIST) floor(sum / n) is histogrammed instead of stored.
template <typename Tin, bool HIST>
__global__ __launch_bounds__(kTB) void k_box(const Tin* in, int64_t s0, int64_t s1, int64_t s2,
                                             int axis, int64_t w, int64_t h, int64_t d, int r,
                                             int seg, uint32_t* out, uint32_t* hist,
                                             uint32_t nwin, int nbins) {
  extern __shared__ uint32_t lh[];
  if (HIST) {  // one workgroup histograms at most 256 * seg <= 65535 means
    for (int i = threadIdx.x; i < nbins / 2; i += kTB) lh[i] = 0;
    __syncthreads();
  }
  const int64_t dims[3] = {w, h, d};
  const int64_t len = dims[axis];
  const int64_t oa = axis == 0 ? 1 : 0, ob = axis == 2 ? 1 : 2;  // the two other axes
  const int64_t na = dims[oa], nbb = dims[ob];
  const int64_t nlines = na * nbb;
  const int64_t nsegs = (len + seg - 1) / seg;
  const int64_t total = nlines * nsegs;
  const int64_t sti[3] = {s0, s1, s2};
  const int64_t sout[3] = {1, w, w * h};
  for (int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * kTB) {
    const int64_t line = t % nlines, sg = t / nlines;
    const int64_t ca = line % na, cb = line / na;
    const int64_t ibase = ca * sti[oa] + cb * sti[ob];
    const int64_t obase = ca * sout[oa] + cb * sout[ob];
    const int64_t st = sti[axis], so = sout[axis];
    const int64_t p0 = sg * seg;
    const int64_t p1 = p0 + seg < len ? p0 + seg : len;
    uint32_t s = 0;
    for (int i = -r; i <= r; ++i) s += (uint32_t)in[ibase + cl(p0 + i, len - 1) * st];
    for (int64_t p = p0; p < p1; ++p) {
      if (p > p0)
        s += (uint32_t)in[ibase + cl(p + r, len - 1) * st] -
             (uint32_t)in[ibase + cl(p - r - 1, len - 1) * st];
      if (HIST)
        lds_bin_add(lh, s / nwin);
      else
        out[obase + p * so] = s;
    }
  }
  if (HIST) {
    __syncthreads();
    lds_hist_flush(lh, hist, nbins);
  }
}

// prefix[v] = sum over u < v of (hist_src[u] + hist_mean[u]); one workgroup.
__global__ __launch_bounds__(1024) void k_prefix(const uint32_t* hs, const uint32_t* hm,
                                                 uint64_t* prefix, int nbins) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  const int chunk = (nbins + 1023) / 1024;
  const int b0 = t * chunk, b1 = b0 + chunk < nbins ? b0 + chunk : nbins;
  uint64_t s = 0;
  for (int i = b0; i < b1; ++i) s += (uint64_t)hs[i] + hm[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint64_t run = t ? part[t - 1] : 0;
  for (int i = b0; i < b1; ++i) {
    prefix[i] = run;
    run += (uint64_t)hs[i] + hm[i];
  }
  if (t == 1023) prefix[nbins] = part[1023];
}

__global__ void k_topo_init(int4* front0, uint32_t* ctrl, int bits) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    front0[0] = make_int4(0, (1 << bits) - 1, -1, 0);
    ctrl[0] = 1;
    ctrl[1] = 0;
    ctrl[2] = 0;
  }
}

__global__ __launch_bounds__(kTB) void k_topo_level(int level, int bits, const uint64_t* P,
                                                    const int4* fin, int4* fout, uint32_t* ctrl,
                                                    TopoNode* topo) {
  const uint32_t n = ctrl[level % 3];
  uint32_t* nout = &ctrl[(level + 1) % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl[(level + 2) % 3] = 0;
  for (uint32_t i = blockIdx.x * kTB + threadIdx.x; i < n; i += gridDim.x * kTB) {
    const int4 f = fin[i];
    const int lo = f.x, hi = f.y;
    const uint64_t plo = P[lo], phi = P[hi + 1];
    int s;
    if (level >= 2 * bits || plo == phi) {
      s = lo + (hi - lo + 1) / 2;
    } else {
      const uint64_t target = plo + phi;  // 2*P[s] >= target: left half reaches half weight
      int a = lo + 1, b = hi;
      while (a < b) {
        const int m = (a + b) >> 1;
        if (2 * P[m] >= target)
          b = m;
        else
          a = m + 1;
      }
      s = a;
      if (2 * P[s] >= target && s > lo + 1) {
        const uint64_t over = 2 * P[s] - target;
        const uint64_t under = target - 2 * P[s - 1];
        if (under <= over) s = s - 1;
      }
    }
    const int idx = s - 1;
    TopoNode nd;
    nd.split = s;
    nd.left = (s - 1 == lo) ? -(lo + 1) : 0;
    nd.right = (s == hi) ? -(s + 1) : 0;
    nd.pad = 0;
    topo[idx] = nd;
    if (f.z < 0)
      topo[(1 << bits) - 1].split = idx;
    else if (f.w == 0)
      topo[f.z].left = idx;
    else
      topo[f.z].right = idx;
    if (s - 1 > lo) fout[atomicAdd(nout, 1u)] = make_int4(lo, s - 1, idx, 0);
    if (hi > s) fout[atomicAdd(nout, 1u)] = make_int4(s, hi, idx, 1);
  }
}

}  // namespace

// Mixed-weight prefix sums, then the table one tree level per launch.
static hipError_t build_levels(const Ws& w, int bits, TopoNode* topo, hipStream_t stream) {
  const size_t nb = (size_t)1 << bits;
  hipLaunchKernelGGL(k_prefix, dim3(1), dim3(1024), 0, stream, w.hist_src, w.hist_mean, w.prefix,
                     (int)nb);
  hipLaunchKernelGGL(k_topo_init, dim3(1), dim3(64), 0, stream, w.front[0], w.ctrl, bits);
  const int lgrid = (int)std::max<size_t>(1, (nb / 2 + kTB - 1) / kTB);
  for (int level = 0; level < 3 * bits; ++level)
    hipLaunchKernelGGL(k_topo_level, dim3(lgrid), dim3(kTB), 0, stream, level, bits, w.prefix,
                       w.front[level & 1], w.front[(level + 1) & 1], w.ctrl, topo);
  return hipGetLastError();
}

hipError_t prime_topology_lds() {
  // the 16-bit histograms: 2^16 16-bit bins
  const size_t hlds = ((size_t)1 << 16) * 2;
  hipError_t e = ensure_dynamic_lds((const void*)k_hist<uint16_t>, hlds);
  if (e == hipSuccess) e = ensure_dynamic_lds((const void*)k_box<uint32_t, true>, hlds);
  return e;
}

size_t topology_workspace_bytes(int bits, int64_t pixels) {
  const size_t nb = (size_t)1 << bits;
  return al(nb * 4) * 2 + al((nb + 1) * 8) + 2 * al(nb / 2 * sizeof(int4)) + al(16) +
         2 * al((size_t)pixels * 4);
}

hipError_t launch_topology(const MedianArgs& a, int bytes, int dims, void* wsp, TopoNode* topo,
                           hipStream_t stream, const void* est, int64_t est_rs) {
  const int bits = 8 * bytes;
  const int64_t pixels = a.w * a.h * a.d;
  Ws w = carve(wsp, bits, pixels);
  const size_t nb = (size_t)1 << bits;
  // the two histograms are adjacent: clear both in one go
  hipLaunchKernelGGL(k_zero, dim3(64), dim3(kTB), 0, stream,
                     w.hist_src, (size_t)(((char*)w.hist_mean - (char*)w.hist_src) / 4 + nb));
  const int hgrid = (int)((pixels + kHistBlock - 1) / kHistBlock);
  const size_t hlds = nb * 2;  // 16-bit bins
  if (bytes == 1) {
    hipLaunchKernelGGL(k_hist<uint8_t>, dim3(hgrid), dim3(kTB), hlds, stream, a, w.hist_src);
  } else {
    hipError_t e = ensure_dynamic_lds((const void*)k_hist<uint16_t>, hlds);
    if (e == hipSuccess) e = ensure_dynamic_lds((const void*)k_box<uint32_t, true>, hlds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hist<uint16_t>, dim3(hgrid), dim3(kTB), hlds, stream, a, w.hist_src);
  }

  if (est) {
    // the estimate's own histogram stands in for the running mean's
    MedianArgs e = a;
    e.src = est;
    e.srs = est_rs;
    e.sss = est_rs * a.h;
    if (bytes == 1)
      hipLaunchKernelGGL(k_hist<uint8_t>, dim3(hgrid), dim3(kTB), hlds, stream, e, w.hist_mean);
    else
      hipLaunchKernelGGL(k_hist<uint16_t>, dim3(hgrid), dim3(kTB), hlds, stream, e, w.hist_mean);
    return build_levels(w, bits, topo, stream);
  }

  // running box mean over the same window: separable clamp-to-edge sums
  const int seg = 64;
  const uint32_t nwin = (uint32_t)((dims == 3 ? (2 * a.r + 1) : 1) * (2 * a.r + 1) * (2 * a.r + 1));
  // the histogramming pass runs one thread per (line, segment) with no grid
  // stride, so each workgroup covers at most 256 * seg values
  auto grid_for = [&](int axis) {
    const int64_t len = axis == 0 ? a.w : (axis == 1 ? a.h : a.d);
    const int64_t lines = pixels / len;
    const int64_t total = lines * ((len + seg - 1) / seg);
    return (int)((total + kTB - 1) / kTB);
  };
  if (bytes == 1)
    hipLaunchKernelGGL((k_box<uint8_t, false>), dim3(grid_for(0)), dim3(kTB), 0, stream,
                       (const uint8_t*)a.src, (int64_t)1, a.srs, a.sss, 0, a.w, a.h, a.d, a.r,
                       seg, w.box[0], nullptr, 1u, 0);
  else
    hipLaunchKernelGGL((k_box<uint16_t, false>), dim3(grid_for(0)), dim3(kTB), 0, stream,
                       (const uint16_t*)a.src, (int64_t)1, a.srs, a.sss, 0, a.w, a.h, a.d, a.r,
                       seg, w.box[0], nullptr, 1u, 0);
  if (dims == 3) {
    hipLaunchKernelGGL((k_box<uint32_t, false>), dim3(grid_for(1)), dim3(kTB), 0, stream,
                       (const uint32_t*)w.box[0], (int64_t)1, a.w, a.w * a.h, 1, a.w, a.h, a.d,
                       a.r, seg, w.box[1], nullptr, 1u, 0);
    hipLaunchKernelGGL((k_box<uint32_t, true>), dim3(grid_for(2)), dim3(kTB), hlds, stream,
                       (const uint32_t*)w.box[1], (int64_t)1, a.w, a.w * a.h, 2, a.w, a.h, a.d,
                       a.r, seg, nullptr, w.hist_mean, nwin, (int)nb);
  } else {
    hipLaunchKernelGGL((k_box<uint32_t, true>), dim3(grid_for(1)), dim3(kTB), hlds, stream,
                       (const uint32_t*)w.box[0], (int64_t)1, a.w, a.w * a.h, 1, a.w, a.h, a.d,
                       a.r, seg, nullptr, w.hist_mean, nwin, (int)nb);
  }
  return build_levels(w, bits, topo, stream);
}

}  // namespace hrrm
