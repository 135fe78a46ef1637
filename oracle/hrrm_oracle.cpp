// Brute-force CPU oracle for the running median / running order-statistic filter.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no code, header, table or helper with the
// HIP path.
//
// What it computes (Alekseychuk, "Hierarchical Recursive Running Median",
// Sec. II, definition of the median and the sort/select baselines):
//   out[p] = the K-th smallest (0-based) element of the multiset
//            { in[clamp(p + o)] : o in [-r, r]^D },     N = (2r+1)^D values,
//   with the median at K = (N-1)/2.  N is always odd, so the median is the
//   unique middle element; "half of the elements are <= m" and "the element at
//   position n^2/2 after sorting" name the same value.
//   Borders replicate the edge pixel (clamp-to-edge), with multiplicity, so
//   every window holds exactly N values.
// How: gather the N clamped values of each window into a private buffer and
// select the K-th with std::nth_element (the Quickselect baseline of Sec. II).
// No histogram, no recursion, no reuse between neighbouring windows.
//
// Reduced precision (Sec. III-D): a descent stopped b levels above the leaves
// of the uniform tree returns the lower bound of the node holding the K-th
// value.  On the uniform tree that node is the aligned block of 2^b grey
// values containing it, so the result is the exact order statistic with its
// b low bits cleared; the drop_bits argument of oracle_rank2d does exactly that.
//
// Threshold decomposition (8-bit images only, oracle_rank2d_u8_thresholds):
// a second, independent route to the same rank-K filter, from the stacking
// property of rank filters: the K-th smallest value m of a window satisfies
// m >= t exactly when at least N - K window values are >= t.  So
//   out = sum over t = 1..255 of [ #{window values >= t} >= N - K ],
// and each count is a plain box sum of the binary image [in >= t], taken from
// a summed-area table of the clamp-extended image.  The cost does not grow
// with r, which makes full-size 8192 x 8192 references at r = 100 affordable.
//
// Parity pinning lives in tests/test_oracle.py (brute-force counting on tiny
// inputs, certificates, invariances, threshold decomposition).
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

inline int64_t clampi(int64_t v, int64_t lo, int64_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Runs body(i) for i in [0, n) on `nthreads` threads, rows handed out one by one.
template <class F>
void parallel_rows(int64_t n, int nthreads, F body) {
  if (nthreads <= 0) {
    unsigned hc = std::thread::hardware_concurrency();
    nthreads = hc ? (int)hc : 1;
  }
  if (nthreads > n) nthreads = (int)(n > 0 ? n : 1);
  std::atomic<int64_t> next(0);
  auto worker = [&]() {
    for (;;) {
      int64_t i = next.fetch_add(1);
      if (i >= n) break;
      body(i);
    }
  };
  if (nthreads == 1) {
    worker();
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
}

// One 2-D window: gather (2r+1)^2 clamped values into buf, select rank k.
template <typename T>
T select2d(const T* src, int64_t w, int64_t h, int64_t stride, int r, int64_t k,
           int64_t x, int64_t y, std::vector<T>& buf) {
  size_t n = 0;
  for (int64_t dy = -r; dy <= r; ++dy) {
    const int64_t yy = clampi(y + dy, 0, h - 1);
    for (int64_t dx = -r; dx <= r; ++dx) {
      const int64_t xx = clampi(x + dx, 0, w - 1);
      buf[n++] = src[yy * stride + xx];
    }
  }
  std::nth_element(buf.begin(), buf.begin() + k, buf.begin() + n);
  return buf[k];
}

template <typename T>
T select3d(const T* src, int64_t w, int64_t h, int64_t d, int64_t rs, int64_t ss,
           int r, int64_t k, int64_t x, int64_t y, int64_t z, std::vector<T>& buf) {
  size_t n = 0;
  for (int64_t dz = -r; dz <= r; ++dz) {
    const int64_t zz = clampi(z + dz, 0, d - 1);
    for (int64_t dy = -r; dy <= r; ++dy) {
      const int64_t yy = clampi(y + dy, 0, h - 1);
      for (int64_t dx = -r; dx <= r; ++dx) {
        const int64_t xx = clampi(x + dx, 0, w - 1);
        buf[n++] = src[zz * ss + yy * rs + xx];
      }
    }
  }
  std::nth_element(buf.begin(), buf.begin() + k, buf.begin() + n);
  return buf[k];
}

template <typename T>
void rank2d(const T* src, T* dst, int64_t w, int64_t h, int64_t ss, int64_t ds, int r,
            int64_t k, int drop_bits, int nthreads) {
  const int64_t n = (2 * (int64_t)r + 1) * (2 * (int64_t)r + 1);
  const T mask = (T)~((1u << drop_bits) - 1u);  // drop_bits <= 16
  parallel_rows(h, nthreads, [&](int64_t y) {
    std::vector<T> buf((size_t)n);
    for (int64_t x = 0; x < w; ++x)
      dst[y * ds + x] = (T)(select2d(src, w, h, ss, r, k, x, y, buf) & mask);
  });
}

template <typename T>
void rank3d(const T* src, T* dst, int64_t w, int64_t h, int64_t d, int64_t srs, int64_t sss,
            int64_t drs, int64_t dss, int r, int64_t k, int nthreads) {
  const int64_t side = 2 * (int64_t)r + 1;
  const int64_t n = side * side * side;
  parallel_rows(h * d, nthreads, [&](int64_t row) {
    const int64_t z = row / h, y = row % h;
    std::vector<T> buf((size_t)n);
    for (int64_t x = 0; x < w; ++x)
      dst[z * dss + y * drs + x] = select3d(src, w, h, d, srs, sss, r, k, x, y, z, buf);
  });
}

template <typename T>
void rank2d_at(const T* src, int64_t w, int64_t h, int64_t ss, int r, int64_t k,
               const int64_t* xs, const int64_t* ys, int64_t m, T* out, int nthreads) {
  const int64_t n = (2 * (int64_t)r + 1) * (2 * (int64_t)r + 1);
  const int64_t chunk = 256;
  parallel_rows((m + chunk - 1) / chunk, nthreads, [&](int64_t c) {
    std::vector<T> buf((size_t)n);
    const int64_t e = std::min(m, (c + 1) * chunk);
    for (int64_t i = c * chunk; i < e; ++i)
      out[i] = select2d(src, w, h, ss, r, k, xs[i], ys[i], buf);
  });
}

template <typename T>
void rank3d_at(const T* src, int64_t w, int64_t h, int64_t d, int64_t rs, int64_t ss, int r,
               int64_t k, const int64_t* xs, const int64_t* ys, const int64_t* zs, int64_t m,
               T* out, int nthreads) {
  const int64_t side = 2 * (int64_t)r + 1;
  const int64_t n = side * side * side;
  const int64_t chunk = 64;
  parallel_rows((m + chunk - 1) / chunk, nthreads, [&](int64_t c) {
    std::vector<T> buf((size_t)n);
    const int64_t e = std::min(m, (c + 1) * chunk);
    for (int64_t i = c * chunk; i < e; ++i)
      out[i] = select3d(src, w, h, d, rs, ss, r, k, xs[i], ys[i], zs[i], buf);
  });
}

// Rank-k filter of an 8-bit image by threshold decomposition (see the file
// comment).  Rows are handled in bands of `band` rows; each band builds, per
// threshold, the summed-area table of its clamp-extended rows and columns.
void rank2d_u8_thresholds(const uint8_t* src, uint8_t* dst, int64_t w, int64_t h, int64_t ss,
                          int64_t ds, int r, int64_t k, int nthreads) {
  const int64_t side = 2 * (int64_t)r + 1;
  const int64_t need = side * side - k;  // #{>= t} needed for out >= t
  const int64_t band = 256;
  const int64_t nb = (h + band - 1) / band;
  parallel_rows(nb, nthreads, [&](int64_t b) {
    const int64_t y0 = b * band, y1 = std::min(h, y0 + band);
    const int64_t eh = (y1 - y0) + 2 * r, ew = w + 2 * r;  // clamp-extended band
    std::vector<uint8_t> ext((size_t)(eh * ew));
    for (int64_t i = 0; i < eh; ++i) {
      const int64_t yy = clampi(y0 - r + i, 0, h - 1);
      for (int64_t j = 0; j < ew; ++j) ext[i * ew + j] = src[yy * ss + clampi(j - r, 0, w - 1)];
    }
    // sat[(i)(ew+1) + j] = number of ext values >= t in rows < i, columns < j
    std::vector<int32_t> sat((size_t)((eh + 1) * (ew + 1)));
    std::vector<int32_t> acc((size_t)((y1 - y0) * w), 0);
    for (int t = 1; t <= 255; ++t) {
      for (int64_t j = 0; j <= ew; ++j) sat[j] = 0;
      for (int64_t i = 0; i < eh; ++i) {
        int32_t row = 0;
        sat[(i + 1) * (ew + 1)] = 0;
        for (int64_t j = 0; j < ew; ++j) {
          row += ext[i * ew + j] >= t ? 1 : 0;
          sat[(i + 1) * (ew + 1) + j + 1] = sat[i * (ew + 1) + j + 1] + row;
        }
      }
      bool any = false;
      for (int64_t y = 0; y < y1 - y0; ++y)
        for (int64_t x = 0; x < w; ++x) {
          // window rows y .. y + 2r, columns x .. x + 2r of the extended band
          const int64_t cnt = (int64_t)sat[(y + side) * (ew + 1) + x + side] -
                              sat[y * (ew + 1) + x + side] - sat[(y + side) * (ew + 1) + x] +
                              sat[y * (ew + 1) + x];
          if (cnt >= need) {
            ++acc[y * w + x];
            any = true;
          }
        }
      if (!any) break;  // counts only fall as t grows
    }
    for (int64_t y = 0; y < y1 - y0; ++y)
      for (int64_t x = 0; x < w; ++x) dst[(y0 + y) * ds + x] = (uint8_t)acc[y * w + x];
  });
}

bool bad2d(int bytes, const void* src, int64_t w, int64_t h, int64_t ss, int r, int64_t k,
           int dims) {
  if (bytes != 1 && bytes != 2) return true;
  if (!src || w <= 0 || h <= 0 || ss < w || r < 0 || r > 4096) return true;
  int64_t side = 2 * (int64_t)r + 1, n = 1;
  for (int i = 0; i < dims; ++i) n *= side;
  return k < 0 || k >= n;
}

}  // namespace

extern "C" {

// Number of threads the oracle uses when asked for 0.
int oracle_default_threads(void) {
  unsigned hc = std::thread::hardware_concurrency();
  return hc ? (int)hc : 1;
}

// Rank-k filter over (2r+1)^2 clamp-to-edge windows.  bytes: 1 = uint8,
// 2 = uint16.  Strides are in elements.  k is 0-based; the median is
// k = ((2r+1)^2 - 1) / 2.  drop_bits clears that many low bits of every result
// (0 = exact).  Returns 0, or -1 on a bad argument.
int oracle_rank2d(int bytes, const void* src, void* dst, int64_t w, int64_t h,
                  int64_t src_stride, int64_t dst_stride, int r, int64_t k, int drop_bits,
                  int nthreads) {
  if (bad2d(bytes, src, w, h, src_stride, r, k, 2) || !dst || dst_stride < w) return -1;
  if (drop_bits < 0 || drop_bits > 8 * bytes) return -1;
  if (bytes == 1)
    rank2d((const uint8_t*)src, (uint8_t*)dst, w, h, src_stride, dst_stride, r, k, drop_bits,
           nthreads);
  else
    rank2d((const uint16_t*)src, (uint16_t*)dst, w, h, src_stride, dst_stride, r, k, drop_bits,
           nthreads);
  return 0;
}

// Rank-k filter of an 8-bit image over (2r+1)^2 clamp-to-edge windows by
// threshold decomposition (independent of oracle_rank2d's selection).
// Returns 0, or -1 on a bad argument.
int oracle_rank2d_u8_thresholds(const void* src, void* dst, int64_t w, int64_t h,
                                int64_t src_stride, int64_t dst_stride, int r, int64_t k,
                                int nthreads) {
  if (bad2d(1, src, w, h, src_stride, r, k, 2) || !dst || dst_stride < w) return -1;
  rank2d_u8_thresholds((const uint8_t*)src, (uint8_t*)dst, w, h, src_stride, dst_stride, r, k,
                       nthreads);
  return 0;
}

// Rank-k filter over (2r+1)^3 clamp-to-edge cubes.  Volume layout: x fastest,
// then rows (row stride), then slices (slice stride), all in elements.
int oracle_rank3d(int bytes, const void* src, void* dst, int64_t w, int64_t h, int64_t d,
                  int64_t src_rs, int64_t src_ss, int64_t dst_rs, int64_t dst_ss, int r,
                  int64_t k, int nthreads) {
  if (bad2d(bytes, src, w, h, src_rs, r, k, 3) || !dst || d <= 0 || dst_rs < w) return -1;
  if (src_ss < src_rs * h || dst_ss < dst_rs * h) return -1;
  if (bytes == 1)
    rank3d((const uint8_t*)src, (uint8_t*)dst, w, h, d, src_rs, src_ss, dst_rs, dst_ss, r, k,
           nthreads);
  else
    rank3d((const uint16_t*)src, (uint16_t*)dst, w, h, d, src_rs, src_ss, dst_rs, dst_ss, r, k,
           nthreads);
  return 0;
}

// Rank-k filter evaluated only at the m points (xs[i], ys[i]); out[i] receives
// the result.  Used to check sampled outputs of full-size images.
int oracle_rank2d_at(int bytes, const void* src, int64_t w, int64_t h, int64_t src_stride,
                     int r, int64_t k, const int64_t* xs, const int64_t* ys, int64_t m,
                     void* out, int nthreads) {
  if (bad2d(bytes, src, w, h, src_stride, r, k, 2) || m < 0 || (m && (!xs || !ys || !out)))
    return -1;
  for (int64_t i = 0; i < m; ++i)
    if (xs[i] < 0 || xs[i] >= w || ys[i] < 0 || ys[i] >= h) return -1;
  if (bytes == 1)
    rank2d_at((const uint8_t*)src, w, h, src_stride, r, k, xs, ys, m, (uint8_t*)out, nthreads);
  else
    rank2d_at((const uint16_t*)src, w, h, src_stride, r, k, xs, ys, m, (uint16_t*)out,
              nthreads);
  return 0;
}

int oracle_rank3d_at(int bytes, const void* src, int64_t w, int64_t h, int64_t d,
                     int64_t src_rs, int64_t src_ss, int r, int64_t k, const int64_t* xs,
                     const int64_t* ys, const int64_t* zs, int64_t m, void* out, int nthreads) {
  if (bad2d(bytes, src, w, h, src_rs, r, k, 3) || d <= 0 || src_ss < src_rs * h || m < 0 ||
      (m && (!xs || !ys || !zs || !out)))
    return -1;
  for (int64_t i = 0; i < m; ++i)
    if (xs[i] < 0 || xs[i] >= w || ys[i] < 0 || ys[i] >= h || zs[i] < 0 || zs[i] >= d)
      return -1;
  if (bytes == 1)
    rank3d_at((const uint8_t*)src, w, h, d, src_rs, src_ss, r, k, xs, ys, zs, m, (uint8_t*)out,
              nthreads);
  else
    rank3d_at((const uint16_t*)src, w, h, d, src_rs, src_ss, r, k, xs, ys, zs, m,
              (uint16_t*)out, nthreads);
  return 0;
}

}  // extern "C"
