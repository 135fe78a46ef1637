// Drives the oracle's C entry points on buffers of exactly the extent their
// sizes and strides describe (tiny, ragged and degenerate images, radii past
// the image, padded strides, 2-D and 3-D, full and sampled outputs), for a
// build with AddressSanitizer and UBSan: any read or write outside those
// buffers, or undefined behaviour, aborts the run.  Prints the number of calls
// that returned an error; exit status 0 only when there are none.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int oracle_rank2d(int, const void*, void*, int64_t, int64_t, int64_t, int64_t, int, int64_t, int,
                  int);
int oracle_rank3d(int, const void*, void*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                  int64_t, int, int64_t, int);
int oracle_rank2d_at(int, const void*, int64_t, int64_t, int64_t, int, int64_t, const int64_t*,
                     const int64_t*, int64_t, void*, int);
int oracle_rank3d_at(int, const void*, int64_t, int64_t, int64_t, int64_t, int64_t, int, int64_t,
                     const int64_t*, const int64_t*, const int64_t*, int64_t, void*, int);
}

int main() {
  std::mt19937 g(1);
  int calls = 0, errors = 0;
  auto fill = [&](std::vector<uint8_t>& v) {
    for (auto& b : v) b = (uint8_t)g();
  };
  for (int bytes : {1, 2})
    for (int64_t w : {1, 2, 3, 7, 17})
      for (int64_t h : {1, 2, 5, 9})
        for (int r : {0, 1, 2, 5, 20}) {
          const int64_t ss = w + w % 3, ds = w;
          std::vector<uint8_t> src(((h - 1) * ss + w) * bytes), dst(((h - 1) * ds + w) * bytes);
          fill(src);
          const int64_t n = (2 * r + 1) * (int64_t)(2 * r + 1);
          for (int64_t k : {(int64_t)0, (n - 1) / 2, n - 1}) {
            ++calls;
            errors += oracle_rank2d(bytes, src.data(), dst.data(), w, h, ss, ds, r, k,
                                    bytes == 2 ? 3 : 1, 2) != 0;
            std::vector<int64_t> xs, ys;
            for (int i = 0; i < 5; ++i) {
              xs.push_back(g() % w);
              ys.push_back(g() % h);
            }
            std::vector<uint8_t> out(5 * bytes);
            ++calls;
            errors += oracle_rank2d_at(bytes, src.data(), w, h, ss, r, k, xs.data(), ys.data(), 5,
                                       out.data(), 2) != 0;
          }
          if (r > 5) continue;
          for (int64_t d : {1, 3}) {
            const int64_t sls = ss * h + 1;
            std::vector<uint8_t> s3(((d - 1) * sls + (h - 1) * ss + w) * bytes),
                d3(d * h * w * bytes);
            fill(s3);
            const int64_t n3 = n * (2 * r + 1);
            ++calls;
            errors += oracle_rank3d(bytes, s3.data(), d3.data(), w, h, d, ss, sls, w, w * h, r,
                                    (n3 - 1) / 2, 2) != 0;
            std::vector<int64_t> xs{0, w - 1}, ys{h - 1, 0}, zs{0, d - 1};
            std::vector<uint8_t> out(2 * bytes);
            ++calls;
            errors += oracle_rank3d_at(bytes, s3.data(), w, h, d, ss, sls, r, n3 - 1, xs.data(),
                                       ys.data(), zs.data(), 2, out.data(), 1) != 0;
          }
        }
  std::printf("calls %d errors %d\n", calls, errors);
  return errors != 0;
}
