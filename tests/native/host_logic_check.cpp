// Host checks of the library's device-free logic (csrc/host_logic.hpp):
// argument validation of the image entry points, the request loop's arena and
// its admission rule, the tile-table cache line parser.  Built by the test with
// the host compiler under AddressSanitizer and UBSan; prints one line per check
// group and "failures N" at the end.
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "host_logic.hpp"

using namespace hrrm;

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      ++failures;                                                     \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);     \
    }                                                                 \
  } while (0)

static int chk2(const void* s, const void* d, int dt, int64_t w, int64_t h, int64_t srs,
                int64_t drs, int r) {
  const char* why;
  return check_image_args(s, d, dt, w, h, 1, srs, 0, drs, 0, r, 2, &why);
}
static int chk3(const void* s, const void* d, int dt, int64_t w, int64_t h, int64_t dd,
                int64_t srs, int64_t sss, int64_t drs, int64_t dss, int r) {
  const char* why;
  return check_image_args(s, d, dt, w, h, dd, srs, sss, drs, dss, r, 3, &why);
}

static void validation() {
  // fake, never dereferenced addresses (the checks only compare them)
  const char* A = (const char*)(uintptr_t)0x100000;
  const char* B = (const char*)(uintptr_t)0x900000;
  CHECK(chk2(A, B, HRRM_U8, 64, 32, 64, 64, 3) == HRRM_OK);
  CHECK(chk2(A, B, HRRM_U16, 64, 32, 80, 64, HRRM_MAX_R_2D) == HRRM_OK);
  CHECK(chk2(A, B, 3, 64, 32, 64, 64, 3) == HRRM_EINVAL);                      // dtype
  CHECK(chk2(A, B, HRRM_U8, -1, 32, 64, 64, 3) == HRRM_EINVAL);                // negative
  CHECK(chk2(A, B, HRRM_U8, 64, 32, 64, 64, -1) == HRRM_EINVAL);               // radius
  CHECK(chk2(A, B, HRRM_U8, 64, 32, 64, 64, HRRM_MAX_R_2D + 1) == HRRM_EUNSUPPORTED);
  CHECK(chk2(nullptr, nullptr, HRRM_U8, 0, 32, 0, 0, 3) == HRRM_OK);           // empty: no-op
  CHECK(chk2(nullptr, B, HRRM_U8, 4, 4, 4, 4, 1) == HRRM_EINVAL);              // null
  CHECK(chk2(A, B, HRRM_U8, 64, 32, 63, 64, 3) == HRRM_EINVAL);                // stride < w
  CHECK(chk2(A + 1, B, HRRM_U16, 8, 8, 8, 8, 1) == HRRM_EINVAL);               // misaligned
  CHECK(chk2(A + 1, B, HRRM_U8, 8, 8, 8, 8, 1) == HRRM_OK);                    // u8 any address
  // overlap: u16 4x4 packed = 32 bytes; a dst starting at byte 32 touches nothing
  CHECK(chk2(A, A + 32, HRRM_U16, 4, 4, 4, 4, 1) == HRRM_OK);
  CHECK(chk2(A, A + 30, HRRM_U16, 4, 4, 4, 4, 1) == HRRM_EINVAL);
  CHECK(chk2(A + 32, A, HRRM_U16, 4, 4, 4, 4, 1) == HRRM_OK);
  // the last row of a strided image ends at (h-1)*stride + w, not h*stride
  CHECK(chk2(A, A + 2 * (3 * 10 + 4), HRRM_U16, 4, 4, 10, 4, 1) == HRRM_OK);
  CHECK(chk2(A, A + 2 * (3 * 10 + 3), HRRM_U16, 4, 4, 10, 4, 1) == HRRM_EINVAL);
  // sizes whose products would overflow int64 are rejected, not wrapped
  const int64_t big = (int64_t)1 << 62;
  CHECK(chk2(A, B, HRRM_U8, 4, 4, big, 4, 1) == HRRM_EINVAL);
  CHECK(chk2(A, B, HRRM_U8, big, 4, big, big, 1) == HRRM_EINVAL);
  CHECK(chk2(A, B, HRRM_U16, 4, (int64_t)1 << 40, (int64_t)1 << 40, 4, 1) == HRRM_EINVAL);
  CHECK(chk2(A, B, HRRM_U8, 4, INT64_MAX, 4, 4, 1) == HRRM_EINVAL);
  // volumes
  CHECK(chk3(A, B, HRRM_U16, 8, 8, 4, 8, 64, 8, 64, 2) == HRRM_OK);
  CHECK(chk3(A, B, HRRM_U16, 8, 8, 4, 8, 63, 8, 64, 2) == HRRM_EINVAL);        // slice < plane
  CHECK(chk3(A, B, HRRM_U16, 8, 8, 4, 8, 64, 8, 64, HRRM_MAX_R_3D + 1) == HRRM_EUNSUPPORTED);
  CHECK(chk3(A, B, HRRM_U16, 8, 8, 4, 8, big, 8, 64, 2) == HRRM_EINVAL);       // slice range
  CHECK(chk3(A, B, HRRM_U16, 8, 8, 4, 8, 64, 8, -5, 2) == HRRM_EINVAL);        // negative
  CHECK(chk3(A, B, HRRM_U16, 8, 8, (int64_t)1 << 45, 8, (int64_t)1 << 45, 8, 64, 2) ==
        HRRM_EINVAL);                                                           // (d-1)*sss
  // volume overlap: dst inside the second slice of src
  CHECK(chk3(A, A + 2 * 100, HRRM_U16, 8, 8, 4, 8, 64, 8, 64, 1) == HRRM_EINVAL);
  CHECK(chk3(A, A + 2 * (3 * 64 + 7 * 8 + 8), HRRM_U16, 8, 8, 4, 8, 64, 8, 64, 1) == HRRM_OK);
  std::printf("validation done\n");
}

// Arena against a byte map: random allocations and releases; no two live
// blocks overlap, every block lies inside the arena, used() matches, and
// after releasing everything the free list is one range again.
static void arena() {
  std::mt19937_64 g(7);
  for (int trial = 0; trial < 20; ++trial) {
    const size_t size = 256 * (64 + g() % 256);
    Arena a;
    a.reset(size);
    std::vector<int> owner(size / 256, -1);
    struct Blk { size_t off, n; int id; };
    std::vector<Blk> live;
    size_t used = 0;
    int next = 0;
    for (int step = 0; step < 4000; ++step) {
      if (live.empty() || g() % 3) {
        const size_t n = 1 + g() % (size / 8);
        size_t off = ~(size_t)0;
        if (a.alloc(n, &off)) {
          const size_t m = Arena::round_up(n);
          CHECK(off % 256 == 0 && off + m <= size);
          for (size_t k = off / 256; k < (off + m) / 256 && k < owner.size(); ++k) {
            CHECK(owner[k] < 0);
            owner[k] = next;
          }
          live.push_back({off, n, next++});
          used += m;
        } else {
          // first fit failed: no free run of that length exists
          size_t run = 0, best = 0;
          for (int o : owner) {
            run = o < 0 ? run + 1 : 0;
            best = run > best ? run : best;
          }
          CHECK(best * 256 < Arena::round_up(n));
        }
      } else {
        const size_t i = g() % live.size();
        const Blk b = live[i];
        a.release(b.off, b.n);
        for (size_t k = b.off / 256; k < (b.off + Arena::round_up(b.n)) / 256; ++k) owner[k] = -1;
        used -= Arena::round_up(b.n);
        live.erase(live.begin() + i);
      }
      CHECK(a.used() == used);
    }
    for (const Blk& b : live) a.release(b.off, b.n);
    CHECK(a.used() == 0 && a.free_ranges() == 1);
  }
  std::printf("arena done\n");
}

static void admission() {
  Arena a;
  a.reset(256 * 100);
  // in order while it fits; the slot limit stops the round
  std::vector<std::pair<size_t, size_t>> need = {{2560, 2560}, {2560, 2560}, {2560, 2560}};
  auto p = plan_admission(a, need, 2, 8);
  CHECK(p.size() == 2 && p[0].index == 0 && p[1].index == 1);
  CHECK(p[0].off_in != p[1].off_in && a.used() == 4 * 2560);
  // a request too large for what is left is passed; later small ones go ahead
  a.reset(256 * 100);
  need = {{256 * 60, 256 * 60}, {256 * 10, 256 * 10}, {256 * 5, 256 * 5}};
  p = plan_admission(a, need, 8, 8);
  CHECK(p.size() == 2 && p[0].index == 1 && p[1].index == 2);
  // ... but at most `bypass` passes per round
  a.reset(256 * 100);
  need.assign(12, {256 * 60, 256 * 60});
  need.push_back({256, 256});
  p = plan_admission(a, need, 8, 3);
  CHECK(p.empty());
  CHECK(a.used() == 0);  // a half-admitted request returns its input buffer
  // the admitted buffers never overlap
  a.reset(256 * 1000);
  need.clear();
  for (int i = 0; i < 40; ++i) need.push_back({(size_t)(100 + 97 * i), (size_t)(3000 - 50 * i)});
  p = plan_admission(a, need, 100, 8);
  std::vector<std::pair<size_t, size_t>> blocks;
  for (auto& q : p) {
    blocks.push_back({q.off_in, Arena::round_up(need[q.index].first)});
    blocks.push_back({q.off_out, Arena::round_up(need[q.index].second)});
  }
  for (size_t i = 0; i < blocks.size(); ++i)
    for (size_t j = i + 1; j < blocks.size(); ++j)
      CHECK(blocks[i].first + blocks[i].second <= blocks[j].first ||
            blocks[j].first + blocks[j].second <= blocks[i].first);
  std::printf("admission done\n");
}

static void tuning_lines() {
  TuningLine t;
  const char* good =
      " {\"bytes\": 2, \"dims\": 2, \"r\": 15, \"adaptive\": 0, \"seg_rows\": 48, \"nslots\": 0, "
      "\"min_group\": 1, \"max_groups\": 1, \"lds_budget\": 81920, \"tiered_u8\": 1, "
      "\"raw_window\": 49, \"wave_slots\": 0, \"ms\": 1.39000},";
  CHECK(parse_tuning_line(good, &t, 64, 163840));
  CHECK(t.bytes == 2 && t.r == 15 && t.seg_rows == 48 && t.lds_budget == 81920 && t.ms > 1.38);
  CHECK(!parse_tuning_line("{\"version\": 1, \"entries\": [", &t, 64, 163840));
  std::string bad = good;
  bad.replace(bad.find("81920"), 5, "99999999");  // LDS budget above the limit
  CHECK(!parse_tuning_line(bad.c_str(), &t, 64, 163840));
  bad = good;
  bad.replace(bad.find("\"r\": 15"), 7, "\"r\": 999");  // radius above the maximum
  CHECK(!parse_tuning_line(bad.c_str(), &t, 64, 163840));
  bad = good;
  bad.replace(bad.find("48"), 2, "nan");
  CHECK(!parse_tuning_line(bad.c_str(), &t, 64, 163840));
  bad = good;
  bad.replace(bad.find("\"ms\": "), 6, "\"ms\":");
  CHECK(parse_tuning_line(bad.c_str(), &t, 64, 163840));
  // truncated line: every key is still looked for inside the buffer only
  char cut[40];
  std::memcpy(cut, good, sizeof cut - 1);
  cut[sizeof cut - 1] = 0;
  CHECK(!parse_tuning_line(cut, &t, 64, 163840));
  std::printf("tuning lines done\n");
}

int main() {
  validation();
  arena();
  admission();
  tuning_lines();
  std::printf("failures %d\n", failures);
  return failures ? 1 : 0;
}
