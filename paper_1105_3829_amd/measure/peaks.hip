// Peak-bandwidth measurements behind the benchmark's roofline (not part of
// the filter): the LDS read bandwidth of the whole GPU (conflict-free
// ds_read_b128 from two 64 KB workgroups per CU) and the HBM bandwidth of a
// plain streaming copy between buffers far larger than the 256 MB last-level
// cache.  Built into libhrrm_measure.so; bench.py calls it through ctypes.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kWords = 16384;  // 64 KB of LDS per workgroup

__global__ __launch_bounds__(256) void k_lds_read(uint32_t* out, int iters) {
  __shared__ uint32_t s[kWords];
  const int tid = threadIdx.x;
  for (int i = tid; i < kWords; i += 256) s[i] = i * 2654435761u;
  __syncthreads();
  uint32_t acc = 0;
  const uint4* s4 = (const uint4*)s;
  int idx = tid;  // uint4 index: kWords / 4 = 4096 entries, 16 consecutive bytes per lane
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint4 v = s4[(idx + k * 256) & (kWords / 4 - 1)];
      acc += v.x ^ v.y ^ v.z ^ v.w;
    }
    idx = (idx + 1024 + (acc & 1)) & (kWords / 4 - 1);  // keeps the loads live, in range
  }
  out[blockIdx.x * 256 + tid] = acc;
}

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ a, uint4* __restrict__ b,
                                              int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    b[i] = a[i];
}

int time_ms(hipEvent_t a, hipEvent_t b, float* ms) {
  if (hipEventSynchronize(b) != hipSuccess) return -4;
  return hipEventElapsedTime(ms, a, b) == hipSuccess ? 0 : -4;
}

}  // namespace

extern "C" {

// Best of `reps` launches: LDS bytes read per second by all CUs of `device`.
int hrrm_measure_lds_read(int device, int reps, double* bytes_per_s) {
  if (!bytes_per_s || reps < 1) return -1;
  if (hipSetDevice(device) != hipSuccess) return -4;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return -4;
  const int grid = cus * 2;
  uint32_t* out = nullptr;
  if (hipMalloc(&out, (size_t)grid * 256 * 4) != hipSuccess) return -2;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  const int iters = 4096;
  double best = 0;
  int rc = 0;
  for (int rep = 0; rep < reps && rc == 0; ++rep) {
    (void)hipEventRecord(a, nullptr);
    hipLaunchKernelGGL(k_lds_read, dim3(grid), dim3(256), 0, nullptr, out, iters);
    (void)hipEventRecord(b, nullptr);
    float ms = 0;
    rc = time_ms(a, b, &ms);
    const double bytes = (double)grid * 256 * iters * 16 * 16;
    if (rc == 0 && ms > 0 && bytes / (ms * 1e-3) > best) best = bytes / (ms * 1e-3);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(out);
  *bytes_per_s = best;
  return rc;
}

// Best of `reps` copies of `bytes` (rounded down to 16) between two device
// buffers: bytes read + written per second.
int hrrm_measure_hbm_copy(int device, int64_t bytes, int reps, double* bytes_per_s) {
  if (!bytes_per_s || reps < 1 || bytes < 16) return -1;
  if (hipSetDevice(device) != hipSuccess) return -4;
  const int64_t n = bytes / 16;
  uint4 *x = nullptr, *y = nullptr;
  if (hipMalloc(&x, n * 16) != hipSuccess) return -2;
  if (hipMalloc(&y, n * 16) != hipSuccess) {
    (void)hipFree(x);
    return -2;
  }
  (void)hipMemset(x, 1, n * 16);
  (void)hipMemset(y, 0, n * 16);
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  const int grid = (cus > 0 ? cus : 256) * 8;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  double best = 0;
  int rc = 0;
  for (int rep = 0; rep < reps && rc == 0; ++rep) {
    (void)hipEventRecord(a, nullptr);
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, nullptr, rep & 1 ? y : x, rep & 1 ? x : y,
                       n);
    (void)hipEventRecord(b, nullptr);
    float ms = 0;
    rc = time_ms(a, b, &ms);
    if (rc == 0 && ms > 0 && 2.0 * n * 16 / (ms * 1e-3) > best) best = 2.0 * n * 16 / (ms * 1e-3);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(x);
  (void)hipFree(y);
  *bytes_per_s = best;
  return rc;
}

}  // extern "C"
