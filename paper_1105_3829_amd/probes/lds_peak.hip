// LDS bandwidth probe behind the roofline's LDS peak: conflict-free
// ds_read_b32 and ds_read_b128 from every CU (two 64 KB workgroups per CU),
// timed with HIP events.
//
//   hipcc --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops -O3 \
//       paper_1105_3829_amd/probes/lds_peak.hip -o lds_peak && ./lds_peak
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
constexpr int kWords = 16384;  // 64 KB of LDS per workgroup
template <int VEC>
__global__ __launch_bounds__(256) void k_lds(uint32_t* out, int iters) {
  __shared__ uint32_t s[kWords];
  const int tid = threadIdx.x;
  for (int i = tid; i < kWords; i += 256) s[i] = i * 2654435761u;
  __syncthreads();
  uint32_t acc = 0;
  if (VEC == 1) {
    int idx = tid;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += s[(idx + k * 256) & (kWords - 1)];
      idx = (idx + 4096 + (acc & 1)) & (kWords - 1);  // keep loads live, stay in range
    }
  } else {
    const uint4* s4 = (const uint4*)s;
    int idx = tid;  // uint4 index, kWords/4 = 4096 entries
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint4 v = s4[(idx + k * 256) & (kWords / 4 - 1)];
        acc += v.x ^ v.y ^ v.z ^ v.w;
      }
      idx = (idx + 1024 + (acc & 1)) & (kWords / 4 - 1);
    }
  }
  out[blockIdx.x * 256 + tid] = acc;
}
int main() {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess) return 1;
  const int grid = cus * 2;  // 2 x 64 KB per CU
  uint32_t* out;
  if (hipMalloc(&out, (size_t)grid * 256 * 4) != hipSuccess) return 1;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 1;
  const int iters = 4096;
  for (int rep = 0; rep < 2; ++rep) {
    for (int vec : {1, 4}) {
      (void)hipEventRecord(a);
      if (vec == 1) hipLaunchKernelGGL(k_lds<1>, dim3(grid), dim3(256), 0, 0, out, iters);
      else hipLaunchKernelGGL(k_lds<4>, dim3(grid), dim3(256), 0, 0, out, iters);
      (void)hipEventRecord(b);
      if (hipEventSynchronize(b) != hipSuccess) return 2;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, a, b);
      const double bytes = (double)grid * 256 * iters * 16 * 4 * vec;
      printf("cus %d ds_read_b%d: %.3f ms, %.1f GB/s (%.1f B/clk/CU at 2.4 GHz)\n", cus, 32 * vec, ms,
             bytes / ms / 1e6, bytes / (ms * 1e-3) / cus / 2.4e9);
    }
  }
  (void)hipFree(out);
  return 0;
}
