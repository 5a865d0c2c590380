// atomic_ceiling.hip -- measures the FP64 global atomic-add throughput of
// the device, the ceiling under the path-length tally of the walk kernel
// (one FP64 atomic per run of equal voxels).
//
// 4096 workgroups of 256 threads each add 1.0 at 1000 addresses of a
// 200^3 FP64 grid (64 MB, the slab workload's grid):
//   pattern 0: independent hashed voxels;
//   pattern 1: a 3-D random walk of unit voxel moves (DDA-like locality).
// Forms: the builtin the walk kernel uses, the same add at agent and at
// workgroup scope, and per-XCD private copies of the grid (each workgroup
// adds into the copy of the XCD it runs on).  Every index is reduced modulo
// the grid size; the exact total of the adds is checked after each run.
// A second part gives the lanes of each instruction hashed segments shared
// by g consecutive lanes (g = 1, 2, 4, 8, 16, 64 contiguous doubles), to show
// whether the rate is per add or per 64-byte memory request (a segment of
// g < 8 doubles is one request, a wider one g / 8).
// Prints one line per form and pattern, one per segment width, then
// "atomics_per_s: <best of the builtin form>".
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                              \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess) {                                                                   \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);              \
      std::exit(1);                                                                           \
    }                                                                                         \
  } while (0)

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// XCD of the executing wave: hwreg(HW_REG_XCC_ID, 0, 4), masked to 0..7
__device__ __forceinline__ int xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7; }

enum { kBuiltin = 0, kAgent = 1, kWorkgroup = 2, kPrivate = 3 };

template <int MODE>
__global__ void __launch_bounds__(256) adds(double* F, uint32_t nx, uint32_t ny, uint32_t nz, int iters, int pattern) {
  const uint32_t n = nx * ny * nz;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  double* G = MODE == kPrivate ? F + (size_t)xcc_id() * n : F;
  const uint32_t h = hash32(tid * 2654435761U + 12345U);
  int x = (int)(h % nx), y = (int)((h >> 8) % ny), z = (int)((h >> 16) % nz);
  for (int i = 0; i < iters; ++i) {
    uint32_t idx;
    if (pattern == 0) {
      idx = hash32(tid ^ hash32((uint32_t)i + 777U)) % n;
    } else {
      const uint32_t r = hash32(tid * 31U + (uint32_t)i * 1000003U);
      const int ax = (int)(r % 3), d = ((r >> 4) & 1) ? 1 : -1;
      if (ax == 0) x = (x + d + (int)nx) % (int)nx;
      else if (ax == 1) y = (y + d + (int)ny) % (int)ny;
      else z = (z + d + (int)nz) % (int)nz;
      idx = (uint32_t)x + nx * ((uint32_t)y + ny * (uint32_t)z);
    }
    double* p = G + idx;
    if (MODE == kBuiltin || MODE == kPrivate)
      __builtin_amdgcn_global_atomic_fadd_f64((__attribute__((address_space(1))) double*)p, 1.0);
    else if (MODE == kAgent)
      __hip_atomic_fetch_add(p, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_fetch_add(p, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// lanes tid..tid+g-1 (g divides 64) add at g consecutive doubles of one
// hashed, g-aligned segment of the n-element grid (g divides n)
__global__ void __launch_bounds__(256) segment_adds(double* F, uint32_t n, int iters, int g) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t seg = tid / (uint32_t)g, nseg = n / (uint32_t)g;
  for (int i = 0; i < iters; ++i) {
    const uint32_t base = (hash32(seg ^ hash32((uint32_t)i + 777U)) % nseg) * (uint32_t)g;
    __builtin_amdgcn_global_atomic_fadd_f64((__attribute__((address_space(1))) double*)(F + base + (threadIdx.x & 63u) % (uint32_t)g), 1.0);
  }
}

__global__ void sum_kernel(const double* F, size_t n, double* out) {
  double s = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) s += F[i];
  atomicAdd(out, s);
}

int main() {
  const uint32_t nx = 200, ny = 200, nz = 200, n = nx * ny * nz;
  const int blocks = 4096, threads = 256, iters = 1000;
  const size_t cells = (size_t)n * 8;  // room for eight private copies
  double* F = nullptr;
  double* d_sum = nullptr;
  CHECK(hipMalloc(&F, sizeof(double) * cells));
  CHECK(hipMalloc(&d_sum, sizeof(double)));
  hipEvent_t a, b;
  CHECK(hipEventCreate(&a));
  CHECK(hipEventCreate(&b));
  const char* names[] = {"builtin", "agent scope", "workgroup scope", "per-XCD copies"};
  const double want = (double)blocks * threads * iters;
  double best_builtin = 0.0;
  for (int pattern = 0; pattern < 2; ++pattern) {
    for (int mode = 0; mode < 4; ++mode) {
      float ms = 0.0f;
      double sum = 0.0;
      for (int rep = 0; rep < 2; ++rep) {  // the first run warms up
        CHECK(hipMemset(F, 0, sizeof(double) * cells));
        CHECK(hipMemset(d_sum, 0, sizeof(double)));
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(a, 0));
        const dim3 g(blocks), t(threads);
        if (mode == kBuiltin) hipLaunchKernelGGL(adds<kBuiltin>, g, t, 0, 0, F, nx, ny, nz, iters, pattern);
        else if (mode == kAgent) hipLaunchKernelGGL(adds<kAgent>, g, t, 0, 0, F, nx, ny, nz, iters, pattern);
        else if (mode == kWorkgroup) hipLaunchKernelGGL(adds<kWorkgroup>, g, t, 0, 0, F, nx, ny, nz, iters, pattern);
        else hipLaunchKernelGGL(adds<kPrivate>, g, t, 0, 0, F, nx, ny, nz, iters, pattern);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(b, 0));
        CHECK(hipEventSynchronize(b));
        CHECK(hipEventElapsedTime(&ms, a, b));
        hipLaunchKernelGGL(sum_kernel, dim3(1024), dim3(256), 0, 0, F, cells, d_sum);
        CHECK(hipGetLastError());
        CHECK(hipMemcpy(&sum, d_sum, sizeof(double), hipMemcpyDeviceToHost));
      }
      const double rate = want / (ms * 1e-3);
      if (mode == kBuiltin && rate > best_builtin) best_builtin = rate;
      std::printf("pattern %d  %-16s %8.2f ms  %.3e atomics/s  total %s\n", pattern, names[mode], ms, rate,
                  sum == want ? "exact" : "WRONG");
      std::fflush(stdout);
    }
  }
  const int widths[] = {1, 2, 4, 8, 16, 64};
  for (int wi = 0; wi < 6; ++wi) {
    const int g = widths[wi];
    if (n % (uint32_t)g != 0) return 2;
    float ms = 0.0f;
    double sum = 0.0;
    for (int rep = 0; rep < 2; ++rep) {
      CHECK(hipMemset(F, 0, sizeof(double) * n));
      CHECK(hipMemset(d_sum, 0, sizeof(double)));
      CHECK(hipDeviceSynchronize());
      CHECK(hipEventRecord(a, 0));
      hipLaunchKernelGGL(segment_adds, dim3(blocks), dim3(threads), 0, 0, F, n, iters, g);
      CHECK(hipGetLastError());
      CHECK(hipEventRecord(b, 0));
      CHECK(hipEventSynchronize(b));
      CHECK(hipEventElapsedTime(&ms, a, b));
      hipLaunchKernelGGL(sum_kernel, dim3(1024), dim3(256), 0, 0, F, (size_t)n, d_sum);
      CHECK(hipGetLastError());
      CHECK(hipMemcpy(&sum, d_sum, sizeof(double), hipMemcpyDeviceToHost));
    }
    std::printf("segment of %2d doubles per %2d lanes %8.2f ms  %.3e atomics/s  %.3e 64-byte requests/s  total %s\n", g, g,
                ms, want / (ms * 1e-3), want / (ms * 1e-3) / (g < 8 ? g : 8),
                sum == want ? "exact" : "WRONG");
    std::fflush(stdout);
  }
  std::printf("atomics_per_s: %.4e\n", best_builtin);
  CHECK(hipFree(F));
  CHECK(hipFree(d_sum));
  return 0;
}
