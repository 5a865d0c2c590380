// serve.hip -- device helpers of the resident request server: the packets
// an epoch leaves in flight are kept in HBM as fixed-size records (slot
// first) and sorted by slot before the next epoch resumes them.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "walk_common.h"

namespace smcrt {

namespace {

__device__ __forceinline__ unsigned int saved_records(const unsigned int* n, unsigned int cap) {
  const unsigned int c = *n;
  return c < cap ? c : cap;
}

__device__ __forceinline__ void copy_record(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
#pragma unroll
  for (int k = 0; k < kSavedPacketBytes / 16; ++k) d[k] = s[k];
}

}  // namespace

// counts[slot] += 1 for every saved record
__global__ void saved_count_kernel(const unsigned char* __restrict__ slab, const unsigned int* __restrict__ n,
                                   unsigned int cap, unsigned int* __restrict__ counts, int n_slots) {
  const unsigned int m = saved_records(n, cap);
  for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const int slot = *reinterpret_cast<const int32_t*>(slab + (size_t)i * kSavedPacketBytes);
    if (slot >= 0 && slot < n_slots) atomicAdd(&counts[slot], 1u);
  }
}

// every record to its slot's segment: dst[offsets[slot] + k], k counted by cursors
__global__ void saved_scatter_kernel(const unsigned char* __restrict__ src, const unsigned int* __restrict__ n,
                                     unsigned int cap, const unsigned int* __restrict__ offsets,
                                     unsigned int* __restrict__ cursors, unsigned char* __restrict__ dst, int n_slots) {
  const unsigned int m = saved_records(n, cap);
  for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const unsigned char* r = src + (size_t)i * kSavedPacketBytes;
    const int slot = *reinterpret_cast<const int32_t*>(r);
    if (slot < 0 || slot >= n_slots) continue;
    const unsigned int k = offsets[slot] + atomicAdd(&cursors[slot], 1u);
    if (k < cap) copy_record(r, dst + (size_t)k * kSavedPacketBytes);
  }
}

// the saved packets a job did not get to resume go back into the save slab
__global__ void saved_carry_kernel(const WalkArgs* __restrict__ jobs, unsigned char* __restrict__ save,
                                   unsigned int* __restrict__ save_count, unsigned int cap) {
  const WalkArgs& J = jobs[blockIdx.x];
  if (J.resume_n == 0 || J.resume == nullptr) return;
  __shared__ unsigned int base, first;
  if (threadIdx.x == 0) {
    const unsigned int taken = *J.resume_next;
    first = taken < J.resume_n ? taken : J.resume_n;
    base = atomicAdd(save_count, J.resume_n - first);
  }
  __syncthreads();
  const unsigned char* src = static_cast<const unsigned char*>(J.resume);
  for (unsigned int i = first + threadIdx.x; i < J.resume_n; i += blockDim.x) {
    const unsigned int k = base + (i - first);
    if (k < cap) copy_record(src + (size_t)i * kSavedPacketBytes, save + (size_t)k * kSavedPacketBytes);
  }
}

__global__ void zero_u32_kernel(unsigned int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t launch_saved_count(const unsigned char* slab, const unsigned int* n, unsigned int cap, unsigned int* counts,
                              int n_slots, hipStream_t stream) {
  hipLaunchKernelGGL(saved_count_kernel, dim3(1024), dim3(256), 0, stream, slab, n, cap, counts, n_slots);
  return hipGetLastError();
}

hipError_t launch_saved_scatter(const unsigned char* src, const unsigned int* n, unsigned int cap,
                                const unsigned int* offsets, unsigned int* cursors, unsigned char* dst, int n_slots,
                                hipStream_t stream) {
  hipLaunchKernelGGL(saved_scatter_kernel, dim3(1024), dim3(256), 0, stream, src, n, cap, offsets, cursors, dst, n_slots);
  return hipGetLastError();
}

hipError_t launch_saved_carry(const WalkArgs* jobs, int n_jobs, unsigned char* save, unsigned int* save_count,
                              unsigned int cap, hipStream_t stream) {
  if (n_jobs < 1) return hipSuccess;
  hipLaunchKernelGGL(saved_carry_kernel, dim3(n_jobs), dim3(256), 0, stream, jobs, save, save_count, cap);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int* p, int n, hipStream_t stream) {
  if (!p || n < 1) return hipErrorInvalidValue;
  const int blocks = (n + 255) / 256;
  hipLaunchKernelGGL(zero_u32_kernel, dim3(blocks < 1024 ? blocks : 1024), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

}  // namespace smcrt
