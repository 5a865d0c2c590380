// voxel.hip -- voxelisation of an SDF scene onto its fluence grid, the
// geometry of the voxelised comparison model (Sec. 3): each voxel takes the
// region that owns its centre (the highest-index region whose SDF is
// negative there, else the ambient slot), evaluated in FP64 through the same
// region SDFs, uniform-grid acceleration included, that the SDF walk uses.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "walk_common.h"

namespace smcrt {

__global__ void __launch_bounds__(256) voxelize_kernel(const WalkArgs* __restrict__ job_table, int job,
                                                       uint8_t* __restrict__ vox, size_t n) {
  JobRef a = kptr(job_table)[job];
  ScP sc = kptr(a.sc);
  const int nx = sc->g_dims[0], ny = sc->g_dims[1];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int ix = (int)(i % (size_t)nx);
    const size_t r = i / (size_t)nx;
    const int iy = (int)(r % (size_t)ny);
    const int iz = (int)(r / (size_t)ny);
    const V3<double> c = mk(sc->g_lo[0] + (ix + 0.5) * sc->g_d[0], sc->g_lo[1] + (iy + 0.5) * sc->g_d[1],
                            sc->g_lo[2] + (iz + 0.5) * sc->g_d[2]);
    vox[i] = (uint8_t)region_of<double, true>(a, c);
  }
}

hipError_t launch_voxelize(const WalkArgs* d_jobs, int job, uint8_t* vox, size_t n_vox, hipStream_t stream) {
  if (!d_jobs || !vox || job < 0 || n_vox == 0) return hipErrorInvalidValue;
  size_t blocks = (n_vox + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(voxelize_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, d_jobs, job, vox, n_vox);
  return hipGetLastError();
}

}  // namespace smcrt
