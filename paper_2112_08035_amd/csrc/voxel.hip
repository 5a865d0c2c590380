// voxel.hip -- voxelisation of an SDF scene onto its fluence grid, the
// geometry of the voxelised comparison model (Sec. 3): each voxel takes the
// region that owns its centre (the highest-index region whose SDF is
// negative there, else the ambient slot), evaluated in FP64 through the same
// region SDFs, uniform-grid acceleration included, that the SDF walk uses;
// and point queries of those SDFs.
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

// Point queries: every region's SDF at each point (through the uniform grid
// for the accelerated region when accelerated), the point's owner by the
// walk's rule, in transport type T; and, when asked, every region's unit
// normal by the interface step's FP64 central differences (step h_normal).
template <typename T>
__global__ void __launch_bounds__(256) distance_kernel(const WalkArgs* __restrict__ job_table, int job,
                                                       const double* __restrict__ pts, uint64_t n, int accelerated,
                                                       double* __restrict__ dist, int32_t* __restrict__ owner,
                                                       double* __restrict__ normals) {
  JobRef a = kptr(job_table)[job];
  ScP sc = kptr(a.sc);
  const int nr = sc->n_regions;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const V3<T> p = mk((T)pts[3 * i], (T)pts[3 * i + 1], (T)pts[3 * i + 2]);
    int own = nr;
    for (int r = 0; r < nr; ++r) {
      const T d = accelerated ? region_dist<T, true>(a, r, p) : region_sdf<T, true>(a, sc->reg[r], p);
      dist[i * (uint64_t)nr + r] = (double)d;
      if (d < T(0)) own = r;
    }
    if (owner) owner[i] = own;
    if (normals) {
      const V3<double> q = mk(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
      const double h = sc->h_normal;
      for (int r = 0; r < nr; ++r) {
        auto f = [&](V3<double> x) {
          return accelerated ? region_dist<double, true>(a, r, x) : region_sdf<double, true>(a, sc->reg[r], x);
        };
        V3<double> g = mk(f(mk(q.x + h, q.y, q.z)) - f(mk(q.x - h, q.y, q.z)),
                          f(mk(q.x, q.y + h, q.z)) - f(mk(q.x, q.y - h, q.z)),
                          f(mk(q.x, q.y, q.z + h)) - f(mk(q.x, q.y, q.z - h)));
        g = (1.0 / __builtin_sqrt(dot(g, g))) * g;
        double* o = normals + 3 * (i * (uint64_t)nr + r);
        o[0] = g.x;
        o[1] = g.y;
        o[2] = g.z;
      }
    }
  }
}

hipError_t launch_distance(int precision, const WalkArgs* d_jobs, int job, const double* points, uint64_t n, int accelerated,
                           double* dist, int32_t* owner, double* normals, hipStream_t stream) {
  if (!d_jobs || !points || !dist || job < 0 || n == 0) return hipErrorInvalidValue;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (precision == 1)
    hipLaunchKernelGGL(distance_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, stream, d_jobs, job, points, n,
                       accelerated, dist, owner, normals);
  else
    hipLaunchKernelGGL(distance_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, stream, d_jobs, job, points, n,
                       accelerated, dist, owner, normals);
  return hipGetLastError();
}

hipError_t launch_voxelize(const WalkArgs* d_jobs, int job, uint8_t* vox, size_t n_vox, hipStream_t stream) {
  if (!d_jobs || !vox || job < 0 || n_vox == 0) return hipErrorInvalidValue;
  size_t blocks = (n_vox + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(voxelize_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, d_jobs, job, vox, n_vox);
  return hipGetLastError();
}

}  // namespace smcrt
