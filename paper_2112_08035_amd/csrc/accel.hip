// accel.hip -- device build of the uniform-grid acceleration of one union
// region (Sec. 5: a space-partitioning structure so that a step need not
// evaluate every SDF of a large collection).
//
// Three passes over the region's primitives, all on the device:
//   count : every primitive adds 1 to each cell its bounding box, grown by
//           the margin, overlaps;
//   scan  : one workgroup turns the counts into CSR offsets;
//   fill  : every primitive writes its index into those cells' lists;
// then the ring distances of the empty cells, over the counts buffer.
// count and fill share one cell-range routine, so they agree exactly; fill
// still checks every write against the capacity the host allocated.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "layout.h"

namespace smcrt {

// inclusive cell range [c0, c1] of a primitive's world box (packed by the
// host for every kind, placement and modifier) grown by the margin, clamped
__device__ __forceinline__ void cell_range(const Accel& A, const PrimD& P, int c0[3], int c1[3]) {
  for (int i = 0; i < 3; ++i) {
    const double a = (P.box_lo[i] - A.margin - A.lo[i]) * A.inv_cell[i];
    const double b = (P.box_hi[i] + A.margin - A.lo[i]) * A.inv_cell[i];
    int x0 = (int)floor(fmax(a, -1.0)), x1 = (int)floor(fmin(b, (double)A.dims[i]));
    x0 = x0 < 0 ? 0 : (x0 >= A.dims[i] ? A.dims[i] - 1 : x0);
    x1 = x1 < 0 ? 0 : (x1 >= A.dims[i] ? A.dims[i] - 1 : x1);
    c0[i] = x0;
    c1[i] = x1;
  }
}

// Whether cell (x, y, z) lists the primitive.  A primitive whose box grown
// by the margin overlaps the cell is listed, except a plain capsule whose
// axis segment lies farther than r + margin + (half the cell diagonal) from
// the cell centre: every point of the cell is then more than margin from
// its surface, so a query there never needs it.  The test errs towards
// listing (a relative slack of 1e-9 covers the rounding of the distance).
__device__ __forceinline__ bool cell_lists(const Accel& A, const PrimD& P, int x, int y, int z) {
  if (P.kind != kCapsule || P.flags != 0) return true;
  double c[3], hd2 = 0.0;
  const int ix[3] = {x, y, z};
  for (int i = 0; i < 3; ++i) {
    const double w = 1.0 / A.inv_cell[i];
    c[i] = A.lo[i] + (ix[i] + 0.5) * w - P.v[i];  // cell centre relative to the segment start
    hd2 += 0.25 * w * w;
  }
  const double t = fmin(fmax((c[0] * P.v[3] + c[1] * P.v[4] + c[2] * P.v[5]) * P.v[6], 0.0), 1.0);
  const double d0 = c[0] - t * P.v[3], d1 = c[1] - t * P.v[4], d2 = c[2] - t * P.v[5];
  const double reach = (P.v[7] + A.margin + sqrt(hd2)) * (1.0 + 1e-9);
  return d0 * d0 + d1 * d1 + d2 * d2 <= reach * reach;
}

__global__ void accel_zero(uint32_t* __restrict__ a, uint32_t* __restrict__ b, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    a[i] = 0u;
    b[i] = 0u;
  }
}

__global__ void accel_count(const SceneHeader* __restrict__ sc, const PrimD* __restrict__ pd, uint32_t* __restrict__ counts) {
  const Accel& A = sc->acc;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n_prims) return;
  int c0[3], c1[3];
  const PrimD& P = pd[A.first_prim + i];
  cell_range(A, P, c0, c1);
  for (int z = c0[2]; z <= c1[2]; ++z)
    for (int y = c0[1]; y <= c1[1]; ++y)
      for (int x = c0[0]; x <= c1[0]; ++x)
        if (cell_lists(A, P, x, y, z)) atomicAdd(&counts[x + A.dims[0] * (y + A.dims[1] * z)], 1u);
}

// exclusive scan of counts into offsets[0..n_cells]; one workgroup of 1024
__global__ void __launch_bounds__(1024) accel_scan(const SceneHeader* __restrict__ sc, const uint32_t* __restrict__ counts,
                                                   uint32_t* __restrict__ offsets) {
  __shared__ uint32_t part[1024];
  const int n = sc->acc.n_cells;
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int b = t * chunk, e = min(n, b + chunk);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += counts[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = t ? part[t - 1] : 0u;
  for (int i = b; i < e; ++i) {
    offsets[i] = run;
    run += counts[i];
  }
  if (t == 1023) offsets[n] = part[1023];
}

__global__ void accel_fill(const SceneHeader* __restrict__ sc, const PrimD* __restrict__ pd,
                           const uint32_t* __restrict__ offsets, uint32_t* __restrict__ cursors, uint32_t* __restrict__ ids) {
  const Accel& A = sc->acc;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n_prims) return;
  int c0[3], c1[3];
  const PrimD& P = pd[A.first_prim + i];
  cell_range(A, P, c0, c1);
  for (int z = c0[2]; z <= c1[2]; ++z)
    for (int y = c0[1]; y <= c1[1]; ++y)
      for (int x = c0[0]; x <= c1[0]; ++x) {
        if (!cell_lists(A, P, x, y, z)) continue;
        const int c = x + A.dims[0] * (y + A.dims[1] * z);
        const uint64_t slot = (uint64_t)offsets[c] + atomicAdd(&cursors[c], 1u);
        if (slot < A.capacity) ids[slot] = (uint32_t)(A.first_prim + i);
      }
}

// ring distances: 0 for a cell that lists a primitive, kRingMax otherwise,
// then relaxed over the 26 neighbours (out = min(in, 1 + neighbours' min));
// pass j makes every distance up to j exact
__global__ void accel_ring_init(const SceneHeader* __restrict__ sc, const uint32_t* __restrict__ counts,
                                uint32_t* __restrict__ ring) {
  const int n = sc->acc.n_cells;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    ring[i] = counts[i] ? 0u : (uint32_t)kRingMax;
}

__global__ void accel_ring_pass(const SceneHeader* __restrict__ sc, const uint32_t* __restrict__ in,
                                uint32_t* __restrict__ out) {
  const Accel& A = sc->acc;
  const int dx = A.dims[0], dy = A.dims[1], dz = A.dims[2];
  const int n = A.n_cells;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int x = i % dx, y = (i / dx) % dy, z = i / (dx * dy);
    uint32_t m = in[i];
    for (int cz = z - 1; cz <= z + 1; ++cz) {
      if (cz < 0 || cz >= dz) continue;
      for (int cy = y - 1; cy <= y + 1; ++cy) {
        if (cy < 0 || cy >= dy) continue;
        for (int cx = x - 1; cx <= x + 1; ++cx) {
          if (cx < 0 || cx >= dx) continue;
          const uint32_t v = in[cx + dx * (cy + dy * cz)] + 1u;
          m = v < m ? v : m;
        }
      }
    }
    out[i] = m;
  }
}

hipError_t launch_accel_build(const SceneHeader* d_sc, const PrimD* d_pd, int n_prims, int n_cells, uint32_t* counts,
                              uint32_t* cursors, uint32_t* offsets, uint32_t* ids, hipStream_t stream) {
  if (!d_sc || !d_pd || !counts || !cursors || !offsets || !ids || n_prims < 1 || n_cells < 1) return hipErrorInvalidValue;
  const int zb = (n_cells + 255) / 256;
  hipLaunchKernelGGL(accel_zero, dim3(zb < 4096 ? zb : 4096), dim3(256), 0, stream, counts, cursors, n_cells);
  const int pb = (n_prims + 255) / 256;
  hipLaunchKernelGGL(accel_count, dim3(pb), dim3(256), 0, stream, d_sc, d_pd, counts);
  hipLaunchKernelGGL(accel_scan, dim3(1), dim3(1024), 0, stream, d_sc, counts, offsets);
  hipLaunchKernelGGL(accel_fill, dim3(pb), dim3(256), 0, stream, d_sc, d_pd, offsets, cursors, ids);
  // counts and cursors are free now: ring distances, ending in counts
  hipLaunchKernelGGL(accel_ring_init, dim3(zb < 4096 ? zb : 4096), dim3(256), 0, stream, d_sc, counts, cursors);
  for (int j = 1; j < kRingMax; ++j) {
    uint32_t* src = (j & 1) ? cursors : counts;
    uint32_t* dst = (j & 1) ? counts : cursors;
    hipLaunchKernelGGL(accel_ring_pass, dim3(zb < 4096 ? zb : 4096), dim3(256), 0, stream, d_sc, src, dst);
  }
  static_assert((kRingMax - 1) % 2 == 1, "the last ring pass writes counts");
  return hipGetLastError();
}

}  // namespace smcrt
