// launch.h -- host-callable launchers of the device kernels (walk.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "layout.h"

namespace smcrt {

// precision: 0 = FP32 transport, 1 = FP64 transport; trace: record events
// (trace launches take exactly one job).  args.geometry selects the kernel
// (sphere tracing or voxel walk) and the jobs it takes.
hipError_t launch_walk(int precision, bool trace, const LaunchCfg& cfg, const BatchArgs& args, hipStream_t stream);
// region slot of every voxel centre of job `job`'s scene into vox (n_vox bytes)
hipError_t launch_voxelize(const WalkArgs* d_jobs, int job, uint8_t* vox, size_t n_vox, hipStream_t stream);
hipError_t launch_distance(int precision, const WalkArgs* d_jobs, int job, const double* points, uint64_t n, int accelerated,
                           double* dist, int32_t* owner, double* normals, hipStream_t stream);
// p[i] = 0 for i < n (a kernel, so resets can sit inside captured graphs)
hipError_t launch_zero_u64_n(unsigned long long* p, int n, hipStream_t stream);
// zero n doubles (a kernel, so it can sit in a captured graph)
hipError_t launch_zero_f64(double* p, size_t n, hipStream_t stream);
// F (x fastest, nx*ny*nz) += S (the 2x2x2-brick grid the walk tallied into)
hipError_t launch_brick_add(const double* S, double* F, int nx, int ny, int nz, hipStream_t stream);
// *p = 0 (a one-thread kernel, so the reset can sit inside captured graphs)
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t stream);
// out[i] = in[i] * scale for i < n
hipError_t launch_scale(const double* in, double* out, size_t n, double scale, hipStream_t stream);
// device build of the uniform grid of the accelerated region (counts and
// cursors: n_cells each; offsets: n_cells + 1; ids: the capacity in the header)
hipError_t launch_accel_build(const SceneHeader* d_sc, const PrimD* d_pd, int n_prims, int n_cells, uint32_t* counts,
                              uint32_t* cursors, uint32_t* offsets, uint32_t* ids, hipStream_t stream);
// resident workgroups per CU of the walk kernel of this launch class at this block size
int walk_max_blocks_per_cu(int precision, int block, int launch_class);

// Resident serving (serve.hip): packets saved at the end of an epoch are
// fixed-size records in a slab, slot first.  counts[slot] += records of the
// slot; scatter puts each record at offsets[slot] + k (cursors count k);
// carry appends the records a job did not resume back to the save slab.
// n: device count of records (clamped to cap).
hipError_t launch_saved_count(const unsigned char* slab, const unsigned int* n, unsigned int cap, unsigned int* counts,
                              int n_slots, hipStream_t stream);
hipError_t launch_saved_scatter(const unsigned char* src, const unsigned int* n, unsigned int cap,
                                const unsigned int* offsets, unsigned int* cursors, unsigned char* dst, int n_slots,
                                hipStream_t stream);
hipError_t launch_saved_carry(const WalkArgs* jobs, int n_jobs, unsigned char* save, unsigned int* save_count,
                              unsigned int cap, hipStream_t stream);
hipError_t launch_zero_u32(unsigned int* p, int n, hipStream_t stream);

// Fixed device scratch of the run that allocates nothing (static_run.hip):
// its size, and its address on `device`, which must be the current device
// (looked up once per device and kept).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
hipError_t static_scratch(int device, void** out);
// *dst = a, with a passed as a kernel argument
hipError_t launch_write_job(const WalkArgs& a, WalkArgs* dst, hipStream_t stream);

}  // namespace smcrt
