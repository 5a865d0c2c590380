// layout.h -- device-side scene tables of libsmcrt (host packer <-> kernels).
//
// One contiguous blob per scene: a SceneHeader, then n_prims PrimD (FP64
// parameters, used by the interface step and by FP64 transport), then
// n_prims PrimF (FP32 copies for FP32 transport).  Every table is read with
// wave-uniform indices, so the kernels fetch it through the scalar cache into
// SGPRs; nothing per lane.
#pragma once
#include <stdint.h>

namespace smcrt {

constexpr int kMaxRegions = 16;     // regions per scene (ambient adds one slot)
constexpr int kMaxPrims = 1 << 20;  // primitives per scene

enum PrimKind : int32_t {
  kSphere = 0, kBox = 1, kCapsule = 2, kCylinder = 3, kTorus = 4,
  // further shapes: evaluated only on the placed-primitive path
  kCone = 5, kOctahedron = 6, kHexPrism = 7, kEllipsoid = 8
};
enum RegionOp : int32_t { kUnion = 0, kSmoothUnion = 1, kIntersect = 2, kSubtract = 3 };
enum SourceKind : int32_t { kPoint = 0, kPencil = 1, kDisc = 2, kRect = 3 };
// geometry model of a scene: the signed distance functions themselves, or
// the voxel grid they induce (region of each voxel centre) -- the voxelised
// comparison model of Sec. 3
enum Geometry : int32_t { kGeomSdf = 0, kGeomVoxel = 1 };
// launch class of a job: its geometry model, plus kLaunchXf when its scene
// has placed or modified primitives (a separate kernel instantiation);
// kLaunchStaged: an FP32 SDF job whose accelerated region is plain capsules
// that fit the workgroup's LDS table (the staged-capsule kernel);
// kLaunchSegment: an SDF job with segment-traced steps
enum LaunchClass : int32_t { kLaunchXf = 2, kLaunchStaged = 4, kLaunchSegment = 5, kLaunchClasses = 6 };
// segment-tracing rule of a region: how the tangent bounds of its members
// bound the way to its surface (none: the distance alone)
enum SegRule : int32_t { kSegNone = 0, kSegUnion = 1, kSegIntersect = 2, kSegSubtract = 3 };

// capsules an FP32 staged-capsule workgroup holds in LDS (two float4 each)
constexpr int kStageCaps = 3072;
// largest ring distance the acceleration build resolves (farther cells keep it)
constexpr int kRingMax = 16;

// Primitive parameters, precomputed on the host:
//   sphere   : c0 c1 c2 r
//   box      : c0 c1 c2 h0 h1 h2
//   capsule  : a0 a1 a2 ba0 ba1 ba2 1/|ba|^2 r
//   cylinder : a0 a1 a2 e0 e1 e2 L L/2 r          (e = unit axis)
//   torus    : c0 c1 c2 e0 e1 e2 R r              (e = unit axis)
//   cone     : a0 a1 a2 e0 e1 e2 L ra rb          (e = unit axis, L = |b - a|)
//   octahedron: c0 c1 c2 s
//   hexprism : c0 c1 c2 h hz R                    (R = 2h/sqrt 3)
//   ellipsoid: c0 c1 c2 1/rx 1/ry 1/rz rmin
// A primitive may be placed (local = m (p - t), m = R^T / s, distance times
// s).  In its own frame the query point is taken to the nearest of the
// repeated copies (offsets (i - (n-1)/2) rep_c, i = 0..n-1 per axis),
// untwisted about z and elongated (q - clamp(q, -elong, elong)); the shape's
// distance there is rounded, made an onion shell and displaced (plus
// disp_a sin(f x) sin(f y) sin(f z) at the unelongated point, times
// disp_inv_lip = 1/(1 + disp_a disp_f sqrt 3)).  Twist: inside the bounding
// cylinder (radius twist_rho, z in twist_zc -/+ twist_zh) the distance is
// multiplied by inv_lip = 1/sqrt(1 + (twist_k twist_rho)^2), outside it the
// distance to the cylinder is used.  Repetition: the smaller of that and
// rep_gap plus the distance to the nearest cell face with another copy
// behind it.  flags = 0: the plain shape.
// kBent (with kTwisted): the turn about the local z axis follows x, not z
enum PrimFlags { kPlaced = 1, kTwisted = 2, kModified = 4, kRepeated = 8, kFurtherShape = 16, kBent = 32 };
template <typename T>
struct Prim {
  int32_t kind;
  int32_t flags;
  T v[10];
  T m[9], t[3], s;
  T round_r, onion_t;
  T twist_k, twist_rho, twist_zc, twist_zh, inv_lip;
  T elong[3], disp_a, disp_f, disp_inv_lip;
  T rep_c[3], rep_gap;
  int32_t rep_n[3], pad;
  double box_lo[3], box_hi[3];  // world box, for the acceleration build
};
using PrimD = Prim<double>;
using PrimF = Prim<float>;

struct Region {
  int32_t first, count, op;       // primitive range (region order) and CSG op
  int32_t seg;                    // SegRule: union or intersection of plain convex
                                  // primitives, or a subtraction from one
  double k, inv_k;                // smooth-union radius
  double mua, mus, mut, inv_mut;  // inv_mut = 0 for the ambient slot
  double absorb;                  // mua / mut
  double g, n;
  // HG constants: 1 + g^2, 1 - g^2, 1 - g, 2g, 1/(2g); iso = |g| < 1e-6
  double hg_a, hg_b, hg_c, hg_d, hg_e;
  int32_t iso, pad2;
  float kf, inv_kf, mutf, inv_mutf, gf, hg_af, hg_bf, hg_cf, hg_df, hg_ef;
};

// Uniform-grid acceleration of one union region with many primitives (the
// space partitioning proposed in Sec. 5 against evaluating every SDF at every
// step).  Cell c lists the primitives whose bounding box grown by `margin`
// overlaps c; a query returns min(margin, min over the listed primitives),
// which equals the region SDF wherever that is below margin and is a lower
// bound elsewhere.  A cell that lists none also has its Chebyshev distance
// in cells to the nearest cell that lists one (kRingMax at most): every
// surface point lies in a cell that lists its primitive, so there the query
// returns (distance - 1) whole cells plus the way to the cell's own faces,
// when that is more than the margin.  Built on the device into the engine's
// accel buffers.
struct Accel {
  int32_t region;                 // accelerated region, -1 = none
  int32_t dims[3];
  int32_t n_cells, first_prim, n_prims;
  // 1: every primitive of the region is a plain capsule, also stored as a
  // compact record (a, b - a, 1/|b - a|^2, r: 8 values, FP64 and FP32
  // copies at cap_offset_d / cap_offset_f of the blob, region order)
  int32_t caps;
  uint64_t cap_offset_d, cap_offset_f;
  uint64_t capacity;              // entries the id list can hold
  double lo[3], inv_cell[3], margin;
  double cell_min;                // the smallest cell side
  double box_lo[3], box_hi[3];    // bounding box of the region's primitives
  float lof[3], inv_cellf[3], marginf, cell_minf;
  float box_lof[3], box_hif[3];
};

struct SceneHeader {
  int32_t n_prims, n_regions;     // the ambient medium is region slot n_regions
  int32_t has_grid, src_kind;
  int32_t g_dims[3], m_survive;
  int32_t max_steps, geometry;    // steps per event: sphere-tracing steps or voxel faces
  int64_t max_events;
  double delta, h_normal, snap_cos, offset;  // surface threshold and surface-step constants
  double bb_c[3], bb_h[3];        // simulation volume (centre, half extents)
  float bb_cf[3], bb_hf[3];
  double g_lo[3], g_inv_d[3], g_d[3], g_hi[3];
  float g_lof[3], g_inv_df[3], g_df[3], g_hif[3];
  double src[8];
  // escape image: face 2*axis + side, pixels over [det_lo, det_hi] in the
  // face's two other axes (increasing axis order, first fastest); det_face
  // -1 = none
  int32_t det_face, det_dims[2];
  int32_t xf;                     // some primitive is placed or modified
  double det_lo[2], det_hi[2];
  double w_threshold, m_d, inv_m;
  float deltaf, relaxf;
  // over-relaxed sphere tracing: factor omega and 2 - omega
  double relax, relax_k;
  float relax_kf;
  // segment-traced steps (kLaunchSegment jobs): a bound on the rounding of
  // a primitive's distance, 16 units in the last place of the largest
  // coordinate of the volume and the primitives
  float seg_errf;
  double seg_err;
  int32_t segment, pad_seg;
  // ambient skip: a box holding each region's surface (the union of its
  // primitives' world boxes, grown by the smooth-union radius and half of
  // delta; the FP32 copy rounded outwards)
  double amb_lo[kMaxRegions][3], amb_hi[kMaxRegions][3];
  float amb_lof[kMaxRegions][3], amb_hif[kMaxRegions][3];
  Region reg[kMaxRegions + 1];
  Accel acc;
  uint64_t prim_offset_d, prim_offset_f;  // byte offsets of the tables in the blob
  uint64_t blob_bytes;
};

// Launch configuration chosen by the host.
struct LaunchCfg {
  int block;          // threads per workgroup
  int grid;           // workgroups
  int refill_min;     // dead lanes gathered before a wave emits
  int surface_min;    // lanes gathered before a wave runs the interface step
};

// Per-run device arguments of the walk kernel.
struct WalkArgs {
  const SceneHeader* sc;
  const PrimD* pd;
  const PrimF* pf;
  uint64_t seed, first, n;
  unsigned long long* counter;   // packets of this job handed out so far (zeroed before launch)
  double* fluence;               // nx*ny*nz, may be null
  double* absorbed;              // n_regions
  const uint32_t* acc_offsets;   // n_cells + 1 (accelerated scenes)
  const uint32_t* acc_ids;       // capacity
  const uint32_t* acc_rings;     // n_cells: 0 for a cell that lists primitives, else
                                 // its Chebyshev distance to one in cells (<= kRingMax)
  void* tallies;                 // smcrt_tallies
  // trace mode
  const uint64_t* trace_ids;
  void* trace_out;
  int32_t* trace_count;
  int32_t n_trace, max_records;
  int32_t acc_region;            // copy of sc->acc.region (-1 = none)
  int32_t geometry;              // launch class: sc->geometry, plus kLaunchXf when sc->xf
  int32_t brick, pad_brick;      // 1: fluence is the 2x2x2-brick scratch grid (brick_index)
  const double* acc_capd;        // compact capsule records of the accelerated region
  const float* acc_capf;         //   (8 values each), or null when acc.caps = 0
  // resident serving: packets of this job saved at the end of the previous
  // epoch (SavedPacket records of the launch's precision), taken through
  // resume_next before new ids; slot = the job's stable index, written into
  // the packets this launch saves
  const void* resume;
  unsigned int* resume_next;
  uint32_t resume_n;
  int32_t slot;
  uint8_t* vox;                  // voxel model: region slot per voxel (nx*ny*nz, x fastest)
  double* detector;              // escape image (det_dims[0] * det_dims[1]), may be null
};

// Arguments of one walk launch: a table of jobs in device memory.
struct BatchArgs {
  const WalkArgs* jobs;
  int32_t n_jobs;
  int32_t refill_min, surface_min;
  int32_t geometry;              // the launch takes only the jobs of this launch class
  // resident serving: a launch that runs for at most deadline ticks of the
  // device wall clock (0 = to the end) writes the packets still live then
  // to save (SavedPacket records, save_count of them, at most save_cap)
  uint64_t deadline;
  void* save;
  unsigned int* save_count;
  uint32_t save_cap;
  int32_t pad_save;
};

// A packet in flight at the end of a resident-serving epoch: its whole
// state (Packet<T> of the walk), the voxel of the voxel model, and the slot
// (job) it belongs to.  Stored at a fixed size for both precisions.
constexpr int kSavedPacketBytes = 256;

}  // namespace smcrt
