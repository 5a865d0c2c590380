/*
 * smcrt.h -- C ABI of libsmcrt, an MI355X (gfx950) implementation of the
 * signed-distance-function photon random walk of McMillan, Bruce &
 * Dholakia, "Meshless Monte Carlo Radiation Transfer Method for Curved
 * Geometries using Signed Distance Functions" (2021).
 *
 * Conventions
 *  - Lengths in cm, attenuation coefficients in 1/cm, angles implicit.
 *  - Every call returns an smcrt_status; 0 is success, negatives are
 *    errors and smcrt_last_error() holds a message for the calling thread.
 *    No C++ exception crosses this boundary.
 *  - Arguments are validated on the host before any device work is queued;
 *    an invalid call queues nothing.
 *  - "Device pointer" means memory on the engine's device (hipMalloc or a
 *    torch CUDA tensor); "host pointer" means ordinary process memory.
 *  - Outputs are owned by the caller, live on the device, are zeroed by the
 *    caller and are ACCUMULATED into (+=), so runs over disjoint packet
 *    ranges add up (resume, split runs, sharding).
 *  - Streams are the caller's HIP streams (hipStream_t passed as void*;
 *    NULL = the null stream).  Runs are asynchronous on that stream; the
 *    caller synchronises before reading outputs.
 */
#ifndef SMCRT_H
#define SMCRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMCRT_ABI_VERSION 1

typedef enum {
  SMCRT_OK = 0,
  SMCRT_E_INVALID = -1,   /* an argument or scene is invalid (message says which) */
  SMCRT_E_NOMEM = -2,     /* host or device allocation failed */
  SMCRT_E_HIP = -3,       /* a HIP runtime call failed */
  SMCRT_E_BUDGET = -4,    /* a request can never fit the engine's memory budget */
  SMCRT_E_CANCELLED = -5, /* the request was cancelled */
  SMCRT_E_STATE = -6      /* the call is not valid in the object's current state */
} smcrt_status;

/* message of the last failed call on this thread ("" if none) */
const char* smcrt_last_error(void);
int smcrt_abi_version(void);

/* ------------------------------------------------------------ scenes ---- */
/* Geometry initialisation (Sec. 2.3): pick SDF primitives, combine them with
 * CSG operators into regions, give each region its optical properties
 * (mu_a, mu_s, n, g), and bound everything with a box.  Scenes are
 * host-side objects owned by the library. */

typedef struct smcrt_scene smcrt_scene;

enum {
  SMCRT_PRIM_SPHERE = 0,   /* params: cx cy cz r           (Eq. 3)              */
  SMCRT_PRIM_BOX = 1,      /* params: cx cy cz hx hy hz    (axis aligned, half extents) */
  SMCRT_PRIM_CAPSULE = 2,  /* params: ax ay az bx by bz r  (segment a-b swept by r) */
  SMCRT_PRIM_CYLINDER = 3, /* params: ax ay az bx by bz r  (axis a-b, flat caps) */
  SMCRT_PRIM_TORUS = 4,    /* params: cx cy cz ex ey ez R r (centre, axis of any length,
                                      ring radius R >= 0, tube radius r > 0) */
  /* further gallery shapes (Sec. 2.2, Fig. 1's basic shapes) */
  SMCRT_PRIM_CONE = 5,     /* params: ax ay az bx by bz ra rb (frustum about a-b, radius
                                      ra at a, rb at b, both >= 0, not both 0; exact) */
  SMCRT_PRIM_OCTAHEDRON = 6, /* params: cx cy cz s          (|x|+|y|+|z| <= s; exact) */
  SMCRT_PRIM_HEXPRISM = 7, /* params: cx cy cz h hz       (regular hexagon of apothem h in
                                      the xy plane, vertices on the x axis, extruded
                                      over z in cz -/+ hz; exact) */
  SMCRT_PRIM_ELLIPSOID = 8 /* params: cx cy cz rx ry rz   (radii > 0; distance bound
                                      min(r) (|(p - c)/r| - 1): exact sign, never more
                                      than the distance) */
};
/* region operators over the region's primitives, in the order given
 * (Sec. 2.2: union, intersection and difference):
 *   UNION min; SMOOTH_UNION polynomial smooth minimum of radius k;
 *   INTERSECT max; SUBTRACT the first primitive minus all the others,
 *   max(d_first, -d_i).  INTERSECT and SUBTRACT give lower bounds of the
 *   distance with Lipschitz constant 1 and the exact sign, which keeps
 *   sphere tracing conservative. */
enum { SMCRT_OP_UNION = 0, SMCRT_OP_SMOOTH_UNION = 1, SMCRT_OP_INTERSECT = 2, SMCRT_OP_SUBTRACT = 3 };
enum {
  SMCRT_SRC_POINT = 0,   /* params: x y z                    isotropic point source */
  SMCRT_SRC_PENCIL = 1,  /* params: x y z ux uy uz           collimated beam */
  SMCRT_SRC_DISC = 2,    /* params: cx cy cz R ux uy uz      top-hat disc in a z-plane */
  SMCRT_SRC_RECT = 3     /* params: cx cy cz hx hy ux uy uz  uniform z-plane rectangle */
};

/* n_ambient: refractive index outside every region (> 0).
 * delta: sphere-tracing surface threshold in cm (Sec. 2.3; > 0).
 * pad: padding of the simulation volume in cm (>= 0). */
smcrt_status smcrt_scene_create(smcrt_scene** out, double n_ambient, double delta, double pad);
smcrt_status smcrt_scene_destroy(smcrt_scene* scene);

/* Adds a primitive (Sec. 2.2).  params: host array of n_params doubles laid
 * out as listed above; radii and half extents > 0, capsule/cylinder ends
 * distinct, torus axis non-zero.  *out_prim receives its index. */
smcrt_status smcrt_scene_add_primitive(smcrt_scene* scene, int kind, const double* params,
                                       int n_params, int32_t* out_prim);

/* Adds a region: the listed primitives combined by op (SMCRT_OP_*; smooth
 * union takes its radius k_cm > 0, the others ignore k_cm), with absorption
 * mu_a >= 0 and scattering mu_s >= 0
 * (mu_a + mu_s > 0), Henyey-Greenstein anisotropy -1 < g < 1 and refractive
 * index n > 0 (Sec. 2.3: one property set per SDF).  Where regions overlap
 * the one added later owns the point.  prims: host array of n_prims indices. */
smcrt_status smcrt_scene_add_region(smcrt_scene* scene, const int32_t* prims, int n_prims, int op,
                                    double k_cm, double mu_a, double mu_s, double g, double n,
                                    int32_t* out_region);

/* Photon source (Sec. 3.1 uses isotropic point and incident beams).
 * Direction vectors are normalised by the library. */
smcrt_status smcrt_scene_set_source(smcrt_scene* scene, int kind, const double* params, int n_params);

/* Rectangular fluence grid (Sec. 3.1): box [lo, hi] cut into dims voxels,
 * voxel (i, j, k) at index i + nx*(j + ny*k).  Without this call the grid is
 * the regions' bounding box at 1x1x1; dims of 0 in any axis disable the
 * tally. */
smcrt_status smcrt_scene_set_grid(smcrt_scene* scene, const double lo[3], const double hi[3],
                                  const int32_t dims[3]);

/* Russian roulette: packets whose weight drops below w_threshold survive
 * with probability 1/m_survive and have their weight multiplied by
 * m_survive (defaults 1e-4 and 10). */
smcrt_status smcrt_scene_set_roulette(smcrt_scene* scene, double w_threshold, int32_t m_survive);

/* Safety caps: a packet that needs more than max_steps sphere-tracing steps
 * for one event, or more than max_events events, is ended and its weight
 * tallied as stalled (defaults 100000 and 1000000). */
smcrt_status smcrt_scene_set_limits(smcrt_scene* scene, int32_t max_steps, int64_t max_events);

/* Placement of primitive prim (Sec. 2.2: SDFs are translated, rotated and
 * scaled): its parameters are then read in its own frame, placed in the
 * world by x_world = scale * R x_local + trans.  rot: host array of 9, R
 * row-major, orthonormal to 1e-9 with determinant +1; scale > 0.  Distances
 * stay exact (times scale).  Errors: SMCRT_E_INVALID for an unknown
 * primitive, a non-rotation, scale <= 0 or non-finite values. */
smcrt_status smcrt_scene_set_primitive_placement(smcrt_scene* scene, int32_t prim, const double rot[9], double scale,
                                                 const double trans[3]);

/* Modifiers of primitive prim, in its own frame and in this order (Sec. 2.2
 * and its gallery: rounded, hollow and twisted shapes): rounding subtracts
 * round_r (>= 0) from the distance; an onion shell of half-thickness
 * onion_t > 0 replaces d by |d| - onion_t; a twist turns the shape about
 * the local z axis by twist_k * z radians.  Rounding and shell keep the
 * distance exact.  A twist keeps its sign only: inside the bounding
 * cylinder about the local z axis (radius 1.001 x the largest distance from
 * the axis of the primitive's local box grown by round_r + onion_t, z range
 * that box's grown by 0.1 % of its length at each end) the distance of the
 * untwisted shape is divided by (k rho + sqrt((k rho)^2 + 4)) / 2 with
 * k = |twist_k|, the untwist map's Lipschitz bound there (the largest
 * singular value of its Jacobian), and outside it the distance to that
 * cylinder is used, so
 * sphere tracing stays conservative.  Zeros remove the modifiers.  Errors:
 * SMCRT_E_INVALID for an unknown primitive, negative or non-finite values. */
smcrt_status smcrt_scene_set_primitive_modifiers(smcrt_scene* scene, int32_t prim, double round_r, double onion_t,
                                                 double twist_k);

/* Bend of primitive prim (Sec. 2.2 gallery: bent shapes): the shape turns
 * by bend_k * x radians about its local z axis at each x, so a rod along x
 * curves in the local x-y plane.  The sign is kept; inside the bounding
 * cylinder about the local z axis (as for a twist: a turn about z keeps the
 * distance from the axis) the distance of the unbent shape is divided by
 * 1 + |bend_k| rho, the unbend map's Lipschitz bound there (its Jacobian's
 * largest singular value, reached on the local y axis), and outside it the
 * distance to that cylinder is used.  0 removes the bend.  A primitive is
 * either twisted or bent.  Errors: SMCRT_E_INVALID for an unknown
 * primitive, a non-finite bend_k, or a bend of a twisted primitive (and
 * smcrt_scene_set_primitive_modifiers rejects a twist of a bent one). */
smcrt_status smcrt_scene_set_primitive_bend(smcrt_scene* scene, int32_t prim, double bend_k);

/* Elongation of primitive prim (gallery: stretched shapes): in its own
 * frame the point q is replaced by q - clamp(q, -h, h) before the shape is
 * evaluated, which stretches the shape by 2 h[i] along axis i (a sphere
 * becomes a capsule).  The result is exact outside and a lower bound with
 * the exact sign inside.  h: host array of 3, each finite and >= 0.
 * Errors: SMCRT_E_INVALID for an unknown primitive or a bad h. */
smcrt_status smcrt_scene_set_primitive_elongation(smcrt_scene* scene, int32_t prim, const double h[3]);

/* Displacement of primitive prim (gallery: bumpy shapes): amplitude *
 * sin(f x) sin(f y) sin(f z), at the point before elongation, is added to
 * the shape's distance after rounding and shell, and the sum is divided by
 * its Lipschitz bound 1 + amplitude * f * sqrt(3), so sphere tracing stays
 * conservative; the shape is the set where the sum is negative.  Errors:
 * SMCRT_E_INVALID for an unknown primitive, negative or non-finite values. */
smcrt_status smcrt_scene_set_primitive_displacement(smcrt_scene* scene, int32_t prim, double amplitude, double frequency);

/* Finite repetition of primitive prim (gallery: repeated shapes): counts[i]
 * copies along local axis i at offsets (k - (counts[i]-1)/2) * spacing[i],
 * k = 0..counts[i]-1.  A point is taken to the nearest copy; the distance is
 * the smaller of that copy's and the gap around a copy plus the distance
 * to the nearest face of its cell that another copy lies behind, a lower
 * bound with the exact sign.  Every copy (with its other modifiers, or its
 * twist's bounding cylinder) must fit inside its cell with a gap > 0.
 * counts in [1, 4096], spacing > 0.  Errors: SMCRT_E_INVALID for an unknown
 * primitive, bad values or copies that do not fit (also when a later
 * modifier makes them not fit: then the run fails). */
smcrt_status smcrt_scene_set_primitive_repetition(smcrt_scene* scene, int32_t prim, const double spacing[3],
                                                  const int32_t counts[3]);

/* Over-relaxed sphere tracing (Sec. 5 names faster marching as the remedy
 * for the many small steps of paths along surfaces).  With omega > 1 a step
 * may move omega times the nearest-surface distance d.  It is taken when it
 * would pass its check were the surface a plane met at the angle the
 * previous step of the same straight segment saw (the fall of d per unit
 * length); near a surface (d below delta/(2 - omega)) it never is.  The
 * next evaluation then checks it: the free
 * balls of radius d at its start and d' at its end must cover it, with
 * d + d' >= step + delta.  A step that fails goes back to the plain step of
 * d, so no surface is ever crossed unseen.  Events, tallies and fluence are
 * those of plain marching, up to rounding and the position of grazing
 * interface hits (within delta); only the step count changes.  omega in
 * [1, 2), default 1 (plain steps).  Errors: SMCRT_E_INVALID outside that
 * range. */
smcrt_status smcrt_scene_set_relaxation(smcrt_scene* scene, double omega);

/* Segment-traced steps (Sec. 5 names segment tracing, beside enhanced
 * sphere tracing, as a cure for the many small steps of paths along
 * surfaces).  Outside a convex shape the exact distance along the ray is a
 * convex function of the path length, so its tangent at the step's start
 * bounds the way to the shape from below: distance / rate of approach, and
 * no bound at all when the ray moves away.  With on = 1 every evaluation
 * also bounds, per region, the way along the ray to its surface: from
 * outside a union of plain spheres, boxes, capsules and capped cylinders
 * the smallest member bound, from outside an intersection of them the
 * largest, from outside a subtraction the bound of its first member when
 * that is such a shape; from inside a region, and for every other region
 * (smooth unions, tori), the distance alone.  A step then runs to the
 * nearest bound less delta (or delta past the volume's boundary) when that
 * is longer than the distance, and an interaction on that free way is taken
 * there.  Each bound is taken less the rounding of a distance (16 units in
 * the last place of the scene's largest coordinate), so no surface is
 * crossed unseen.  Events, tallies and fluence are those of plain marching
 * up to where in the delta band a surface is met, which moves interface
 * points by O(delta^2 curvature), by O(delta) for rays that meet a surface
 * at a grazing angle, and decides anew for rays that pass within delta of a
 * surface without crossing it.  on in {0, 1}, default 0.  Errors:
 * SMCRT_E_INVALID for another value or when the scene takes relaxed steps
 * (omega > 1: the two exclude each other); at run time, for a scene with
 * placed, modified or further primitives or the voxel geometry. */
smcrt_status smcrt_scene_set_segment_tracing(smcrt_scene* scene, int32_t on);

/* Uniform-grid acceleration of one union region (Sec. 5 proposes a
 * space-partitioning structure for large SDF collections).  The grid is the
 * box of the region's primitives grown by a margin of one cell, cut into
 * cells[0] x cells[1] x cells[2] cells (1..256 each); it is built on the
 * device at every run.  A step then evaluates only the primitives listed in
 * its cell and never steps further than the margin, so results match the
 * brute-force walk.  region = -1 removes the acceleration. */
smcrt_status smcrt_scene_set_accel(smcrt_scene* scene, int32_t region, const int32_t cells[3]);

/* Escape image: the light leaving through one face of the simulation volume
 * (of the fluence grid in the voxel model).  Sec. 3.2 and Sec. 5 single out
 * outputs at a single plane of interest as the case where the SDF walk
 * needs no voxel grid.  face = 2*axis + side: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z,
 * 5 +z.  A packet leaving through that face adds its weight to the pixel
 * holding the point where its straight path crosses the face's plane.  The
 * image spans [lo[0], hi[0]] x [lo[1], hi[1]] in the face's two other axes
 * in increasing order (x then y for a z face) with dims[0] x dims[1]
 * pixels, first axis fastest; dims of 0 remove the detector.  Errors:
 * SMCRT_E_INVALID for a face outside 0..5, lo >= hi, negative dims or
 * more than 2^31-1 pixels. */
smcrt_status smcrt_scene_set_detector(smcrt_scene* scene, int face, const double lo[2], const double hi[2],
                                      const int32_t dims[2]);

/* Geometry model.  Sec. 3 measures the SDF model against a voxelised one;
 * both run here on the same emission, interactions and random stream.
 *   SMCRT_GEOM_SDF (default): packets sphere-trace the region SDFs.
 *   SMCRT_GEOM_VOXEL: at every run the scene is first sampled onto its
 *     fluence grid (each voxel takes the region that owns its centre, as
 *     smcrt_voxelize returns) and packets move voxel face to voxel face;
 *     a face where the refractive index changes is a Fresnel interface with
 *     the face normal, beyond the grid lies the ambient medium, and a packet
 *     transmitted through a grid face escapes through it.  A packet born
 *     outside the grid travels to it unattenuated (escapes if it misses).
 *     Needs a grid set with dims >= 1 in every axis; the step cap of
 *     smcrt_scene_set_limits then counts voxel faces per event.
 * Errors: SMCRT_E_INVALID for an unknown mode. */
enum { SMCRT_GEOM_SDF = 0, SMCRT_GEOM_VOXEL = 1 };
smcrt_status smcrt_scene_set_geometry(smcrt_scene* scene, int mode);

/* number of regions and primitives; bounding box actually used */
smcrt_status smcrt_scene_info(const smcrt_scene* scene, int32_t* n_regions, int32_t* n_prims,
                              double bb_lo[3], double bb_hi[3]);

/* ------------------------------------------------------------ engine ---- */
/* An engine binds a device and owns its device-side staging (scene tables,
 * work counters).  Runs on one engine must not overlap in time: queue them
 * on one stream, or synchronise between streams. */

typedef struct smcrt_engine smcrt_engine;

smcrt_status smcrt_engine_create(smcrt_engine** out, int device);
smcrt_status smcrt_engine_destroy(smcrt_engine* engine);

enum { SMCRT_PREC_F32 = 0, SMCRT_PREC_F64 = 1 };

/* Launch options.  precision: F32 keeps positions, directions, distances and
 * transcendentals in FP32 (interface geometry, Fresnel, weights and tallies
 * stay FP64); F64 runs the whole walk in FP64.  block: threads per workgroup
 * (64, 128, 192 or 256).  blocks_per_cu: resident workgroups per CU the
 * grid is sized for (1..32; 0 = as many as fit).  refill_min: dead lanes a wave waits for
 * before it emits new packets (1..64).  surface_min: lanes a wave gathers at
 * surfaces before it runs the FP64 interface step (1..64).  Results do not
 * depend on any of these except precision. */
typedef struct {
  int32_t precision;
  int32_t block;
  int32_t blocks_per_cu;
  int32_t refill_min;
  int32_t surface_min;
  int32_t use_graph;    /* 1: capture the device work of a launch (grid builds,
                           counter reset, walk) in a hipGraph and replay it
                           while the launch shape is unchanged */
  int32_t tally_layout; /* 0: the library picks: FP32 SDF jobs whose voxels are
                           cubes (grids up to 2^27 voxels) tally into an
                           engine-owned grid of 2x2x2 bricks (the eight voxels
                           of a brick in one 64-byte segment, so neighbouring
                           voxels share atomic requests), added into the
                           caller's x-fastest grid after the walk; 1: always
                           tally into the caller's grid directly.  Results
                           agree to the order of FP64 sums. */
  int32_t no_stage;     /* 0: FP32 SDF jobs whose accelerated region is plain
                           capsules (at most 3072) run in workgroups of 1024
                           threads that hold the job's capsule records in LDS
                           (Sec. 5's grid queries then gather from LDS); 1:
                           they read the records from global memory.  Same
                           arithmetic, same results. */
} smcrt_opts;

smcrt_status smcrt_engine_get_opts(const smcrt_engine* engine, smcrt_opts* out);
smcrt_status smcrt_engine_set_opts(smcrt_engine* engine, const smcrt_opts* opts);

/* Autotuner: times runs of n_trial packets (>= 1000) of the scene under a
 * small grid of launch options -- block 256 or 128, as many workgroups per
 * CU as fit or one fewer, refill_min 1/4/16, surface_min 4/8/16 -- keeping
 * the engine's precision; then, from the fastest of these, the other
 * tally_layout where the scene's grid could take bricks and the other
 * no_stage where its capsules could be staged in LDS.  Sets the fastest
 * of all as the engine's options.
 * Synchronous; allocates and frees its own scratch outputs and stream.
 * out_best and out_packets_per_s (host, may be NULL) receive the winner. */
smcrt_status smcrt_engine_autotune(smcrt_engine* engine, const smcrt_scene* scene, uint64_t n_trial,
                                   smcrt_opts* out_best, double* out_packets_per_s);
/* The same search timed on one batched launch of n scenes (n_trial packets
 * each, n >= 1), for engines that run batches: the batch decides what one
 * scene cannot show (jobs sharing the device, their tables in the L2s).
 * out_packets_per_s counts the packets of all n jobs.  Errors as
 * smcrt_engine_autotune, and SMCRT_E_INVALID for a NULL scene or n < 1. */
smcrt_status smcrt_engine_autotune_batch(smcrt_engine* engine, int n, const smcrt_scene* const* scenes,
                                         uint64_t n_trial, smcrt_opts* out_best, double* out_packets_per_s);

/* ------------------------------------------------------------ tallies --- */

typedef struct {
  double launched;          /* packets emitted (unit weight each) */
  double escaped_face[6];   /* weight leaving the volume through -x,+x,-y,+y,-z,+z */
  double roulette_gain;     /* weight added by roulette survivors */
  double roulette_loss;     /* weight removed by roulette */
  double stalled;           /* weight of packets ended by the safety caps */
  uint64_t events;          /* interactions + interface events */
  uint64_t steps;           /* sphere-tracing steps */
  uint64_t interactions;
  uint64_t interfaces;      /* changes of medium met (reflect + refract + cross) */
  uint64_t reflections;
  uint64_t refractions;
  uint64_t crossings;       /* index-matched crossings */
  uint64_t advances;        /* forced advances past surfaces with no change of medium */
  uint64_t voxel_pieces;    /* voxel-sized pieces credited to the fluence grid */
  uint64_t kills;           /* roulette losses */
  uint64_t stalls;
  uint64_t escapes;
  uint64_t grid_atomics;    /* global FP64 atomic updates issued for the grid */
} smcrt_tallies;

/* ------------------------------------------------------------ runs ------ */

/* Runs packets [first_packet, first_packet + n_packets) of the scene with
 * random stream seed (Philox4x32-10 keyed by seed, counter by packet id and
 * event index, so results do not depend on the launch shape).
 *   d_fluence_raw: device, nx*ny*nz doubles, += sum of weight * path length
 *                  per voxel (cm).  NULL runs without the fluence tally (the
 *                  scalar tallies only; a voxel-geometry scene still walks
 *                  its grid): the tally-free regime of Sec. 3's speed test.
 *   d_absorbed:    device, n_regions doubles, += absorbed weight per region.
 *   d_tallies:     device, one smcrt_tallies, += scalar tallies.
 * Asynchronous on hip_stream. */
smcrt_status smcrt_run(smcrt_engine* engine, const smcrt_scene* scene, uint64_t seed,
                       uint64_t first_packet, uint64_t n_packets, double* d_fluence_raw,
                       double* d_absorbed, smcrt_tallies* d_tallies, void* hip_stream);

/* Batched runs: job j runs packets [first_packets[j], first_packets[j] +
 * n_packets[j]) of scenes[j] with seeds[j] into its own outputs, all jobs in
 * ONE persistent launch.  Waves spread over the jobs in proportion and move
 * to jobs with packets left when theirs are handed out, so many small scenes
 * fill the device together.  Host arrays of length n; first_packets may be
 * NULL (all 0); jobs with n_packets[j] = 0 are skipped; the same scene may
 * appear in several jobs.  Output rules as for smcrt_run (per job).  Each
 * job's result equals its smcrt_run alone up to FP64 summation order. */
smcrt_status smcrt_run_batch(smcrt_engine* engine, int n, const smcrt_scene* const* scenes, const uint64_t* seeds,
                             const uint64_t* first_packets, const uint64_t* n_packets, double* const* d_fluence_raw,
                             double* const* d_absorbed, smcrt_tallies* const* d_tallies, void* hip_stream);

/* Outputs of one job: caller-owned device buffers on the engine's device,
 * zeroed by the caller and accumulated into (+=).
 *   fluence_raw: as d_fluence_raw of smcrt_run (NULL: no fluence tally);
 *   absorbed, tallies: as d_absorbed and d_tallies of smcrt_run (required);
 *   detector: dims[0] * dims[1] doubles of the scene's escape image
 *             (smcrt_scene_set_detector), += escaped weight per pixel;
 *             NULL: no image. */
typedef struct {
  double* fluence_raw;
  double* absorbed;
  smcrt_tallies* tallies;
  double* detector;
} smcrt_outputs;

/* smcrt_run and smcrt_run_batch with the outputs of each job in one
 * smcrt_outputs (outs: host array of n for the batch). */
smcrt_status smcrt_run_ex(smcrt_engine* engine, const smcrt_scene* scene, uint64_t seed, uint64_t first_packet,
                          uint64_t n_packets, const smcrt_outputs* out, void* hip_stream);
smcrt_status smcrt_run_batch_ex(smcrt_engine* engine, int n, const smcrt_scene* const* scenes, const uint64_t* seeds,
                                const uint64_t* first_packets, const uint64_t* n_packets, const smcrt_outputs* outs,
                                void* hip_stream);

/* smcrt_run_ex for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc, hipFree or other allocating routine.
 * Its device scratch -- the scene's tables, the job record, the packet
 * counter, the uniform-grid build buffers and the voxel model's region
 * grid -- lives in a fixed array of 32 MiB that each GPU the library runs
 * on holds from its first use until the process ends; the walk tallies
 * straight into out->fluence_raw (no brick grid), so results equal
 * smcrt_run_ex's up to the order of FP64 sums.  The engine supplies the
 * device and launch options only.  Every call on one GPU shares that GPU's
 * scratch: calls that overlap on one GPU (on different streams, or from
 * different engines or threads) race and must be serialised by the caller.
 * The scene's packed tables are copied from host memory on hip_stream: the
 * scene must not change or be destroyed until that work has completed.
 * Errors: as smcrt_run_ex, and SMCRT_E_INVALID when the scene needs more
 * scratch than 32 MiB (e.g. a voxel-model grid above about 3.3e7 voxels, or
 * tables of about 6e4 primitives); nothing is queued then. */
smcrt_status smcrt_run_ex_static(smcrt_engine* engine, const smcrt_scene* scene, uint64_t seed, uint64_t first_packet,
                                 uint64_t n_packets, const smcrt_outputs* out, void* hip_stream);

/* Fluence normalisation: d_phi[v] = d_raw[v] / (launched * voxel volume),
 * in cm^-2 per launched unit weight.  d_raw and d_phi: device, nx*ny*nz
 * doubles (may alias). */
smcrt_status smcrt_normalize_fluence(const smcrt_scene* scene, const double* d_raw, double launched,
                                     double* d_phi, void* hip_stream);

/* ------------------------------------------------------------ serving --- */
/* Continuous batching of requests with device-resident state.  A server
 * owns an engine on `device` and a worker thread.  Requests are admitted in
 * arrival order, up to 128 at a time, while the device bytes they hold
 * (outputs, scene tables, grid buffers, voxel grid) fit the budget; an
 * admitted request keeps its tables and a packet-id counter on the device.
 * The worker runs epochs of a fixed length of device time (20 ms unless
 * smcrt_server_set_epoch_us says otherwise): one launch per kernel class in
 * which every resident request is a job; waves resume the packets the last
 * epoch left in flight, then take new ids, and when the epoch's time is up
 * the packets still in flight are saved whole to device memory and resumed
 * by the next epoch -- so requests arriving meanwhile join at the next
 * epoch without waiting for long packets to end.  Served requests tally
 * straight into their outputs.  A request is done when all its ids are
 * handed out and none of its packets is in flight; its outputs then equal
 * an smcrt_run of the same scene, seed and packets up to FP64 summation
 * order.  Beside the budget the server holds fixed device memory: two slabs
 * of 256 bytes per resident lane (one packet each) and small per-slot
 * tables.  Scenes and outputs are borrowed until the request is DONE,
 * FAILED or CANCELLED and must not change meanwhile.  device = -1 runs the
 * scheduler without a device (epochs in which every admitted request takes
 * its next epoch_packets / (admitted requests) ids, at least 1e4, and
 * completes at once; outputs untouched): a dry run for admission, ordering,
 * budget and cancellation.  Times are seconds since the server was
 * created. */

typedef struct smcrt_server smcrt_server;
enum { SMCRT_REQ_QUEUED = 0, SMCRT_REQ_RUNNING = 1, SMCRT_REQ_DONE = 2, SMCRT_REQ_FAILED = 3, SMCRT_REQ_CANCELLED = 4 };

typedef struct {
  uint64_t epochs, packets_done, queued, active, bytes_in_use;
  double busy_s, uptime_s;
  uint64_t in_flight;    /* packets saved at the end of the last epoch (device servers) */
  uint64_t saved_total;  /* packets saved at epoch ends so far, summed (each resumed later) */
} smcrt_server_info;

/* hbm_budget_bytes > 0; epoch_packets: dry runs only (0 = 2e6); opts NULL =
 * engine defaults */
smcrt_status smcrt_server_create(smcrt_server** out, int device, uint64_t hbm_budget_bytes,
                                 uint64_t epoch_packets, const smcrt_opts* opts);
/* cancels queued requests, finishes the running epoch, frees everything */
smcrt_status smcrt_server_destroy(smcrt_server* server);
/* SMCRT_E_BUDGET if the request alone exceeds the budget */
smcrt_status smcrt_submit(smcrt_server* server, const smcrt_scene* scene, uint64_t seed, uint64_t n_packets,
                          double* d_fluence_raw, double* d_absorbed, smcrt_tallies* d_tallies, uint64_t* out_request);
/* state SMCRT_REQ_*; times of submission, admission and completion (-1 = not yet) */
smcrt_status smcrt_poll(smcrt_server* server, uint64_t request, int* out_state, double* out_t_submit,
                        double* out_t_admit, double* out_t_done);
/* blocks until the request finishes (timeout_s < 0: no limit); returns its outcome */
smcrt_status smcrt_wait(smcrt_server* server, uint64_t request, double timeout_s);
/* queued: dropped; running: dropped at the end of the current epoch */
smcrt_status smcrt_cancel(smcrt_server* server, uint64_t request);
smcrt_status smcrt_server_stats(smcrt_server* server, smcrt_server_info* out);
/* length of a device epoch in microseconds of device time, 100 to 1e7
 * (default 20000): shorter epochs admit arrivals sooner, longer ones spend
 * less time between launches */
smcrt_status smcrt_server_set_epoch_us(smcrt_server* server, uint64_t epoch_us);

/* ------------------------------------------------------------ traces ---- */

enum {
  SMCRT_EV_EMIT = 0, SMCRT_EV_SCATTER = 1, SMCRT_EV_ABSORB = 2, SMCRT_EV_KILL = 3,
  SMCRT_EV_REFLECT = 4, SMCRT_EV_REFRACT = 5, SMCRT_EV_CROSS = 6, SMCRT_EV_ESCAPE = 7,
  SMCRT_EV_STALL = 8
};

typedef struct {
  uint32_t event;   /* event index (0 = emission) */
  uint32_t type;    /* SMCRT_EV_* */
  int32_t region;   /* region after the event (-1 = ambient) */
  int32_t pad;
  double p[3], u[3], w, tau;  /* state after the event */
} smcrt_event;

/* Event-by-event records of the listed packets through the same device walk
 * as smcrt_run (with recording compiled in).  d_packet_ids: device, n_ids
 * uint64.  d_out: device, n_ids * max_events records; packet i writes its
 * first max_events records from d_out[i * max_events]; d_count: device,
 * n_ids int32 record counts.  No fluence is tallied. */
smcrt_status smcrt_trace(smcrt_engine* engine, const smcrt_scene* scene, uint64_t seed,
                         const uint64_t* d_packet_ids, int n_ids, int max_events,
                         smcrt_event* d_out, int32_t* d_count, void* hip_stream);

/* The voxelised geometry of Sec. 3: the region owning each voxel centre of
 * the scene's fluence grid, from the FP64 region SDFs (the highest-index
 * region whose SDF is negative, else the ambient medium).  d_out: device,
 * nx*ny*nz bytes, x fastest; each byte is a region index, or n_regions for
 * the ambient medium.  Asynchronous on hip_stream; the caller owns d_out.
 * Errors: SMCRT_E_INVALID without a grid (dims >= 1 in every axis) or with
 * a NULL argument; SMCRT_E_HIP on a device failure. */
smcrt_status smcrt_voxelize(smcrt_engine* engine, const smcrt_scene* scene, uint8_t* d_out, void* hip_stream);

/* Point queries of the scene SDF (Sec. 2.2: the primitives' distances,
 * Eq. 3 for the sphere, their placement and modifiers, and each region's
 * CSG of them), by the device functions the walk steps with, in the
 * engine's precision (FP32 engines evaluate at the points rounded to
 * float).  d_points: device, n x 3 doubles (x, y, z per point).  d_dist:
 * device, n x n_regions doubles, one row per point, region order.
 * accelerated: 0 = every region's SDF from all its primitives; 1 = the
 * accelerated region (smcrt_scene_set_accel) through its uniform grid, the
 * lower bound the walk steps by (equal to the SDF within the grid's margin
 * of a surface).  d_owner (device, may be NULL): n int32, the highest-index
 * region whose distance is negative, else n_regions (ambient), as the walk
 * assigns regions.  d_normals (device, may be NULL): n x n_regions x 3
 * doubles, each region's unit normal at the point by the interface step's
 * FP64 central differences (Sec. 1: normals by numerical differentiation;
 * step delta/100), through the grid when accelerated.  n = 0 does nothing.
 * Asynchronous on hip_stream; the caller owns the buffers.  Errors:
 * SMCRT_E_INVALID for a NULL engine, scene, d_points or d_dist (n > 0),
 * accelerated outside {0, 1}, or an incomplete scene; SMCRT_E_HIP on a
 * device failure. */
smcrt_status smcrt_scene_distance(smcrt_engine* engine, const smcrt_scene* scene, const double* d_points, uint64_t n,
                                  int32_t accelerated, double* d_dist, int32_t* d_owner, double* d_normals,
                                  void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
