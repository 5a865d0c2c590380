/*
 * smcrt_oracle.h -- plain, slow FP64 CPU oracle of the SDF photon random walk
 * of McMillan, Bruce & Dholakia, "Meshless Monte Carlo Radiation Transfer
 * Method for Curved Geometries using Signed Distance Functions" (2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper
 * with the GPU path.
 *
 * Units: lengths in cm, coefficients in 1/cm.  Every double is IEEE FP64.
 */
#ifndef SMCRT_ORACLE_H
#define SMCRT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* primitive kinds (Sec. 2.2, Eq. 3 for the sphere; box, capsule, capped
 * cylinder and torus are basic shapes of the Sec. 2.2 gallery) */
enum { ORC_SPHERE = 0, ORC_BOX = 1, ORC_CAPSULE = 2, ORC_CYLINDER = 3, ORC_TORUS = 4,
       ORC_CONE = 5, ORC_OCTAHEDRON = 6, ORC_HEXPRISM = 7, ORC_ELLIPSOID = 8 };
/* CSG operators (Sec. 2.2: union, intersection and difference; gallery
 * panels e to h) */
enum { ORC_UNION = 0, ORC_SMOOTH_UNION = 1, ORC_INTERSECT = 2, ORC_SUBTRACT = 3 };
/* photon sources */
enum { ORC_SRC_POINT = 0, ORC_SRC_PENCIL = 1, ORC_SRC_DISC = 2, ORC_SRC_RECT = 3 };
/* trace record types */
enum {
  ORC_EV_EMIT = 0, ORC_EV_SCATTER = 1, ORC_EV_ABSORB = 2, ORC_EV_KILL = 3,
  ORC_EV_REFLECT = 4, ORC_EV_REFRACT = 5, ORC_EV_CROSS = 6, ORC_EV_ESCAPE = 7,
  ORC_EV_STALL = 8
};

/* sphere: c[3], r | box: c[3], half[3] | capsule and capped cylinder: a[3], b[3], r
 * | torus: c[3], axis[3] (any length), R (ring radius), r (tube radius) */
/* A primitive is defined in its own frame by p[] and placed in the world by
 * x_world = s * R x_local + t (rotation R, uniform scale s > 0).  In the
 * local frame the query point q is, in this order: repeated (copies of the
 * shape at offsets (i - (n-1)/2) * rep_c per axis, i = 0..n-1, q taken to
 * the nearest copy), untwisted (angle -twist_k * z about z) or unbent
 * (angle -twist_k * x about z), and elongated (q - clamp(q, -elong,
 * elong)).  The distance of the shape there is rounded (minus round_r),
 * made an onion shell (|d| - onion_t) and displaced (plus disp_a *
 * sin(f q0x) sin(f q0y) sin(f q0z), q0 the point before elongation,
 * divided by 1 + disp_a disp_f sqrt(3)).  A twist or a bend stretches
 * distances: inside the bounding cylinder about z (radius twist_rho, z in
 * [twist_zlo, twist_zhi]; a turn about z keeps the distance from the axis)
 * the distance is divided by the map's Lipschitz bound there, with
 * kr = |twist_k| twist_rho: (kr + sqrt(kr^2 + 4)) / 2 for a twist, 1 + kr
 * for a bend; outside it, the distance to that cylinder is used.  A
 * repeated shape takes the smaller of its copy's distance and rep_gap plus
 * the distance to the nearest face of its copy's cell shared with another
 * copy.  flags: bit 0 transform, bit 1 twist, bit 2 repetition, bit 3 bend
 * (with bit 1: the turn angle follows x instead of z). */
typedef struct {
  int32_t kind;
  int32_t flags;
  double p[8];
  double rot[9];                  /* R, row-major (local -> world) */
  double t[3], s;
  double round_r, onion_t;
  double twist_k, twist_rho, twist_zlo, twist_zhi;
  double elong[3];
  double disp_a, disp_f;
  double rep_c[3];
  int32_t rep_n[3], pad;
  double rep_gap;
} orc_prim;

typedef struct {
  int32_t first_prim, n_prims, op, pad;
  double k;                       /* smooth-union radius (cm) */
  double mua, mus, g, n;          /* optical properties (Sec. 2.3) */
  /* a box holding the region's surface: the union of its primitives'
   * boxes, grown by the smooth-union radius and half of delta (ambient skip) */
  double box_lo[3], box_hi[3];
} orc_region;

typedef struct {
  int32_t n_prims, n_regions;
  const orc_prim* prims;
  const orc_region* regions;
  double n_ambient;               /* refractive index outside every region */
  double delta;                   /* sphere-tracing surface threshold (cm) */
  double bb_lo[3], bb_hi[3];      /* simulation volume (escape when outside) */
  double g_lo[3], g_hi[3];        /* fluence grid extent */
  int32_t g_dims[3];              /* voxels per axis; 0 in any axis = no grid */
  int32_t src_kind;
  double src[8];
  double w_threshold;             /* roulette threshold on the packet weight */
  int32_t m_survive;              /* survive with probability 1/m, weight * m */
  int32_t max_steps;              /* sphere-tracing steps allowed per event */
  int64_t max_events;             /* events allowed per packet */
  /* escape image: face 2*axis + side of the simulation volume (of the grid
   * in the voxel model), pixels over [det_lo, det_hi] in the face's two
   * other axes (increasing axis order, first fastest); det_dims 0 = none */
  int32_t det_face;
  int32_t det_dims[2];
  double det_lo[2], det_hi[2];
  /* over-relaxation factor of sphere-tracing steps in [1, 2); 1 = plain
   * steps of the nearest-surface distance */
  double relax;
  /* The plain march (reuse = skip = 0, relax = 1) is the default walk.  The
   * switches below select the step-count mirror of the kernels' shortcuts,
   * used only where a pin or a test compares numbers of SDF evaluations:
   * 1: free-flight reuse (no new evaluation for an interaction inside the
   * last evaluated free ball) */
  int32_t reuse;
  /* 1: ambient skip (outside every region, move to the first region box
   * the ray enters in one move) */
  int32_t skip;
  /* 1: segment-traced steps (outside a region built of plain convex
   * primitives, the ray is free up to the tangent bounds of its members);
   * excludes relax > 1 */
  int32_t segment;
  int32_t pad_segment;
} orc_scene;

/* Segment bound of region r at p along the unit direction u (segment
 * tracing): no surface of the region lies on the ray closer than the value
 * returned.  Exposed for the pins. */
double orc_segment_bound(const orc_scene* s, int r, const double p[3], const double u[3]);

/* free-flight reuse: at most this many interactions per evaluation */
#define ORC_REUSE_LINKS 32

typedef struct {
  double launched, escaped_face[6], roulette_gain, roulette_loss, stalled;
  uint64_t events, steps, interactions, interfaces, reflections, refractions,
           crossings, advances, voxel_segments, kills, stalls, escapes;
} orc_tallies;

typedef struct {
  uint32_t event, type;
  int32_t region, pad;
  double p[3], u[3], w, tau;
} orc_event;

/* one Philox4x32-10 block (Salmon et al., SC'11) */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* the uniform variate (0,1) that a 32-bit word maps to */
double orc_xi(uint32_t x);

double orc_prim_sdf(const orc_prim* pr, const double p[3]);
double orc_smooth_union(double a, double b, double k);
double orc_region_sdf(const orc_scene* s, int r, const double p[3]);
int orc_region_of(const orc_scene* s, const double p[3]);
void orc_region_normal(const orc_scene* s, int r, const double p[3], double h, double n[3]);
double orc_box_sdf(const double lo[3], const double hi[3], const double p[3]);

/* unpolarised Fresnel reflectance; *cos_t gets the transmitted cosine
 * (0 under total internal reflection, where R = 1) */
double orc_fresnel(double n1, double n2, double cos_i, double* cos_t);
double orc_hg_cos(double g, double xi);
void orc_rotate(double u[3], double cos_t, double phi);

/* adds w * (path length in voxel v) to f[v] for the straight segment a->b;
 * returns the number of voxel pieces */
int64_t orc_tally_segment(const orc_scene* s, const double a[3], const double b[3],
                          double w, double* f);

/* whole-run entry: packets [first, first+n); f (nx*ny*nz, x fastest),
 * absorbed (n_regions) and t are accumulated into (+=).  Returns 0 or a
 * negative error code. */
int orc_run(const orc_scene* s, uint64_t seed, uint64_t first, uint64_t n,
            int n_threads, double* f, double* absorbed, orc_tallies* t);

/* as orc_run (voxel = 0) or orc_run_voxel (voxel = 1), with the escape
 * image accumulated into image (det_dims[0] * det_dims[1]; may be NULL) */
int orc_run_ex(const orc_scene* s, uint64_t seed, uint64_t first, uint64_t n, int n_threads, int voxel,
               double* f, double* absorbed, double* image, orc_tallies* t);

/* event records of one packet; returns the number written (<= cap) */
int orc_trace(const orc_scene* s, uint64_t seed, uint64_t pid, int cap, orc_event* out);

/* voxel-geometry model (the paper's comparison model): region per voxel of
 * the fluence grid at its centre; vox receives nx*ny*nz region indices
 * (-1 ambient).  orc_run_voxel / orc_trace_voxel walk packets through that
 * voxel grid with the same emission, interaction and RNG protocol. */
void orc_voxelize(const orc_scene* s, int8_t* vox);
int orc_run_voxel(const orc_scene* s, uint64_t seed, uint64_t first, uint64_t n, int n_threads, double* f,
                  double* absorbed, orc_tallies* t);
int orc_trace_voxel(const orc_scene* s, uint64_t seed, uint64_t pid, int cap, orc_event* out);

#ifdef __cplusplus
}
#endif
#endif
