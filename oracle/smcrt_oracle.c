/*
 * smcrt_oracle.c -- plain FP64 CPU oracle of the SDF photon random walk.
 *
 * TEST INFRASTRUCTURE ONLY (see smcrt_oracle.h).  Written for a reader to
 * check against the paper by eye: no acceleration structure, no blocking,
 * no merging of path segments, brute-force evaluation of every SDF at every
 * step (Sec. 2.3), a tally that finds voxel pieces by intersecting the
 * segment with every voxel plane it spans, and OpenMP over packets with
 * per-thread accumulators reduced in thread order.
 *
 * walk_plain is the walk: the step loop of Sec. 2.3 and nothing else.  A
 * second walk, walk_mirror, takes the same steps through the shortcuts the
 * kernels take -- free-flight reuse, the ambient skip, over-relaxed steps
 * and segment-traced steps (both named in Sec. 5) -- and runs only when a
 * scene asks for one of them (orc_scene.reuse, .skip, .segment, .relax > 1):
 * pins compare its events and tallies with walk_plain's, and tests that
 * count SDF evaluations use its step counts.  Every other comparison is
 * against walk_plain.
 *
 * Where the paper is silent the code follows the readings listed in the
 * repository's design notes; each such place says "reading:".
 */
#include "smcrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_INF (1.0 / 0.0)
/* reading: a surface hit is found by snapping along the ray when the ray
 * meets the surface at a cosine of at least this, else by projecting along
 * the normal */
#define ORC_SNAP_COS 0.1
/* reading: probe distance across a surface, re-placement distance and the
 * forced advance past a surface that is not a physical interface, in units
 * of the threshold delta */
#define ORC_OFFSET 2.0
/* reading: central-difference step of the numerical normal, in units of delta */
#define ORC_H_NORMAL 1e-2

/* ---------------------------------------------------------------- RNG --- */

/* Philox4x32-10: ten rounds of the Philox S-box with multipliers
 * 0xD2511F53 and 0xCD9E8D57 and Weyl key increments 0x9E3779B9, 0xBB67AE85
 * (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2,
 * 3", SC'11).  The key is bumped before every round except the first. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* reading of Eq. 1's "xi in [0, 1]": the top 23 bits m of the word give
 * xi = (m + 1/2) / 2^23, strictly inside (0, 1) and exact in FP32 and FP64 */
double orc_xi(uint32_t x) {
  return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* the four variates of event k of packet pid */
static void event_xi(uint64_t seed, uint64_t pid, uint32_t k, double xi[4]) {
  uint32_t ctr[4] = {k, (uint32_t)pid, (uint32_t)(pid >> 32), 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  for (int i = 0; i < 4; ++i) xi[i] = orc_xi(w[i]);
}

/* ------------------------------------------------------------ vectors --- */

static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double len3(const double a[3]) { return sqrt(dot3(a, a)); }
static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }
static double maxd(double a, double b) { return a > b ? a : b; }
static double mind(double a, double b) { return a < b ? a : b; }

/* --------------------------------------------------------------- SDFs --- */

/* distance from (x, y) to the segment (ax, ay)-(bx, by) */
static double seg2_dist(double x, double y, double ax, double ay, double bx, double by) {
  double dx = bx - ax, dy = by - ay, px = x - ax, py = y - ay;
  double t = clampd((px * dx + py * dy) / (dx * dx + dy * dy), 0.0, 1.0);
  double ex = px - t * dx, ey = py - t * dy;
  return sqrt(ex * ex + ey * ey);
}

/* distance from p to the segment a-b (3-D) */
static double seg3_dist(const double p[3], const double a[3], const double b[3]) {
  double ba[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, pa[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  double t = clampd(dot3(pa, ba) / dot3(ba, ba), 0.0, 1.0);
  double d[3] = {pa[0] - t * ba[0], pa[1] - t * ba[1], pa[2] - t * ba[2]};
  return len3(d);
}

/* Exact Euclidean distance functions, positive outside (Sec. 2.2, Eq. 2),
 * of the primitive shapes in their own frame. */
static double shape_sdf(const orc_prim* pr, const double p[3]) {
  const double* q = pr->p;
  switch (pr->kind) {
    case ORC_SPHERE: { /* Eq. 3: |p - c| - r */
      double d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
      return len3(d) - q[3];
    }
    case ORC_BOX: { /* distance to an axis-aligned box with half extents h */
      double e[3], out[3];
      for (int i = 0; i < 3; ++i) {
        e[i] = fabs(p[i] - q[i]) - q[3 + i];
        out[i] = maxd(e[i], 0.0);
      }
      double inside = mind(maxd(e[0], maxd(e[1], e[2])), 0.0);
      return len3(out) + inside;
    }
    case ORC_CAPSULE: { /* distance to the segment a-b, minus r */
      double ba[3] = {q[3] - q[0], q[4] - q[1], q[5] - q[2]};
      double pa[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
      double t = clampd(dot3(pa, ba) / dot3(ba, ba), 0.0, 1.0);
      double d[3] = {pa[0] - t * ba[0], pa[1] - t * ba[1], pa[2] - t * ba[2]};
      return len3(d) - q[6];
    }
    case ORC_CYLINDER: { /* solid cylinder of radius r about a-b, flat caps */
      double ba[3] = {q[3] - q[0], q[4] - q[1], q[5] - q[2]};
      double L = len3(ba);
      double e[3] = {ba[0] / L, ba[1] / L, ba[2] / L};
      double pa[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
      double x = dot3(pa, e);
      double radial[3] = {pa[0] - x * e[0], pa[1] - x * e[1], pa[2] - x * e[2]};
      double rho = len3(radial);
      double q1 = rho - q[6];
      double q2 = fabs(x - 0.5 * L) - 0.5 * L;
      double o1 = maxd(q1, 0.0), o2 = maxd(q2, 0.0);
      return mind(maxd(q1, q2), 0.0) + sqrt(o1 * o1 + o2 * o2);
    }
    case ORC_TORUS: { /* distance to the ring of radius R about the axis, minus r */
      double a[3] = {q[3], q[4], q[5]};
      double al = len3(a);
      double e[3] = {a[0] / al, a[1] / al, a[2] / al};
      double pc[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
      double x = dot3(pc, e);
      double radial[3] = {pc[0] - x * e[0], pc[1] - x * e[1], pc[2] - x * e[2]};
      double rho = len3(radial) - q[6];
      return sqrt(rho * rho + x * x) - q[7];
    }
    case ORC_CONE: { /* solid cone frustum about a-b, radius ra at a, rb at b:
                      * in the (axial x, radial y) half plane its boundary is
                      * the cap at a, the cap at b and the slanted side */
      double ba[3] = {q[3] - q[0], q[4] - q[1], q[5] - q[2]};
      double L = len3(ba);
      double e[3] = {ba[0] / L, ba[1] / L, ba[2] / L};
      double pa[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
      double x = dot3(pa, e);
      double radial[3] = {pa[0] - x * e[0], pa[1] - x * e[1], pa[2] - x * e[2]};
      double y = len3(radial), ra = q[6], rb = q[7];
      double d = mind(mind(seg2_dist(x, y, 0.0, 0.0, 0.0, ra), seg2_dist(x, y, L, 0.0, L, rb)),
                      seg2_dist(x, y, 0.0, ra, L, rb));
      int inside = x > 0.0 && x < L && y < ra + (rb - ra) * x / L;
      return inside ? -d : d;
    }
    case ORC_OCTAHEDRON: { /* |x|+|y|+|z| = s about c: by symmetry the face in
                            * the positive octant, a triangle with corners s e_i */
      const double sz = q[3];
      double a[3] = {fabs(p[0] - q[0]), fabs(p[1] - q[1]), fabs(p[2] - q[2])};
      double m = a[0] + a[1] + a[2] - sz;
      /* foot of the perpendicular on the face plane; inside the triangle
       * (all coordinates >= 0) the plane distance is the distance */
      double f[3] = {a[0] - m / 3.0, a[1] - m / 3.0, a[2] - m / 3.0};
      if (m <= 0.0 || (f[0] >= 0.0 && f[1] >= 0.0 && f[2] >= 0.0)) return m / sqrt(3.0);
      double v0[3] = {sz, 0, 0}, v1[3] = {0, sz, 0}, v2[3] = {0, 0, sz};
      return mind(mind(seg3_dist(a, v0, v1), seg3_dist(a, v1, v2)), seg3_dist(a, v2, v0));
    }
    case ORC_HEXPRISM: { /* regular hexagon of apothem h in the xy plane
                          * (vertices at angles 0, 60, ... deg) extruded over
                          * z in c -/+ hz */
      const double h = q[3], hz = q[4], R = 2.0 * h / sqrt(3.0);
      double x = fabs(p[0] - q[0]), y = fabs(p[1] - q[1]);
      /* first quadrant: the edges are (R, 0)-(R/2, h) and (R/2, h)-(-R/2, h) */
      double d2 = mind(seg2_dist(x, y, R, 0.0, 0.5 * R, h), seg2_dist(x, y, 0.5 * R, h, -0.5 * R, h));
      int in2 = y < h && sqrt(3.0) * x + y < 2.0 * h;  /* below the top edge and the slanted one */
      if (in2) d2 = -d2;
      double dz = fabs(p[2] - q[2]) - hz;
      double o1 = maxd(d2, 0.0), o2 = maxd(dz, 0.0);
      return mind(maxd(d2, dz), 0.0) + sqrt(o1 * o1 + o2 * o2);
    }
    case ORC_ELLIPSOID: { /* radii r about c: r_min (|(p - c)/r| - 1), which is
                           * 1-Lipschitz and zero on the surface, a lower
                           * bound of the distance with the exact sign */
      double rmin = mind(q[3], mind(q[4], q[5]));
      double u[3] = {(p[0] - q[0]) / q[3], (p[1] - q[1]) / q[4], (p[2] - q[2]) / q[5]};
      return rmin * (len3(u) - 1.0);
    }
    default:
      return ORC_INF;
  }
}

/* distance from p to the solid capped cylinder about the z axis, radius rho,
 * z in [zlo, zhi] (positive outside) */
static double zcyl_sdf(const double p[3], double rho, double zlo, double zhi) {
  double q1 = sqrt(p[0] * p[0] + p[1] * p[1]) - rho;
  double q2 = fabs(p[2] - 0.5 * (zlo + zhi)) - 0.5 * (zhi - zlo);
  double o1 = maxd(q1, 0.0), o2 = maxd(q2, 0.0);
  return mind(maxd(q1, q2), 0.0) + sqrt(o1 * o1 + o2 * o2);
}

/* Sec. 2.2: SDFs are translated, rotated, scaled, twisted and bent.  A
 * rigid motion with uniform scale s keeps a distance exact (times s);
 * rounding and an onion shell keep it exact; a twist or a bend keeps only
 * the sign.  The untwist map q(p) = (Rot(-k z)(x, y), z) has Jacobian Rot *
 * [[1, 0, -k y], [0, 1, k x], [0, 0, 1]], whose largest singular value at
 * radius rho is (k rho + sqrt((k rho)^2 + 4)) / 2.  The unbend map
 * q(p) = (Rot(-k x)(x, y), z) has Jacobian Rot * (I + k [[y, 0, 0],
 * [-x, 0, 0], [0, 0, 0]]), whose largest singular value is at most
 * 1 + k rho (reached at x = 0).  Inside a convex set whose points are
 * within rho of the z axis these bound the map's Lipschitz constant, and
 * the distance is divided by them there. */
double orc_prim_sdf(const orc_prim* pr, const double p[3]) {
  double q[3] = {p[0], p[1], p[2]};
  if (pr->flags & 1) { /* local = R^T (p - t) / s */
    const double* R = pr->rot;
    double d[3] = {p[0] - pr->t[0], p[1] - pr->t[1], p[2] - pr->t[2]};
    for (int i = 0; i < 3; ++i) q[i] = (R[i] * d[0] + R[3 + i] * d[1] + R[6 + i] * d[2]) / pr->s;
  }
  /* repetition: to the nearest copy; b = distance to the nearest face of
   * that copy's cell with another copy behind it */
  double b = ORC_INF;
  if (pr->flags & 4) {
    for (int a = 0; a < 3; ++a) {
      const int n = pr->rep_n[a];
      const double c = pr->rep_c[a], half = 0.5 * (n - 1) * c;
      /* clamp before converting: a far point must not overflow the int */
      const int i = (int)clampd(floor((q[a] + half) / c + 0.5), 0.0, (double)(n - 1));
      q[a] -= i * c - half;
      if (q[a] > 0.0 && i < n - 1) b = mind(b, 0.5 * c - q[a]);
      if (q[a] < 0.0 && i > 0) b = mind(b, 0.5 * c + q[a]);
    }
  }
  double d;
  double dcyl = 0.0;
  if (pr->flags & 2) {
    dcyl = zcyl_sdf(q, pr->twist_rho, pr->twist_zlo, pr->twist_zhi);
    /* untwist: rotate by -k z about z; unbend: by -k x */
    double a = -pr->twist_k * ((pr->flags & 8) ? q[0] : q[2]), c = cos(a), sn = sin(a);
    double u0 = c * q[0] - sn * q[1], u1 = sn * q[0] + c * q[1];
    q[0] = u0;
    q[1] = u1;
  }
  double e[3];
  for (int i = 0; i < 3; ++i) e[i] = q[i] - clampd(q[i], -pr->elong[i], pr->elong[i]);
  d = shape_sdf(pr, e) - pr->round_r;
  if (pr->onion_t > 0.0) d = fabs(d) - pr->onion_t;
  if (pr->disp_a > 0.0)
    d = (d + pr->disp_a * sin(pr->disp_f * q[0]) * sin(pr->disp_f * q[1]) * sin(pr->disp_f * q[2])) /
        (1.0 + pr->disp_a * pr->disp_f * sqrt(3.0));
  if (pr->flags & 2) {
    const double kr = fabs(pr->twist_k) * pr->twist_rho;
    d = dcyl > 0.0 ? dcyl : d / ((pr->flags & 8) ? 1.0 + kr : 0.5 * (kr + sqrt(kr * kr + 4.0)));
  }
  if (pr->flags & 4) d = mind(d, pr->rep_gap + b);
  return (pr->flags & 1) ? pr->s * d : d;
}

/* polynomial smooth minimum of radius k (Sec. 2.2 gallery, panel e):
 * equals min(a, b) when |a - b| >= k and is never above it */
double orc_smooth_union(double a, double b, double k) {
  double h = clampd(0.5 + 0.5 * (b - a) / k, 0.0, 1.0);
  return h * a + (1.0 - h) * b - k * h * (1.0 - h);
}

/* A region's SDF from its primitives, in their order:
 *   union min, smooth union folded left to right (reading 17),
 *   intersection max, difference max(d_first, -d_i) over the others
 *   (the first primitive minus all the others).
 * Intersection and difference give lower bounds of the true distance that
 * keep Lipschitz constant 1 and the correct sign, which is what sphere
 * tracing needs (Sec. 2.3). */
double orc_region_sdf(const orc_scene* s, int r, const double p[3]) {
  const orc_region* rg = &s->regions[r];
  double d = orc_prim_sdf(&s->prims[rg->first_prim], p);
  for (int i = 1; i < rg->n_prims; ++i) {
    double di = orc_prim_sdf(&s->prims[rg->first_prim + i], p);
    switch (rg->op) {
      case ORC_SMOOTH_UNION: d = orc_smooth_union(d, di, rg->k); break;
      case ORC_INTERSECT: d = maxd(d, di); break;
      case ORC_SUBTRACT: d = maxd(d, -di); break;
      default: d = mind(d, di); break;
    }
  }
  return d;
}

/* reading: a point belongs to the highest-index region whose SDF is
 * negative there; -1 (ambient) if none */
int orc_region_of(const orc_scene* s, const double p[3]) {
  for (int r = s->n_regions - 1; r >= 0; --r)
    if (orc_region_sdf(s, r, p) < 0.0) return r;
  return -1;
}

/* unit outward normal of region r at p by central differences (Sec. 1:
 * normals by numerical differentiation) */
void orc_region_normal(const orc_scene* s, int r, const double p[3], double h, double n[3]) {
  for (int i = 0; i < 3; ++i) {
    double a[3] = {p[0], p[1], p[2]}, b[3] = {p[0], p[1], p[2]};
    a[i] += h;
    b[i] -= h;
    n[i] = (orc_region_sdf(s, r, a) - orc_region_sdf(s, r, b)) / (2.0 * h);
  }
  double l = len3(n);
  for (int i = 0; i < 3; ++i) n[i] /= l;
}

/* signed distance of the simulation volume (Sec. 2.3: positive = outside) */
double orc_box_sdf(const double lo[3], const double hi[3], const double p[3]) {
  orc_prim b;
  memset(&b, 0, sizeof(b));
  b.kind = ORC_BOX;
  for (int i = 0; i < 3; ++i) {
    b.p[i] = 0.5 * (lo[i] + hi[i]);
    b.p[3 + i] = 0.5 * (hi[i] - lo[i]);
  }
  return shape_sdf(&b, p);
}

/* ------------------------------------------------------------ physics --- */

double orc_fresnel(double n1, double n2, double cos_i, double* cos_t) {
  double eta = n1 / n2;
  double sin2_t = eta * eta * (1.0 - cos_i * cos_i);
  if (sin2_t >= 1.0) { /* total internal reflection */
    *cos_t = 0.0;
    return 1.0;
  }
  double ct = sqrt(1.0 - sin2_t);
  double rs = (n1 * cos_i - n2 * ct) / (n1 * cos_i + n2 * ct);
  double rp = (n1 * ct - n2 * cos_i) / (n1 * ct + n2 * cos_i);
  *cos_t = ct;
  return 0.5 * (rs * rs + rp * rp);
}

/* Henyey-Greenstein scattering cosine by inversion of its CDF (Sec. 3.1);
 * isotropic when |g| < 1e-6 */
double orc_hg_cos(double g, double xi) {
  if (fabs(g) < 1e-6) return 2.0 * xi - 1.0;
  double frac = (1.0 - g * g) / (1.0 - g + 2.0 * g * xi);
  double c = (1.0 + g * g - frac * frac) / (2.0 * g);
  return clampd(c, -1.0, 1.0);
}

/* turn u by polar angle acos(cos_t) and azimuth phi about itself
 * (the direction update of MCML, Wang, Jacques & Zheng 1995) */
void orc_rotate(double u[3], double cos_t, double phi) {
  double sin_t = sqrt(maxd(0.0, 1.0 - cos_t * cos_t));
  double cp = cos(phi), sp = sin(phi);
  double ux = u[0], uy = u[1], uz = u[2];
  double v[3];
  if (fabs(uz) > 1.0 - 1e-5) {
    v[0] = sin_t * cp;
    v[1] = sin_t * sp;
    v[2] = (uz >= 0.0 ? 1.0 : -1.0) * cos_t;
  } else {
    double t = sqrt(1.0 - uz * uz);
    v[0] = sin_t * (ux * uz * cp - uy * sp) / t + ux * cos_t;
    v[1] = sin_t * (uy * uz * cp + ux * sp) / t + uy * cos_t;
    v[2] = -sin_t * cp * t + uz * cos_t;
  }
  double l = len3(v);
  for (int i = 0; i < 3; ++i) u[i] = v[i] / l;
}

/* ------------------------------------------------------------- tally --- */

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* Path-length fluence estimator on rectangular bins (Sec. 3.1, Table 2
 * runs): every voxel plane the segment crosses splits it; each piece is
 * credited to the voxel holding its midpoint.  Voxel i spans
 * [lo + i*D, lo + (i+1)*D); the grid's upper face belongs to the last voxel. */
int64_t orc_tally_segment(const orc_scene* s, const double a[3], const double b[3],
                          double w, double* f) {
  const int* nd = s->g_dims;
  if (!f || nd[0] <= 0 || nd[1] <= 0 || nd[2] <= 0) return 0;
  double d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  double len = len3(d);
  if (!(len > 0.0)) return 0;
  double u[3] = {d[0] / len, d[1] / len, d[2] / len};
  /* clip the parameter range [0, len] to the grid box */
  double t0 = 0.0, t1 = len;
  for (int i = 0; i < 3; ++i) {
    if (u[i] == 0.0) {
      if (a[i] < s->g_lo[i] || a[i] > s->g_hi[i]) return 0;
    } else {
      double ta = (s->g_lo[i] - a[i]) / u[i], tb = (s->g_hi[i] - a[i]) / u[i];
      t0 = maxd(t0, mind(ta, tb));
      t1 = mind(t1, maxd(ta, tb));
    }
  }
  if (!(t1 > t0)) return 0;
  /* every interior voxel plane crossed strictly inside (t0, t1): for each
   * axis, scan the plane indices between the clipped end coordinates */
  int lo_j[3] = {0, 0, 0}, hi_j[3] = {-1, -1, -1}, cap = 2;
  for (int i = 0; i < 3; ++i) {
    if (u[i] == 0.0) continue;
    double D = (s->g_hi[i] - s->g_lo[i]) / nd[i];
    double xa = a[i] + t0 * u[i], xb = a[i] + t1 * u[i];
    double x0 = mind(xa, xb), x1 = maxd(xa, xb);
    lo_j[i] = (int)floor((x0 - s->g_lo[i]) / D);
    hi_j[i] = (int)ceil((x1 - s->g_lo[i]) / D);
    if (lo_j[i] < 1) lo_j[i] = 1;
    if (hi_j[i] > nd[i] - 1) hi_j[i] = nd[i] - 1;
    if (hi_j[i] >= lo_j[i]) cap += hi_j[i] - lo_j[i] + 1;
  }
  double stackbuf[512];
  double* ts = cap <= 512 ? stackbuf : (double*)malloc(sizeof(double) * (size_t)cap);
  if (!ts) return 0;
  int m = 0;
  ts[m++] = t0;
  for (int i = 0; i < 3; ++i) {
    if (u[i] == 0.0) continue;
    double D = (s->g_hi[i] - s->g_lo[i]) / nd[i];
    for (int j = lo_j[i]; j <= hi_j[i]; ++j) {
      double plane = s->g_lo[i] + j * D;
      double t = (plane - a[i]) / u[i];
      if (t > t0 && t < t1) ts[m++] = t;
    }
  }
  ts[m++] = t1;
  qsort(ts, (size_t)m, sizeof(double), cmp_double);
  int64_t pieces = 0;
  for (int q = 0; q + 1 < m; ++q) {
    double l = ts[q + 1] - ts[q];
    if (!(l > 0.0)) continue;
    double tm = 0.5 * (ts[q] + ts[q + 1]);
    int idx[3];
    for (int i = 0; i < 3; ++i) {
      double D = (s->g_hi[i] - s->g_lo[i]) / nd[i];
      int v = (int)floor((a[i] + tm * u[i] - s->g_lo[i]) / D);
      idx[i] = v < 0 ? 0 : (v >= nd[i] ? nd[i] - 1 : v);
    }
    f[(size_t)idx[0] + (size_t)nd[0] * ((size_t)idx[1] + (size_t)nd[1] * (size_t)idx[2])] += w * l;
    ++pieces;
  }
  if (ts != stackbuf) free(ts);
  return pieces;
}

/* ------------------------------------------------------------ the walk --- */

typedef struct {
  const orc_scene* s;
  double* f;
  double* absorbed;
  orc_tallies* t;
  orc_event* rec;
  int cap, nrec;
  double* img; /* escape image, or NULL */
} walker;

typedef struct {
  double p[3], u[3], w, tau;
  int region;
  uint32_t k;
} packet;

static double reg_mua(const orc_scene* s, int r) { return r < 0 ? 0.0 : s->regions[r].mua; }
static double reg_mus(const orc_scene* s, int r) { return r < 0 ? 0.0 : s->regions[r].mus; }
static double reg_n(const orc_scene* s, int r) { return r < 0 ? s->n_ambient : s->regions[r].n; }

/* reading: the escape image (Sec. 3.2 and Sec. 5: the light at a single
 * plane of interest).  A packet leaving through the detector face adds its
 * weight to the pixel holding the point where its straight path crosses
 * the face's plane: traced back along u from its position when that lies
 * beyond the plane and the packet moves outward, else its position. */
static void detect(walker* wk, const packet* pk, int face, double plane) {
  const orc_scene* s = wk->s;
  if (!wk->img || face != s->det_face || s->det_dims[0] < 1 || s->det_dims[1] < 1) return;
  const int ax = face / 2;
  const double sg = (face % 2) ? 1.0 : -1.0;
  double q[3] = {pk->p[0], pk->p[1], pk->p[2]};
  double over = (pk->p[ax] - plane) * sg, out = pk->u[ax] * sg;
  if (over > 0.0 && out > 0.0) {
    double t = over / out;
    for (int a = 0; a < 3; ++a) q[a] = pk->p[a] - t * pk->u[a];
  }
  const int a1 = ax == 0 ? 1 : 0, a2 = ax == 2 ? 1 : 2;
  double x = (q[a1] - s->det_lo[0]) / (s->det_hi[0] - s->det_lo[0]) * s->det_dims[0];
  double y = (q[a2] - s->det_lo[1]) / (s->det_hi[1] - s->det_lo[1]) * s->det_dims[1];
  /* bounds in floating point, before any conversion (NaN fails too) */
  if (!(x >= 0.0 && y >= 0.0 && x < s->det_dims[0] && y < s->det_dims[1])) return;
  int i = (int)floor(x), j = (int)floor(y);
  wk->img[(size_t)i + (size_t)s->det_dims[0] * (size_t)j] += pk->w;
}

static void record(walker* wk, const packet* pk, int type) {
  if (!wk->rec || wk->nrec >= wk->cap) return;
  orc_event* e = &wk->rec[wk->nrec++];
  e->event = pk->k;
  e->type = (uint32_t)type;
  e->region = pk->region;
  e->pad = 0;
  for (int i = 0; i < 3; ++i) { e->p[i] = pk->p[i]; e->u[i] = pk->u[i]; }
  e->w = pk->w;
  e->tau = pk->tau;
}

/* straight move of length l along u, tallied with the current weight */
static void move(walker* wk, packet* pk, double l) {
  double b[3] = {pk->p[0] + l * pk->u[0], pk->p[1] + l * pk->u[1], pk->p[2] + l * pk->u[2]};
  wk->t->voxel_segments += (uint64_t)orc_tally_segment(wk->s, pk->p, b, pk->w, wk->f);
  for (int i = 0; i < 3; ++i) pk->p[i] = b[i];
}

/* emission, event 0 */
static void emit(walker* wk, packet* pk, uint64_t seed, uint64_t pid) {
  const orc_scene* s = wk->s;
  const double* q = s->src;
  double xi[4];
  pk->k = 0;
  event_xi(seed, pid, 0, xi);
  switch (s->src_kind) {
    case ORC_SRC_POINT: { /* isotropic point source (Sec. 3.1) */
      double ct = 2.0 * xi[0] - 1.0, st = sqrt(maxd(0.0, 1.0 - ct * ct));
      double phi = 2.0 * M_PI * xi[1];
      for (int i = 0; i < 3; ++i) pk->p[i] = q[i];
      pk->u[0] = st * cos(phi); pk->u[1] = st * sin(phi); pk->u[2] = ct;
      break;
    }
    case ORC_SRC_PENCIL: /* collimated beam from one point */
      for (int i = 0; i < 3; ++i) { pk->p[i] = q[i]; pk->u[i] = q[3 + i]; }
      break;
    case ORC_SRC_DISC: { /* top-hat disc of radius q[3] in a z-plane */
      double r = q[3] * sqrt(xi[0]), phi = 2.0 * M_PI * xi[1];
      pk->p[0] = q[0] + r * cos(phi); pk->p[1] = q[1] + r * sin(phi); pk->p[2] = q[2];
      for (int i = 0; i < 3; ++i) pk->u[i] = q[4 + i];
      break;
    }
    case ORC_SRC_RECT: /* uniform over a z-plane rectangle of half sides q[3], q[4] */
      pk->p[0] = q[0] + q[3] * (2.0 * xi[0] - 1.0);
      pk->p[1] = q[1] + q[4] * (2.0 * xi[1] - 1.0);
      pk->p[2] = q[2];
      for (int i = 0; i < 3; ++i) pk->u[i] = q[5 + i];
      break;
  }
  double l = len3(pk->u);
  for (int i = 0; i < 3; ++i) pk->u[i] /= l;
  pk->w = 1.0;
  pk->tau = -log(xi[3]); /* Eq. 1 */
  pk->region = orc_region_of(s, pk->p);
  wk->t->launched += 1.0;
  record(wk, pk, ORC_EV_EMIT);
}

/* absorption, scattering and roulette at an interaction point; returns 0
 * when the packet ends */
static int interact(walker* wk, packet* pk, uint64_t seed, uint64_t pid) {
  const orc_scene* s = wk->s;
  const orc_region* rg = &s->regions[pk->region];
  double xi[4];
  pk->k += 1;
  event_xi(seed, pid, pk->k, xi);
  wk->t->events++;
  wk->t->interactions++;
  /* reading: implicit capture, the fraction mu_a/mu_t of the weight is
   * deposited at every interaction */
  double dA = pk->w * rg->mua / (rg->mua + rg->mus);
  wk->absorbed[pk->region] += dA;
  pk->w -= dA;
  if (pk->w == 0.0) {
    record(wk, pk, ORC_EV_ABSORB);
    return 0;
  }
  orc_rotate(pk->u, orc_hg_cos(rg->g, xi[0]), 2.0 * M_PI * xi[1]);
  if (pk->w < s->w_threshold) { /* Russian roulette */
    if (xi[2] < 1.0 / (double)s->m_survive) {
      wk->t->roulette_gain += (double)(s->m_survive - 1) * pk->w;
      pk->w *= (double)s->m_survive;
    } else {
      wk->t->roulette_loss += pk->w;
      wk->t->kills++;
      record(wk, pk, ORC_EV_KILL);
      return 0;
    }
  }
  pk->tau = -log(xi[3]); /* Eq. 1 */
  record(wk, pk, ORC_EV_SCATTER);
  return 1;
}

enum { GO_ON = 0, DO_INTERACT = 1, ENDED = 2 };

/* the packet is within delta of a surface (Sec. 2.3); s_rem is the
 * remaining free path in cm */
static int surface(walker* wk, packet* pk, double s_rem, uint64_t seed, uint64_t pid) {
  const orc_scene* s = wk->s;
  const double delta = s->delta;
  double mut = reg_mua(s, pk->region) + reg_mus(s, pk->region);
  /* nearest surface j: smallest |d_r|, ties to the lowest index */
  int j = 0;
  double dj = orc_region_sdf(s, 0, pk->p);
  for (int r = 1; r < s->n_regions; ++r) {
    double d = orc_region_sdf(s, r, pk->p);
    if (fabs(d) < fabs(dj)) { dj = d; j = r; }
  }
  double h = ORC_H_NORMAL * delta;
  double n0[3];
  orc_region_normal(s, j, pk->p, h, n0);
  double c0 = dot3(pk->u, n0);
  /* reading: the surface point is where the ray meets the surface
   * (one Newton step along u); grazing rays fall back to the normal foot */
  double t_ray = 0.0, ps[3];
  if (fabs(c0) >= ORC_SNAP_COS) {
    t_ray = -dj / c0;
    for (int i = 0; i < 3; ++i) ps[i] = pk->p[i] + t_ray * pk->u[i];
  } else {
    for (int i = 0; i < 3; ++i) ps[i] = pk->p[i] - dj * n0[i];
  }
  double nrm[3];
  orc_region_normal(s, j, ps, h, nrm);
  double c = dot3(pk->u, nrm);
  double sg = c > 0.0 ? 1.0 : -1.0;
  double q[3];
  for (int i = 0; i < 3; ++i) q[i] = ps[i] + sg * ORC_OFFSET * delta * nrm[i];
  int r2 = (c == 0.0) ? pk->region : orc_region_of(s, q);
  if (r2 == pk->region) {
    /* reading: no change of medium ahead (moving away, parallel, or a face
     * hidden inside one region): advance 2*delta along the ray */
    wk->t->advances++;
    double l = ORC_OFFSET * delta;
    if (s_rem <= l) {
      move(wk, pk, s_rem);
      pk->tau = 0.0;
      return DO_INTERACT;
    }
    move(wk, pk, l);
    pk->tau -= mut * l;
    return GO_ON;
  }
  /* a change of medium: go to the surface point first */
  if (t_ray > 0.0) {
    if (s_rem <= t_ray) {
      move(wk, pk, s_rem);
      pk->tau = 0.0;
      return DO_INTERACT;
    }
    move(wk, pk, t_ray);
    pk->tau -= mut * t_ray;
  }
  for (int i = 0; i < 3; ++i) pk->p[i] = ps[i];
  pk->k += 1;
  wk->t->events++;
  wk->t->interfaces++;
  double n1 = reg_n(s, pk->region), n2 = reg_n(s, r2);
  if (n1 == n2) { /* index matched: cross without deflection */
    for (int i = 0; i < 3; ++i) pk->p[i] = q[i];
    pk->region = r2;
    wk->t->crossings++;
    record(wk, pk, ORC_EV_CROSS);
    return GO_ON;
  }
  double xi[4];
  event_xi(seed, pid, pk->k, xi);
  double cos_i = fabs(c), cos_t;
  double R = orc_fresnel(n1, n2, cos_i, &cos_t);
  if (xi[0] < R) { /* specular reflection back into the current medium */
    for (int i = 0; i < 3; ++i) {
      pk->u[i] -= 2.0 * c * nrm[i];
      pk->p[i] = ps[i] - sg * ORC_OFFSET * delta * nrm[i];
    }
    double l = len3(pk->u);
    for (int i = 0; i < 3; ++i) pk->u[i] /= l;
    wk->t->reflections++;
    record(wk, pk, ORC_EV_REFLECT);
  } else { /* refraction by Snell's law into the far medium */
    double eta = n1 / n2;
    for (int i = 0; i < 3; ++i) pk->u[i] = eta * pk->u[i] + (cos_t - eta * cos_i) * sg * nrm[i];
    double l = len3(pk->u);
    for (int i = 0; i < 3; ++i) { pk->u[i] /= l; pk->p[i] = q[i]; }
    pk->region = r2;
    wk->t->refractions++;
    record(wk, pk, ORC_EV_REFRACT);
  }
  return GO_ON;
}

/* Ambient skip, an acceleration that leaves the walk as it is: outside
 * every region, the straight path from p along u cuts no surface before it
 * enters the box of some region's surface (orc_region.box_lo/hi); when it
 * enters none inside the volume, only the volume's boundary lies ahead.
 * Returns the path to the first box entered, or delta past the boundary;
 * 0 when p is inside a box.  Slab test per axis with t = (plane - p) / u
 * taken as (plane - p) * (1/u); an axis with u = 0 meets the box only when
 * p lies between its planes. */
static double ambient_free(const orc_scene* s, const double p[3], const double u[3]) {
  double r[3], t = ORC_INF;
  for (int i = 0; i < 3; ++i) {
    r[i] = 1.0 / u[i];
    if (u[i] != 0.0) t = mind(t, ((u[i] > 0.0 ? s->bb_hi[i] : s->bb_lo[i]) - p[i]) * r[i]);
  }
  t += s->delta;
  for (int k = 0; k < s->n_regions; ++k) {
    const orc_region* rg = &s->regions[k];
    double t0 = 0.0, t1 = t;
    int hit = 1;
    for (int i = 0; i < 3; ++i) {
      if (u[i] == 0.0) {
        if (p[i] < rg->box_lo[i] || p[i] > rg->box_hi[i]) hit = 0;
      } else {
        const double a = (rg->box_lo[i] - p[i]) * r[i], b = (rg->box_hi[i] - p[i]) * r[i];
        t0 = maxd(t0, mind(a, b));
        t1 = mind(t1, maxd(a, b));
      }
    }
    if (hit && t0 <= t1) t = t0;
  }
  return t;
}

/* Segment tracing (Sec. 5 names it beside enhanced sphere tracing against
 * the many small steps near surfaces).  Outside a convex shape the exact
 * distance along a ray, f(t) = d(p + t u), is a convex function of t, so it
 * never falls below its tangent: f(t) >= f(0) + f'(0) t.  The ray cannot
 * reach the shape before t = f(0) / (-f'(0)), and never when f'(0) >= 0.
 * f'(0) = grad d . u, and outside the shape grad d is the unit vector from
 * the nearest surface point to p.  A union is reached when one of its
 * members is, so the smallest member bound holds for it; an intersection
 * only when every member is, so the largest bound of a member not yet
 * reached holds; a subtraction (the first member less the others) lies
 * inside its first member and is not reached before it.  The distance
 * itself is a bound too, and the larger of two bounds holds.  Inside a
 * region, and for smooth unions and every other shape, the bound is the
 * distance alone. */

/* whether a primitive is one of the convex shapes with exact distances,
 * unplaced and unmodified */
static int plain_convex(const orc_prim* pr) {
  if (pr->flags != 0 || pr->round_r != 0.0 || pr->onion_t != 0.0 || pr->disp_a != 0.0 ||
      pr->elong[0] != 0.0 || pr->elong[1] != 0.0 || pr->elong[2] != 0.0)
    return 0;
  return pr->kind == ORC_SPHERE || pr->kind == ORC_BOX || pr->kind == ORC_CAPSULE || pr->kind == ORC_CYLINDER;
}

/* outward unit gradient of the distance to a plain convex primitive at a
 * point p outside it */
static void convex_gradient(const orc_prim* pr, const double p[3], double g[3]) {
  const double* q = pr->p;
  double v[3] = {0.0, 0.0, 0.0};
  switch (pr->kind) {
    case ORC_SPHERE: /* from the centre */
      for (int i = 0; i < 3; ++i) v[i] = p[i] - q[i];
      break;
    case ORC_BOX: /* from the nearest point of the box */
      for (int i = 0; i < 3; ++i) {
        double e = fabs(p[i] - q[i]) - q[3 + i];
        v[i] = e > 0.0 ? (p[i] > q[i] ? e : -e) : 0.0;
      }
      break;
    case ORC_CAPSULE: { /* from the nearest point of the axis segment */
      double ba[3] = {q[3] - q[0], q[4] - q[1], q[5] - q[2]};
      double pa[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
      double t = clampd(dot3(pa, ba) / dot3(ba, ba), 0.0, 1.0);
      for (int i = 0; i < 3; ++i) v[i] = pa[i] - t * ba[i];
      break;
    }
    case ORC_CYLINDER: { /* in the (radial, axial) half plane: from the nearest point of the rectangle */
      double ba[3] = {q[3] - q[0], q[4] - q[1], q[5] - q[2]};
      double L = len3(ba);
      double e[3] = {ba[0] / L, ba[1] / L, ba[2] / L};
      double pa[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
      double x = dot3(pa, e);
      double radial[3] = {pa[0] - x * e[0], pa[1] - x * e[1], pa[2] - x * e[2]};
      double rho = len3(radial);
      double o1 = maxd(rho - q[6], 0.0), o2 = maxd(fabs(x - 0.5 * L) - 0.5 * L, 0.0);
      double sa = x > 0.5 * L ? 1.0 : -1.0;
      for (int i = 0; i < 3; ++i) v[i] = (rho > 0.0 ? o1 * radial[i] / rho : 0.0) + o2 * sa * e[i];
      break;
    }
  }
  double l = len3(v);
  for (int i = 0; i < 3; ++i) g[i] = l > 0.0 ? v[i] / l : 0.0;
}

/* rounding slack of the directional derivative (FP64) */
#define ORC_SEG_EPS 1e-12

/* the tangent bound of a plain convex primitive at p, where its distance
 * is a > 0 */
static double convex_bound(const orc_prim* pr, const double p[3], const double u[3], double a) {
  double g[3];
  convex_gradient(pr, p, g);
  const double slope = ORC_SEG_EPS - dot3(g, u); /* -f'(0), made no smaller by the slack */
  return slope > 0.0 ? a / slope : ORC_INF;
}

double orc_segment_bound(const orc_scene* s, int r, const double p[3], const double u[3]) {
  const double d = orc_region_sdf(s, r, p);
  const orc_region* rg = &s->regions[r];
  const orc_prim* pr = &s->prims[rg->first_prim];
  if (d <= 0.0) return fabs(d);
  double T = d;
  switch (rg->op) {
    case ORC_UNION: {
      for (int i = 0; i < rg->n_prims; ++i)
        if (!plain_convex(&pr[i])) return d;
      double t = ORC_INF;
      for (int i = 0; i < rg->n_prims; ++i) t = mind(t, convex_bound(&pr[i], p, u, shape_sdf(&pr[i], p)));
      T = maxd(T, t);
      break;
    }
    case ORC_INTERSECT:
      for (int i = 0; i < rg->n_prims; ++i)
        if (!plain_convex(&pr[i])) return d;
      for (int i = 0; i < rg->n_prims; ++i) {
        const double a = shape_sdf(&pr[i], p);
        if (a > 0.0) T = maxd(T, convex_bound(&pr[i], p, u, a));
      }
      break;
    case ORC_SUBTRACT:
      if (plain_convex(pr)) {
        const double a = shape_sdf(pr, p);
        if (a > 0.0) T = maxd(T, convex_bound(pr, p, u, a));
      }
      break;
    default:
      break;
  }
  return T;
}

/* length of a segment-traced step from p: the smallest bound over the
 * regions less delta, or delta past the simulation volume's boundary when
 * that comes first (so that a ray that meets nothing leaves); never
 * shorter than d */
static double segment_step(const orc_scene* s, const double p[3], const double u[3], double d) {
  double exit = ORC_INF, T = ORC_INF;
  for (int i = 0; i < 3; ++i)
    if (u[i] != 0.0) exit = mind(exit, ((u[i] > 0.0 ? s->bb_hi[i] : s->bb_lo[i]) - p[i]) / u[i]);
  for (int r = 0; r < s->n_regions; ++r) T = mind(T, orc_segment_bound(s, r, p, u));
  return maxd(d, mind(T - s->delta, exit + s->delta));
}

/* the over-relaxed step rule (see walk) */
static int relaxed_step(const orc_scene* s, double dmin, double pd, double pl, double s_rem) {
  return s->relax > 1.0 && pd >= 0.0 &&
         dmin * ((2.0 - s->relax) * pl - s->relax * (pd - dmin)) >= s->delta * pl &&
         s->relax * dmin < s_rem;
}

/* length of the ambient skip from p, or 0 when the step the march would
 * take (plain or over-relaxed) is as long, or when the boxes' margin of
 * delta/2 does not cover the rounding of the box test and of the move: 4
 * units in the last place of the largest coordinate plus the skip */
static double ambient_skip(const orc_scene* s, const double p[3], const double u[3], double dmin, double pd,
                           double pl, double s_rem) {
  const double len = relaxed_step(s, dmin, pd, pl, s_rem) ? s->relax * dmin : dmin;
  const double tf = ambient_free(s, p, u);
  const double pmax = maxd(fabs(p[0]), maxd(fabs(p[1]), fabs(p[2])));
  return tf > len && 0.5 * s->delta >= 0x1p-50 * (pmax + tf) ? tf : 0.0;
}

/* escape (Sec. 2.3: the bounding-box SDF is positive): the weight leaves
 * through the face of the box's largest component of |p - c| - h
 * (reading: escape bookkeeping per face) */
static void leave(walker* wk, packet* pk) {
  const orc_scene* s = wk->s;
  double best = -ORC_INF;
  int face = 0;
  for (int i = 0; i < 3; ++i) {
    double c = 0.5 * (s->bb_lo[i] + s->bb_hi[i]), hw = 0.5 * (s->bb_hi[i] - s->bb_lo[i]);
    double e = fabs(pk->p[i] - c) - hw;
    if (e > best) { best = e; face = 2 * i + (pk->p[i] > c ? 1 : 0); }
  }
  wk->t->escaped_face[face] += pk->w;
  wk->t->escapes++;
  detect(wk, pk, face, (face % 2) ? s->bb_hi[face / 2] : s->bb_lo[face / 2]);
  record(wk, pk, ORC_EV_ESCAPE);
}

/* reading: a packet past the safety caps (grazing stalls, Sec. 5) ends,
 * its weight kept in the stalled ledger */
static void stall(walker* wk, packet* pk) {
  wk->t->stalled += pk->w;
  wk->t->stalls++;
  record(wk, pk, ORC_EV_STALL);
}

/* The walk of one packet, Sec. 2.3.  Emit (event 0), then repeat: sphere
 * trace -- evaluate every region's SDF at p, d = min |d_r| -- and, in this
 * order (reading: the order of the checks), escape when the bounding box's
 * SDF is positive; move the remaining free path s = tau/mu_t and interact
 * when s <= d; handle the surface when d < delta; else move d along u,
 * spending mu_t d of optical depth.  Every move is tallied. */
static void walk_plain(walker* wk, uint64_t seed, uint64_t pid) {
  const orc_scene* s = wk->s;
  packet pk;
  emit(wk, &pk, seed, pid);
  for (;;) {
    int32_t steps = 0; /* sphere-tracing steps in this event */
    int state = GO_ON;
    while (state == GO_ON) {
      if (++steps > s->max_steps || (int64_t)pk.k > s->max_events) {
        stall(wk, &pk);
        return;
      }
      wk->t->steps++;
      double d = ORC_INF;
      for (int r = 0; r < s->n_regions; ++r) d = mind(d, fabs(orc_region_sdf(s, r, pk.p)));
      if (orc_box_sdf(s->bb_lo, s->bb_hi, pk.p) > 0.0) {
        leave(wk, &pk);
        return;
      }
      const double mut = reg_mua(s, pk.region) + reg_mus(s, pk.region);
      const double s_rem = mut > 0.0 ? pk.tau / mut : ORC_INF; /* reading: tau compared as a length */
      if (s_rem <= d) {
        move(wk, &pk, s_rem);
        pk.tau = 0.0;
        state = DO_INTERACT;
      } else if (d < s->delta) {
        const uint32_t k_before = pk.k;
        state = surface(wk, &pk, s_rem, seed, pid);
        if (pk.k != k_before) steps = 0; /* an interface event starts a new event */
      } else {
        move(wk, &pk, d);
        pk.tau -= mut * d;
      }
    }
    if (!interact(wk, &pk, seed, pid)) return;
  }
}

/* The same walk through the kernels' shortcuts, for step counts.  None of
 * them changes an event: an interaction inside the free ball of the last
 * evaluation is the one a new evaluation would give (free-flight reuse);
 * outside every region no surface lies before the first region box the ray
 * enters (ambient skip); an over-relaxed step is kept only when the free
 * balls at its ends cover it (Sec. 5), else replaced by the plain step. */
static void walk_mirror(walker* wk, uint64_t seed, uint64_t pid) {
  const orc_scene* s = wk->s;
  packet pk;
  emit(wk, &pk, seed, pid);
  /* free-flight reuse: a ball of radius safe around the packet that holds
   * no surface (< 0: none known), and the interactions taken in it since
   * the distance was evaluated */
  double safe = -1.0;
  int links = 0;
  for (;;) {
    /* one event: sphere-trace until interaction (Sec. 2.3) */
    int32_t steps = 0;
    int state = GO_ON;
    /* the previous sphere-tracing step of this segment: surface distance
     * at its start pd (< 0: none yet), its length pl; a relaxed one waits
     * for its check (pending) with its start point q and the depth there */
    double q[3] = {0.0, 0.0, 0.0}, pd = -1.0, pl = 0.0, tau_q = 0.0;
    int pending = 0;
    while (state == GO_ON) {
      if (s->reuse && safe > 0.0 && pk.region >= 0 && links < ORC_REUSE_LINKS) {
        /* the last evaluated distance, less the path since, bounds the
         * distance to every surface: an interaction inside that ball is the
         * one a new evaluation would give, so none is made.  Inside a region
         * the ball is inside the volume too.  Margin: delta, plus per
         * interaction in the ball 4 units in the last place of the position
         * for the rounding of the moves */
        const double mut_r = reg_mua(s, pk.region) + reg_mus(s, pk.region);
        const double s_r = mut_r > 0.0 ? pk.tau / mut_r : ORC_INF;
        const double pmax = maxd(fabs(pk.p[0]), maxd(fabs(pk.p[1]), fabs(pk.p[2])));
        if (s_r <= safe - s->delta - (links + 1) * pmax * 0x1p-50) {
          move(wk, &pk, s_r);
          pk.tau = 0.0;
          safe -= s_r;
          ++links;
          state = DO_INTERACT;
          continue;
        }
      }
      safe = -1.0;
      if (++steps > s->max_steps || (int64_t)pk.k > s->max_events) {
        if (pending) wk->t->voxel_segments += (uint64_t)orc_tally_segment(s, q, pk.p, pk.w, wk->f);
        stall(wk, &pk);
        return;
      }
      wk->t->steps++;
      double dmin = ORC_INF;
      for (int r = 0; r < s->n_regions; ++r) dmin = mind(dmin, fabs(orc_region_sdf(s, r, pk.p)));
      if (pending) {
        /* check of an over-relaxed step (enhanced sphere tracing, the
         * remedy for slow grazing steps named in Sec. 5): the open balls of
         * radius pd around q and dmin around its end hold no surface, so if
         * together they cover the step (with a margin of delta against
         * rounding) it crossed none.  Any crossing forces pd + dmin <= pl.
         * Otherwise fall back to the plain step of pd from q. */
        const int keep = pd + dmin >= pl + s->delta;
        if (!keep) {
          for (int i = 0; i < 3; ++i) pk.p[i] = q[i] + pd * pk.u[i];
          pk.tau = tau_q - (reg_mua(s, pk.region) + reg_mus(s, pk.region)) * pd;
          pl = pd;
        }
        wk->t->voxel_segments += (uint64_t)orc_tally_segment(s, q, pk.p, pk.w, wk->f);
        pending = 0;
        if (!keep) continue; /* the next step starts from the plain step's end */
      }
      if (orc_box_sdf(s->bb_lo, s->bb_hi, pk.p) > 0.0) { /* left the volume */
        leave(wk, &pk);
        return;
      }
      double mut = reg_mua(s, pk.region) + reg_mus(s, pk.region);
      double s_rem = mut > 0.0 ? pk.tau / mut : ORC_INF;
      double skip = 0.0;
      if (s->skip && pk.region < 0 && dmin >= s->delta) skip = ambient_skip(s, pk.p, pk.u, dmin, pd, pl, s_rem);
      /* segment-traced step: the ray is free of surfaces for seg */
      const double seg = s->segment && dmin >= s->delta ? segment_step(s, pk.p, pk.u, dmin) : dmin;
      if (seg > dmin && s_rem <= seg && s_rem > dmin) {
        /* the interaction point lies on the free segment: the one plain
         * steps reach; no free ball about it is known */
        move(wk, &pk, s_rem);
        pk.tau = 0.0;
        state = DO_INTERACT;
      } else if (s_rem <= dmin) { /* the optical depth runs out first */
        move(wk, &pk, s_rem);
        pk.tau = 0.0;
        state = DO_INTERACT;
        if (pk.region >= 0) { /* the ball of radius dmin about the step's start holds no surface */
          safe = dmin - s_rem;
          links = 0;
        }
      } else if (dmin < s->delta) { /* on a boundary */
        uint32_t k_before = pk.k;
        state = surface(wk, &pk, s_rem, seed, pid);
        if (pk.k != k_before) { /* an interface event starts a new event */
          steps = 0;
          pd = -1.0;
        }
      } else if (skip > 0.0 && skip >= seg) {
        /* no surface along the skip: one move (the ambient medium has
         * mu_t = 0), and no previous step for the over-relaxation rule */
        move(wk, &pk, skip);
        pd = -1.0;
        pl = 0.0;
      } else if (seg > dmin) { /* segment-traced step */
        move(wk, &pk, seg);
        pk.tau -= mut * seg;
        pd = -1.0;
        pl = 0.0;
      } else if (relaxed_step(s, dmin, pd, pl, s_rem)) {
        /* over-relaxed step, taken when it would pass its check were the
         * surface a plane met at the angle the previous step saw: the
         * distance falls by (pd - dmin)/pl per unit length, so at the end
         * of a step w dmin it is dmin - w (pd - dmin) dmin / pl, and the
         * check needs dmin + that >= w dmin + delta.  Its path is credited
         * once the check passes */
        for (int i = 0; i < 3; ++i) q[i] = pk.p[i];
        pd = dmin;
        pl = s->relax * dmin;
        tau_q = pk.tau;
        for (int i = 0; i < 3; ++i) pk.p[i] += pl * pk.u[i];
        pk.tau -= mut * pl;
        pending = 1;
      } else { /* sphere-tracing step of the full distance */
        move(wk, &pk, dmin);
        pk.tau -= mut * dmin;
        pd = dmin;
        pl = dmin;
      }
    }
    if (!interact(wk, &pk, seed, pid)) return;
  }
}

/* the plain walk unless the scene asks for the shortcuts */
static void walk(walker* wk, uint64_t seed, uint64_t pid) {
  const orc_scene* s = wk->s;
  if (s->reuse || s->skip || s->segment || s->relax > 1.0) walk_mirror(wk, seed, pid);
  else walk_plain(wk, seed, pid);
}

/* --------------------------------------------------------------- runs --- */

static int check_scene(const orc_scene* s) {
  if (!s || s->n_regions < 1 || s->n_prims < 1 || !s->prims || !s->regions) return -1;
  if (!(s->delta > 0.0) || s->m_survive < 1 || s->max_steps < 1) return -1;
  if (!(s->relax >= 1.0 && s->relax < 2.0)) return -1;
  if (s->segment && s->relax > 1.0) return -1;
  for (int r = 0; r < s->n_regions; ++r) {
    const orc_region* rg = &s->regions[r];
    if (rg->first_prim < 0 || rg->n_prims < 1 || rg->first_prim + rg->n_prims > s->n_prims) return -1;
    if (!(rg->mua >= 0.0) || !(rg->mus >= 0.0) || !(rg->mua + rg->mus > 0.0)) return -1;
  }
  return 0;
}

int orc_trace(const orc_scene* s, uint64_t seed, uint64_t pid, int cap, orc_event* out) {
  if (check_scene(s) != 0 || !out || cap < 1) return -1;
  double* absorbed = (double*)calloc((size_t)s->n_regions, sizeof(double));
  orc_tallies t;
  memset(&t, 0, sizeof(t));
  walker wk = {s, NULL, absorbed, &t, out, cap, 0, NULL};
  walk(&wk, seed, pid);
  free(absorbed);
  return wk.nrec;
}


/* ------------------------------------------------------ voxel model --- */
/* The voxel-geometry MCRT the paper compares against (Sec. 2.3, Sec. 3.2):
 * every voxel of the fluence grid carries the optical properties of the
 * region that owns its centre; a packet is ray traced from voxel to voxel
 * until its optical depth runs out or it leaves the grid.  Refractive
 * index changes happen only on voxel faces, whose normals are the axes.
 * reading: a source outside the grid first travels (untallied, unattenuated)
 * to the grid; beyond the grid lies the ambient medium, so a packet leaving
 * it meets Fresnel at that face like at any index change, and escapes when
 * transmitted; faces between voxels of equal index are crossed without an
 * event; faces with an index change are interface events (event index + 1,
 * variate xi0). */

void orc_voxelize(const orc_scene* s, int8_t* vox) {
  const int* nd = s->g_dims;
  for (int k = 0; k < nd[2]; ++k)
    for (int j = 0; j < nd[1]; ++j)
      for (int i = 0; i < nd[0]; ++i) {
        double c[3];
        const int ijk[3] = {i, j, k};
        for (int a = 0; a < 3; ++a) {
          double D = (s->g_hi[a] - s->g_lo[a]) / nd[a];
          c[a] = s->g_lo[a] + (ijk[a] + 0.5) * D;
        }
        vox[(size_t)i + (size_t)nd[0] * ((size_t)j + (size_t)nd[1] * (size_t)k)] = (int8_t)orc_region_of(s, c);
      }
}

typedef struct {
  const int8_t* vox;
} voxel_geo;

static int vox_region(const orc_scene* s, const voxel_geo* vg, const int v[3]) {
  return vg->vox[(size_t)v[0] + (size_t)s->g_dims[0] * ((size_t)v[1] + (size_t)s->g_dims[1] * (size_t)v[2])];
}

/* tally a straight piece that lies inside voxel v */
static void vox_tally(walker* wk, const int v[3], double w, double l) {
  const orc_scene* s = wk->s;
  if (!wk->f || !(l > 0.0)) return;
  wk->f[(size_t)v[0] + (size_t)s->g_dims[0] * ((size_t)v[1] + (size_t)s->g_dims[1] * (size_t)v[2])] += w * l;
  wk->t->voxel_segments++;
}

static void walk_voxel(walker* wk, const voxel_geo* vg, uint64_t seed, uint64_t pid) {
  const orc_scene* s = wk->s;
  const int* nd = s->g_dims;
  double D[3];
  for (int a = 0; a < 3; ++a) D[a] = (s->g_hi[a] - s->g_lo[a]) / nd[a];
  packet pk;
  emit(wk, &pk, seed, pid);  /* sets the SDF-model region; replaced below */
  int v[3];
  int inside = 1;
  for (int a = 0; a < 3; ++a)
    if (pk.p[a] < s->g_lo[a] || pk.p[a] > s->g_hi[a]) inside = 0;
  int entry_axis = -1;
  if (!inside) { /* reach the grid through ambient, or miss it */
    double t0 = 0.0, t1 = ORC_INF;
    for (int a = 0; a < 3; ++a) {
      if (pk.u[a] == 0.0) {
        if (pk.p[a] < s->g_lo[a] || pk.p[a] > s->g_hi[a]) t1 = -1.0;
      } else {
        double ta = (s->g_lo[a] - pk.p[a]) / pk.u[a], tb = (s->g_hi[a] - pk.p[a]) / pk.u[a];
        double tn = mind(ta, tb), tx = maxd(ta, tb);
        if (tn > t0) { t0 = tn; entry_axis = a; }
        t1 = mind(t1, tx);
      }
    }
    if (!(t1 > t0) || entry_axis < 0) {
      int face = 0;
      double best = -ORC_INF;
      for (int a = 0; a < 3; ++a) {
        double c = 0.5 * (s->g_lo[a] + s->g_hi[a]), e = fabs(pk.p[a] - c) - 0.5 * (s->g_hi[a] - s->g_lo[a]);
        if (e > best) { best = e; face = 2 * a + (pk.p[a] > c ? 1 : 0); }
      }
      pk.region = -1;
      wk->t->escaped_face[face] += pk.w;
      wk->t->escapes++;
      record(wk, &pk, ORC_EV_ESCAPE);
      return;
    }
    for (int a = 0; a < 3; ++a) pk.p[a] += t0 * pk.u[a];
    pk.region = -1; /* still in ambient, on the grid face */
  }
  /* voxel holding the point, ties broken by the direction of travel */
  for (int a = 0; a < 3; ++a) {
    double x = (pk.p[a] - s->g_lo[a]) / D[a];
    int i = (int)floor(x);
    if (pk.u[a] < 0.0 && x == floor(x)) i -= 1;
    if (a == entry_axis) i = pk.u[a] > 0.0 ? 0 : nd[a] - 1;
    v[a] = i < 0 ? 0 : (i >= nd[a] ? nd[a] - 1 : i);
  }
  if (entry_axis >= 0) { /* crossing the grid face from ambient into voxel v */
    int r2 = vox_region(s, vg, v);
    double n1 = s->n_ambient, n2 = reg_n(s, r2);
    if (n1 != n2) {
      pk.k += 1;
      wk->t->events++;
      wk->t->interfaces++;
      double xi[4];
      event_xi(seed, pid, pk.k, xi);
      double ci = fabs(pk.u[entry_axis]), ct;
      double R = orc_fresnel(n1, n2, ci, &ct);
      if (xi[0] < R) { /* reflected off the grid: it leaves */
        pk.u[entry_axis] = -pk.u[entry_axis];
        wk->t->reflections++;
        record(wk, &pk, ORC_EV_REFLECT);
        int face = 2 * entry_axis + (pk.u[entry_axis] > 0.0 ? 1 : 0);
        wk->t->escaped_face[face] += pk.w;
        wk->t->escapes++;
        detect(wk, &pk, face, (face % 2) ? s->g_hi[face / 2] : s->g_lo[face / 2]);
        record(wk, &pk, ORC_EV_ESCAPE);
        return;
      }
      double eta = n1 / n2, sg = pk.u[entry_axis] > 0.0 ? 1.0 : -1.0;
      for (int a = 0; a < 3; ++a) pk.u[a] *= eta;
      pk.u[entry_axis] += (ct - eta * ci) * sg;
      double l = len3(pk.u);
      for (int a = 0; a < 3; ++a) pk.u[a] /= l;
      wk->t->refractions++;
      pk.region = r2;
      record(wk, &pk, ORC_EV_REFRACT);
    } else {
      pk.region = r2;
    }
  } else {
    pk.region = vox_region(s, vg, v);
  }
  int32_t steps = 0; /* voxel faces crossed since the last event */
  for (;;) {
    if (++steps > s->max_steps || (int64_t)pk.k > s->max_events) {
      wk->t->stalled += pk.w;
      wk->t->stalls++;
      record(wk, &pk, ORC_EV_STALL);
      return;
    }
    wk->t->steps++;
    /* distance to the exit face of voxel v along each axis */
    double texit = ORC_INF;
    int ax = -1;
    for (int a = 0; a < 3; ++a) {
      if (pk.u[a] == 0.0) continue;
      double face = s->g_lo[a] + (v[a] + (pk.u[a] > 0.0 ? 1 : 0)) * D[a];
      double t = (face - pk.p[a]) / pk.u[a];
      if (t < 0.0) t = 0.0;
      if (t < texit) { texit = t; ax = a; }
    }
    double mut = reg_mua(s, pk.region) + reg_mus(s, pk.region);
    double s_rem = mut > 0.0 ? pk.tau / mut : ORC_INF;
    if (s_rem <= texit) { /* interaction inside this voxel */
      vox_tally(wk, v, pk.w, s_rem);
      for (int a = 0; a < 3; ++a) pk.p[a] += s_rem * pk.u[a];
      pk.tau = 0.0;
      if (!interact(wk, &pk, seed, pid)) return;
      steps = 0;
      continue;
    }
    vox_tally(wk, v, pk.w, texit);
    for (int a = 0; a < 3; ++a) pk.p[a] += texit * pk.u[a];
    pk.tau -= mut * texit;
    int w2[3] = {v[0], v[1], v[2]};
    w2[ax] += pk.u[ax] > 0.0 ? 1 : -1;
    const int off_grid = w2[ax] < 0 || w2[ax] >= nd[ax];
    /* beyond the grid lies the ambient medium */
    int r2 = off_grid ? -1 : vox_region(s, vg, w2);
    double n1 = reg_n(s, pk.region), n2 = reg_n(s, r2);
    if (off_grid && n1 == n2) {
      int face = 2 * ax + (pk.u[ax] > 0.0 ? 1 : 0);
      pk.region = -1;
      wk->t->escaped_face[face] += pk.w;
      wk->t->escapes++;
      detect(wk, &pk, face, (face % 2) ? s->g_hi[face / 2] : s->g_lo[face / 2]);
      record(wk, &pk, ORC_EV_ESCAPE);
      return;
    }
    if (n1 == n2) {
      v[0] = w2[0]; v[1] = w2[1]; v[2] = w2[2];
      pk.region = r2;
      continue;
    }
    pk.k += 1;
    steps = 0;
    wk->t->events++;
    wk->t->interfaces++;
    double xi[4];
    event_xi(seed, pid, pk.k, xi);
    double ci = fabs(pk.u[ax]), ct;
    double R = orc_fresnel(n1, n2, ci, &ct);
    if (xi[0] < R) { /* reflect off the face, stay in v */
      pk.u[ax] = -pk.u[ax];
      wk->t->reflections++;
      record(wk, &pk, ORC_EV_REFLECT);
    } else {
      double eta = n1 / n2, sg = pk.u[ax] > 0.0 ? 1.0 : -1.0;
      for (int a = 0; a < 3; ++a) pk.u[a] *= eta;
      pk.u[ax] += (ct - eta * ci) * sg;
      double l = len3(pk.u);
      for (int a = 0; a < 3; ++a) pk.u[a] /= l;
      pk.region = r2;
      wk->t->refractions++;
      record(wk, &pk, ORC_EV_REFRACT);
      if (off_grid) { /* transmitted out of the grid */
        int face = 2 * ax + (sg > 0.0 ? 1 : 0);
        wk->t->escaped_face[face] += pk.w;
        wk->t->escapes++;
        detect(wk, &pk, face, (face % 2) ? s->g_hi[face / 2] : s->g_lo[face / 2]);
        record(wk, &pk, ORC_EV_ESCAPE);
        return;
      }
      v[0] = w2[0]; v[1] = w2[1]; v[2] = w2[2];
    }
  }
}

/* packets [first, first + n) over n_threads OpenMP threads in contiguous
 * chunks, each thread with private outputs, reduced in thread order; the
 * SDF walk, or the voxel walk when vg is given */
static int run_impl(const orc_scene* s, const voxel_geo* vg, uint64_t seed, uint64_t first, uint64_t n,
                    int n_threads, double* f, double* absorbed, double* image, orc_tallies* t) {
  int nt = 1;
#ifdef _OPENMP
  nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
  size_t nvox = (s->g_dims[0] > 0 && s->g_dims[1] > 0 && s->g_dims[2] > 0 && f)
                    ? (size_t)s->g_dims[0] * (size_t)s->g_dims[1] * (size_t)s->g_dims[2]
                    : 0;
  size_t npix = (image && s->det_dims[0] > 0 && s->det_dims[1] > 0)
                    ? (size_t)s->det_dims[0] * (size_t)s->det_dims[1]
                    : 0;
  double** fs = (double**)calloc((size_t)nt, sizeof(double*));
  double** as = (double**)calloc((size_t)nt, sizeof(double*));
  double** is = (double**)calloc((size_t)nt, sizeof(double*));
  orc_tallies* ts = (orc_tallies*)calloc((size_t)nt, sizeof(orc_tallies));
  int fail = !fs || !as || !is || !ts;
  for (int i = 0; !fail && i < nt; ++i) {
    fs[i] = nvox ? (double*)calloc(nvox, sizeof(double)) : NULL;
    as[i] = (double*)calloc((size_t)s->n_regions, sizeof(double));
    is[i] = npix ? (double*)calloc(npix, sizeof(double)) : NULL;
    if ((nvox && !fs[i]) || !as[i] || (npix && !is[i])) fail = 1;
  }
  if (!fail) {
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
      int me = 0;
#ifdef _OPENMP
      me = omp_get_thread_num();
#endif
      walker wk = {s, fs[me], as[me], &ts[me], NULL, 0, 0, is[me]};
      uint64_t lo = first + n * (uint64_t)me / (uint64_t)nt;
      uint64_t hi = first + n * (uint64_t)(me + 1) / (uint64_t)nt;
      for (uint64_t pid = lo; pid < hi; ++pid) {
        if (vg) walk_voxel(&wk, vg, seed, pid);
        else walk(&wk, seed, pid);
      }
    }
    for (int i = 0; i < nt; ++i) { /* reduce in thread order */
      for (size_t v = 0; v < nvox; ++v) f[v] += fs[i][v];
      for (size_t q = 0; q < npix; ++q) image[q] += is[i][q];
      for (int r = 0; r < s->n_regions; ++r) absorbed[r] += as[i][r];
      t->launched += ts[i].launched;
      for (int k = 0; k < 6; ++k) t->escaped_face[k] += ts[i].escaped_face[k];
      t->roulette_gain += ts[i].roulette_gain;
      t->roulette_loss += ts[i].roulette_loss;
      t->stalled += ts[i].stalled;
      t->events += ts[i].events;
      t->steps += ts[i].steps;
      t->interactions += ts[i].interactions;
      t->interfaces += ts[i].interfaces;
      t->reflections += ts[i].reflections;
      t->refractions += ts[i].refractions;
      t->crossings += ts[i].crossings;
      t->advances += ts[i].advances;
      t->voxel_segments += ts[i].voxel_segments;
      t->kills += ts[i].kills;
      t->stalls += ts[i].stalls;
      t->escapes += ts[i].escapes;
    }
  }
  for (int i = 0; i < nt; ++i) {
    if (fs) free(fs[i]);
    if (as) free(as[i]);
    if (is) free(is[i]);
  }
  free(fs); free(as); free(is); free(ts);
  return fail ? -2 : 0;
}

int orc_run_ex(const orc_scene* s, uint64_t seed, uint64_t first, uint64_t n, int n_threads, int voxel,
               double* f, double* absorbed, double* image, orc_tallies* t) {
  if (check_scene(s) != 0 || !absorbed || !t) return -1;
  if (!voxel) return run_impl(s, NULL, seed, first, n, n_threads, f, absorbed, image, t);
  const int* nd = s->g_dims;
  if (nd[0] <= 0 || nd[1] <= 0 || nd[2] <= 0) return -1;
  int8_t* vox = (int8_t*)malloc((size_t)nd[0] * (size_t)nd[1] * (size_t)nd[2]);
  if (!vox) return -2;
  orc_voxelize(s, vox);
  voxel_geo vg = {vox};
  int rc = run_impl(s, &vg, seed, first, n, n_threads, f, absorbed, image, t);
  free(vox);
  return rc;
}

int orc_run(const orc_scene* s, uint64_t seed, uint64_t first, uint64_t n,
            int n_threads, double* f, double* absorbed, orc_tallies* t) {
  return orc_run_ex(s, seed, first, n, n_threads, 0, f, absorbed, NULL, t);
}

int orc_run_voxel(const orc_scene* s, uint64_t seed, uint64_t first, uint64_t n, int n_threads, double* f,
                  double* absorbed, orc_tallies* t) {
  return orc_run_ex(s, seed, first, n, n_threads, 1, f, absorbed, NULL, t);
}

int orc_trace_voxel(const orc_scene* s, uint64_t seed, uint64_t pid, int cap, orc_event* out) {
  if (check_scene(s) != 0 || !out || cap < 1) return -1;
  const int* nd = s->g_dims;
  if (nd[0] <= 0 || nd[1] <= 0 || nd[2] <= 0) return -1;
  size_t nvox = (size_t)nd[0] * (size_t)nd[1] * (size_t)nd[2];
  int8_t* vox = (int8_t*)malloc(nvox);
  double* absorbed = (double*)calloc((size_t)s->n_regions, sizeof(double));
  if (!vox || !absorbed) { free(vox); free(absorbed); return -2; }
  orc_voxelize(s, vox);
  voxel_geo vg = {vox};
  orc_tallies t;
  memset(&t, 0, sizeof(t));
  walker wk = {s, NULL, absorbed, &t, out, cap, 0, NULL};
  walk_voxel(&wk, &vg, seed, pid);
  free(vox);
  free(absorbed);
  return wk.nrec;
}
