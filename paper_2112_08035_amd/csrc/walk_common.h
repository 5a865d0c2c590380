// walk_common.h -- device code shared by the SDF walk (walk.hip) and the
// voxel-model walk (voxel.hip): vector types, the Philox stream, scene
// table access, the region SDFs, the path-length tally, the packet state,
// emission, interactions, and the wave-level job picking and flushing.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/smcrt.h"
#include "layout.h"

namespace smcrt {

// Scene tables, primitives, uniform grids and job tables are read-only for a
// kernel's lifetime: they are read through the constant address space, so
// wave-uniform reads become scalar loads into SGPRs and per-lane reads plain
// global loads.  The fluence grid is written through the global space.
#define SMCRT_K __attribute__((address_space(4)))
#define SMCRT_G __attribute__((address_space(1)))
using ScP = const SMCRT_K SceneHeader*;
using RegRef = const SMCRT_K Region&;
using JobRef = const SMCRT_K WalkArgs&;
template <class X>
__device__ __forceinline__ const SMCRT_K X* kptr(const X* p) {
  return (const SMCRT_K X*)p;
}

// ------------------------------------------------------------------ types

template <typename T>
struct V3 {
  T x, y, z;
};
template <typename T>
__device__ __forceinline__ V3<T> mk(T x, T y, T z) { return V3<T>{x, y, z}; }
template <typename T>
__device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__device__ __forceinline__ V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T>
__device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __forceinline__ V3<double> to_d(V3<T> a) { return {(double)a.x, (double)a.y, (double)a.z}; }
template <typename T>
__device__ __forceinline__ V3<T> from_d(V3<double> a) { return {(T)a.x, (T)a.y, (T)a.z}; }

__device__ __forceinline__ float tsqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double tsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float tlog(float x) { return __logf(x); }
__device__ __forceinline__ double tlog(double x) { return log(x); }
__device__ __forceinline__ void tsincos_2pi(float xi, float* s, float* c) {
  float a = 6.2831853071795864769f * xi;
  *s = __sinf(a);
  *c = __cosf(a);
}
__device__ __forceinline__ void tsincos_2pi(double xi, double* s, double* c) { sincos(2.0 * M_PI * xi, s, c); }
__device__ __forceinline__ float tdiv(float a, float b) { return __fdividef(a, b); }
__device__ __forceinline__ double tdiv(double a, double b) { return a / b; }
// min, max, abs and clamp as single instructions (v_min/v_max, an abs
// source modifier, v_med3 for a clamp); a NaN operand yields the other one
template <typename T>
__device__ __forceinline__ T tmin(T a, T b) {
  if constexpr (sizeof(T) == 4) return __builtin_fminf(a, b);
  else return __builtin_fmin(a, b);
}
template <typename T>
__device__ __forceinline__ T tmax(T a, T b) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaxf(a, b);
  else return __builtin_fmax(a, b);
}
template <typename T>
__device__ __forceinline__ T tabs(T a) {
  if constexpr (sizeof(T) == 4) return __builtin_fabsf(a);
  else return __builtin_fabs(a);
}
template <typename T>
__device__ __forceinline__ T tclamp(T x, T lo, T hi) { return tmin(tmax(x, lo), hi); }
template <typename T>
__device__ __forceinline__ T tinf();
template <>
__device__ __forceinline__ float tinf<float>() { return __builtin_inff(); }
template <>
__device__ __forceinline__ double tinf<double>() { return __builtin_inf(); }

// ------------------------------------------------------------------ Philox

// Philox4x32-10 (Salmon et al., SC'11): ten rounds; each multiplies words 0
// and 2 by the round constants, swaps in the high halves xor-ed with the
// other words and the round key, and bumps the key by the Weyl constants.
struct U4 {
  uint32_t w0, w1, w2, w3;
};
__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t x0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
    const uint32_t x2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)m1;
    c3 = (uint32_t)m0;
    c0 = x0;
    c2 = x2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// a 32-bit word -> (m + 1/2) / 2^23 with m its top 23 bits; exact in FP32
template <typename T>
__device__ __forceinline__ T xi_of(uint32_t w) {
  return ((T)(w >> 9) + T(0.5)) * T(1.0 / 8388608.0);
}

// ------------------------------------------------------------------ scene

// the capsule table a staged-capsule workgroup holds in LDS (two float4 per
// capsule: a.x a.y a.z ba.x | ba.y ba.z 1/|ba|^2 r)
typedef float F4 __attribute__((ext_vector_type(4)));
using LdsCaps = const __attribute__((address_space(3))) F4*;

template <typename T>
struct Tab;
template <>
struct Tab<float> {
  static __device__ __forceinline__ const SMCRT_K PrimF* prims(JobRef a) { return kptr(a.pf); }
  static __device__ __forceinline__ const SMCRT_K float* caps(JobRef a) { return kptr(a.acc_capf); }
  static __device__ __forceinline__ float k(RegRef r) { return r.kf; }
  static __device__ __forceinline__ float inv_k(RegRef r) { return r.inv_kf; }
  static __device__ __forceinline__ float mut(RegRef r) { return r.mutf; }
  static __device__ __forceinline__ float inv_mut(RegRef r) { return r.inv_mutf; }
  static __device__ __forceinline__ V3<float> bb_c(ScP s) { return {s->bb_cf[0], s->bb_cf[1], s->bb_cf[2]}; }
  static __device__ __forceinline__ V3<float> bb_h(ScP s) { return {s->bb_hf[0], s->bb_hf[1], s->bb_hf[2]}; }
  static __device__ __forceinline__ float bb_c(ScP s, int i) { return s->bb_cf[i]; }
  static __device__ __forceinline__ float bb_h(ScP s, int i) { return s->bb_hf[i]; }
  static __device__ __forceinline__ V3<float> g_lo(ScP s) { return {s->g_lof[0], s->g_lof[1], s->g_lof[2]}; }
  static __device__ __forceinline__ V3<float> g_inv(ScP s) { return {s->g_inv_df[0], s->g_inv_df[1], s->g_inv_df[2]}; }
  static __device__ __forceinline__ float g_d(ScP s, int i) { return s->g_df[i]; }
  static __device__ __forceinline__ float g_lo(ScP s, int i) { return s->g_lof[i]; }
  static __device__ __forceinline__ float g_hi(ScP s, int i) { return s->g_hif[i]; }
  static __device__ __forceinline__ float delta(ScP s) { return s->deltaf; }
  static __device__ __forceinline__ float relax(ScP s) { return s->relaxf; }
  static __device__ __forceinline__ float relax_k(ScP s) { return s->relax_kf; }
  static __device__ __forceinline__ float amb_lo(ScP s, int r, int i) { return s->amb_lof[r][i]; }
  static __device__ __forceinline__ float amb_hi(ScP s, int r, int i) { return s->amb_hif[r][i]; }
  static __device__ __forceinline__ V3<float> acc_lo(const SMCRT_K Accel& A) { return {A.lof[0], A.lof[1], A.lof[2]}; }
  static __device__ __forceinline__ V3<float> acc_inv(const SMCRT_K Accel& A) { return {A.inv_cellf[0], A.inv_cellf[1], A.inv_cellf[2]}; }
  static __device__ __forceinline__ V3<float> acc_blo(const SMCRT_K Accel& A) { return {A.box_lof[0], A.box_lof[1], A.box_lof[2]}; }
  static __device__ __forceinline__ V3<float> acc_bhi(const SMCRT_K Accel& A) { return {A.box_hif[0], A.box_hif[1], A.box_hif[2]}; }
  static __device__ __forceinline__ float acc_margin(const SMCRT_K Accel& A) { return A.marginf; }
  static __device__ __forceinline__ float acc_cell_min(const SMCRT_K Accel& A) { return A.cell_minf; }
  static __device__ __forceinline__ float seg_err(ScP s) { return s->seg_errf; }
  // slack of a rate of approach: a few units in the last place
  static __device__ __forceinline__ float seg_eps() { return 0x1p-20f; }
};
template <>
struct Tab<double> {
  static __device__ __forceinline__ const SMCRT_K PrimD* prims(JobRef a) { return kptr(a.pd); }
  static __device__ __forceinline__ const SMCRT_K double* caps(JobRef a) { return kptr(a.acc_capd); }
  static __device__ __forceinline__ double k(RegRef r) { return r.k; }
  static __device__ __forceinline__ double inv_k(RegRef r) { return r.inv_k; }
  static __device__ __forceinline__ double mut(RegRef r) { return r.mut; }
  static __device__ __forceinline__ double inv_mut(RegRef r) { return r.inv_mut; }
  static __device__ __forceinline__ V3<double> bb_c(ScP s) { return {s->bb_c[0], s->bb_c[1], s->bb_c[2]}; }
  static __device__ __forceinline__ V3<double> bb_h(ScP s) { return {s->bb_h[0], s->bb_h[1], s->bb_h[2]}; }
  static __device__ __forceinline__ double bb_c(ScP s, int i) { return s->bb_c[i]; }
  static __device__ __forceinline__ double bb_h(ScP s, int i) { return s->bb_h[i]; }
  static __device__ __forceinline__ V3<double> g_lo(ScP s) { return {s->g_lo[0], s->g_lo[1], s->g_lo[2]}; }
  static __device__ __forceinline__ V3<double> g_inv(ScP s) { return {s->g_inv_d[0], s->g_inv_d[1], s->g_inv_d[2]}; }
  static __device__ __forceinline__ double g_d(ScP s, int i) { return s->g_d[i]; }
  static __device__ __forceinline__ double g_lo(ScP s, int i) { return s->g_lo[i]; }
  static __device__ __forceinline__ double g_hi(ScP s, int i) { return s->g_hi[i]; }
  static __device__ __forceinline__ double delta(ScP s) { return s->delta; }
  static __device__ __forceinline__ double relax(ScP s) { return s->relax; }
  static __device__ __forceinline__ double relax_k(ScP s) { return s->relax_k; }
  static __device__ __forceinline__ double amb_lo(ScP s, int r, int i) { return s->amb_lo[r][i]; }
  static __device__ __forceinline__ double amb_hi(ScP s, int r, int i) { return s->amb_hi[r][i]; }
  static __device__ __forceinline__ V3<double> acc_lo(const SMCRT_K Accel& A) { return {A.lo[0], A.lo[1], A.lo[2]}; }
  static __device__ __forceinline__ V3<double> acc_inv(const SMCRT_K Accel& A) { return {A.inv_cell[0], A.inv_cell[1], A.inv_cell[2]}; }
  static __device__ __forceinline__ V3<double> acc_blo(const SMCRT_K Accel& A) { return {A.box_lo[0], A.box_lo[1], A.box_lo[2]}; }
  static __device__ __forceinline__ V3<double> acc_bhi(const SMCRT_K Accel& A) { return {A.box_hi[0], A.box_hi[1], A.box_hi[2]}; }
  static __device__ __forceinline__ double acc_margin(const SMCRT_K Accel& A) { return A.margin; }
  static __device__ __forceinline__ double acc_cell_min(const SMCRT_K Accel& A) { return A.cell_min; }
  static __device__ __forceinline__ double seg_err(ScP s) { return s->seg_err; }
  static __device__ __forceinline__ double seg_eps() { return 1e-12; }
};

// exact Euclidean SDF of one primitive's shape in its own frame (Sec. 2.2;
// Eq. 3 for the sphere)
template <typename T>
__device__ __forceinline__ T shape_sdf(const SMCRT_K Prim<T>* P, int i, V3<T> p) {
  const int kind = P[i].kind;
  const SMCRT_K T* v = P[i].v;
  const V3<T> q = p - mk(v[0], v[1], v[2]);
  if (kind == kSphere) return tsqrt(dot(q, q)) - v[3];
  if (kind == kBox) {
    const T ex = tabs(q.x) - v[3], ey = tabs(q.y) - v[4], ez = tabs(q.z) - v[5];
    const V3<T> o = mk(tmax(ex, T(0)), tmax(ey, T(0)), tmax(ez, T(0)));
    return tsqrt(dot(o, o)) + tmin(tmax(ex, tmax(ey, ez)), T(0));
  }
  const V3<T> e = mk(v[3], v[4], v[5]);
  if (kind == kTorus) {  // e unit axis, v[6] = ring radius R, v[7] = tube radius r
    const T x = dot(q, e);
    const V3<T> rad = q - x * e;
    const T rho = tsqrt(dot(rad, rad)) - v[6];
    return tsqrt(rho * rho + x * x) - v[7];
  }
  if (kind == kCapsule) {  // e = b - a, v[6] = 1/|b-a|^2
    const T t = tclamp(dot(q, e) * v[6], T(0), T(1));
    const V3<T> d = q - t * e;
    return tsqrt(dot(d, d)) - v[7];
  }
  // capped cylinder: e unit axis, v[6] = L, v[7] = L/2, v[8] = r
  const T x = dot(q, e);
  const V3<T> rad = q - x * e;
  const T q1 = tsqrt(dot(rad, rad)) - v[8];
  const T q2 = tabs(x - v[7]) - v[7];
  const T o1 = tmax(q1, T(0)), o2 = tmax(q2, T(0));
  return tmin(tmax(q1, q2), T(0)) + tsqrt(o1 * o1 + o2 * o2);
}

// sin and cos of a twist or displacement angle (moderate arguments):
// Cody-Waite reduction by pi/2, split into the precision's nearest value and
// its residual, to r in [-pi/4, pi/4], then the Taylor series of sin and cos
// to r^17 / r^16 (FP64: last term < 4e-18) or r^11 / r^10 (FP32: < 1e-9),
// evaluated by Horner's rule; the quadrant n mod 4 picks signs and order.
// Kept in registers: the library routine's reduction for huge arguments
// needs a stack array, which in the sphere-tracing loop moved other
// values to scratch.
template <typename T>
__device__ __forceinline__ void tsincos(T a, T* sn, T* cs) {
  const T n = rint(a * T(0.63661977236758134308));  // 2/pi
  // pi/2 = hi + lo: FP64 0x3FF921FB54442D18 + 6.1232e-17, FP32 0x3FC90FDB - 4.3711e-8
  const T hi = sizeof(T) == 8 ? T(1.5707963267948966) : T(1.57079637050628662109375);
  const T lo = sizeof(T) == 8 ? T(6.123233995736766e-17) : T(-4.371139000186241e-08);
  const T r = (a - n * hi) - n * lo;
  const T r2 = r * r;
  T s, c;
  if constexpr (sizeof(T) == 8) {
    s = T(1) / T(355687428096000);
    s = s * -r2 + T(1) / T(1307674368000);
    s = s * -r2 + T(1) / T(6227020800);
    s = s * -r2 + T(1) / T(39916800);
    s = s * -r2 + T(1) / T(362880);
    s = s * -r2 + T(1) / T(5040);
    s = s * -r2 + T(1) / T(120);
    s = s * -r2 + T(1) / T(6);
    s = r - r * r2 * s;
    c = T(1) / T(20922789888000);
    c = c * -r2 + T(1) / T(87178291200);
    c = c * -r2 + T(1) / T(479001600);
    c = c * -r2 + T(1) / T(3628800);
    c = c * -r2 + T(1) / T(40320);
    c = c * -r2 + T(1) / T(720);
    c = c * -r2 + T(1) / T(24);
    c = c * -r2 + T(1) / T(2);
    c = T(1) - r2 * c;
  } else {
    s = T(1) / T(39916800);
    s = s * -r2 + T(1) / T(362880);
    s = s * -r2 + T(1) / T(5040);
    s = s * -r2 + T(1) / T(120);
    s = s * -r2 + T(1) / T(6);
    s = r - r * r2 * s;
    c = T(1) / T(3628800);
    c = c * -r2 + T(1) / T(40320);
    c = c * -r2 + T(1) / T(720);
    c = c * -r2 + T(1) / T(24);
    c = c * -r2 + T(1) / T(2);
    c = T(1) - r2 * c;
  }
  const int q = ((int)n) & 3;
  *sn = q == 0 ? s : (q == 1 ? c : (q == 2 ? -s : -c));
  *cs = q == 0 ? c : (q == 1 ? -s : (q == 2 ? -c : s));
}

// SDF of primitive i (Sec. 2.2: SDFs are translated, rotated, scaled,
// twisted and bent).  Placement with uniform scale keeps the distance exact
// (times s), and so do rounding and the onion shell.  A twist or a bend
// keeps the sign; inside its bounding cylinder (radius rho) the distance is
// divided by the untwist (unbend) map's Lipschitz bound there, the largest
// singular value of its Jacobian, (k rho + sqrt((k rho)^2 + 4)) / 2 for a
// twist and 1 + k rho for a bend; outside it the distance to the cylinder
// is used.  The flags are the
// same for every lane (primitives are visited in a wave-uniform order).
// distance from (x, y) to the segment (ax, ay)-(bx, by)
template <typename T>
__device__ __forceinline__ T seg2_dist(T x, T y, T ax, T ay, T bx, T by) {
  const T dx = bx - ax, dy = by - ay, px = x - ax, py = y - ay;
  const T t = tclamp((px * dx + py * dy) / (dx * dx + dy * dy), T(0), T(1));
  const T ex = px - t * dx, ey = py - t * dy;
  return tsqrt(ex * ex + ey * ey);
}

// distance from p to the segment a-b
template <typename T>
__device__ __forceinline__ T seg3_dist(V3<T> p, V3<T> a, V3<T> b) {
  const V3<T> ba = b - a, pa = p - a;
  const T t = tclamp(dot(pa, ba) / dot(ba, ba), T(0), T(1));
  const V3<T> d = pa - t * ba;
  return tsqrt(dot(d, d));
}

// further gallery shapes in their own frame (Sec. 2.2, Fig. 1's basic
// shapes): capped cone, octahedron and hexagonal prism (exact distances),
// ellipsoid (a lower bound with the exact sign)
template <typename T>
__device__ __forceinline__ T further_shape_sdf(const SMCRT_K Prim<T>* P, int i, V3<T> p) {
  const int kind = P[i].kind;
  const SMCRT_K T* v = P[i].v;
  const V3<T> q = p - mk(v[0], v[1], v[2]);
  if (kind == kCone) {  // (axial x, radial y) half plane: the two caps and the slanted side
    const V3<T> e = mk(v[3], v[4], v[5]);
    const T L = v[6], ra = v[7], rb = v[8];
    const T x = dot(q, e);
    const V3<T> rad = q - x * e;
    const T y = tsqrt(dot(rad, rad));
    const T d = tmin(tmin(seg2_dist(x, y, T(0), T(0), T(0), ra), seg2_dist(x, y, L, T(0), L, rb)),
                     seg2_dist(x, y, T(0), ra, L, rb));
    const bool inside = x > T(0) && x < L && y < ra + (rb - ra) * x / L;
    return inside ? -d : d;
  }
  if (kind == kOctahedron) {  // by symmetry the face in the positive octant
    const T s = v[3];
    const V3<T> a = mk(tabs(q.x), tabs(q.y), tabs(q.z));
    const T m = a.x + a.y + a.z - s;
    const T third = m * T(1.0 / 3.0);
    if (m <= T(0) || (a.x >= third && a.y >= third && a.z >= third)) return m * T(0.57735026918962576451);
    const V3<T> v0 = mk(s, T(0), T(0)), v1 = mk(T(0), s, T(0)), v2 = mk(T(0), T(0), s);
    return tmin(tmin(seg3_dist(a, v0, v1), seg3_dist(a, v1, v2)), seg3_dist(a, v2, v0));
  }
  if (kind == kHexPrism) {  // first quadrant: edges (R,0)-(R/2,h) and (R/2,h)-(-R/2,h)
    const T h = v[3], hz = v[4], R = v[5];
    const T x = tabs(q.x), y = tabs(q.y);
    T d2 = tmin(seg2_dist(x, y, R, T(0), T(0.5) * R, h), seg2_dist(x, y, T(0.5) * R, h, T(-0.5) * R, h));
    if (y < h && T(1.7320508075688772935) * x + y < T(2) * h) d2 = -d2;
    const T dz = tabs(q.z) - hz;
    const T o1 = tmax(d2, T(0)), o2 = tmax(dz, T(0));
    return tmin(tmax(d2, dz), T(0)) + tsqrt(o1 * o1 + o2 * o2);
  }
  // ellipsoid: rmin (|q / r| - 1), 1-Lipschitz and zero on the surface
  const V3<T> u = mk(q.x * v[3], q.y * v[4], q.z * v[5]);
  return v[6] * (tsqrt(dot(u, u)) - T(1));
}

template <typename T>
__device__ __attribute__((noinline)) T placed_prim_sdf(const SMCRT_K Prim<T>* P, int i, V3<T> p) {
  const SMCRT_K Prim<T>& Q = P[i];
  const int fl = Q.flags;
  V3<T> q = p;
  if (fl & kPlaced) {
    const V3<T> d = p - mk(Q.t[0], Q.t[1], Q.t[2]);
    q = mk(Q.m[0] * d.x + Q.m[1] * d.y + Q.m[2] * d.z, Q.m[3] * d.x + Q.m[4] * d.y + Q.m[5] * d.z,
           Q.m[6] * d.x + Q.m[7] * d.y + Q.m[8] * d.z);
  }
  // repetition: to the nearest copy; b = distance to the nearest face of its
  // cell with another copy behind it
  T b = tinf<T>();
  if (fl & kRepeated) {
    T c3[3] = {q.x, q.y, q.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int n = Q.rep_n[a];
      const T c = Q.rep_c[a], half = T(0.5) * T(n - 1) * c;
      // clamp before converting: a far point must not overflow the int
      const int k = (int)tclamp(floor((c3[a] + half) / c + T(0.5)), T(0), T(n - 1));
      c3[a] -= T(k) * c - half;
      if (c3[a] > T(0) && k < n - 1) b = tmin(b, T(0.5) * c - c3[a]);
      if (c3[a] < T(0) && k > 0) b = tmin(b, T(0.5) * c + c3[a]);
    }
    q = mk(c3[0], c3[1], c3[2]);
  }
  T dcyl = T(0);
  if (fl & kTwisted) {  // distance to the bounding cylinder, then untwist by -k z (unbend: -k x) about z
    const T q1 = tsqrt(q.x * q.x + q.y * q.y) - Q.twist_rho;
    const T q2 = tabs(q.z - Q.twist_zc) - Q.twist_zh;
    const T o1 = tmax(q1, T(0)), o2 = tmax(q2, T(0));
    dcyl = tmin(tmax(q1, q2), T(0)) + tsqrt(o1 * o1 + o2 * o2);
    T sn, cs;
    tsincos(-Q.twist_k * ((fl & kBent) ? q.x : q.z), &sn, &cs);
    q = mk(cs * q.x - sn * q.y, sn * q.x + cs * q.y, q.z);
  }
  const V3<T> e = mk(q.x - tclamp(q.x, -Q.elong[0], Q.elong[0]), q.y - tclamp(q.y, -Q.elong[1], Q.elong[1]),
                     q.z - tclamp(q.z, -Q.elong[2], Q.elong[2]));
  T d = ((fl & kFurtherShape) ? further_shape_sdf(P, i, e) : shape_sdf(P, i, e)) - Q.round_r;
  if (Q.onion_t > T(0)) d = tabs(d) - Q.onion_t;
  if (Q.disp_a > T(0)) {
    T sx, cx, sy, cy, sz, cz;
    tsincos(Q.disp_f * q.x, &sx, &cx);
    tsincos(Q.disp_f * q.y, &sy, &cy);
    tsincos(Q.disp_f * q.z, &sz, &cz);
    d = (d + Q.disp_a * sx * sy * sz) * Q.disp_inv_lip;
  }
  if (fl & kTwisted) d = dcyl > T(0) ? dcyl : d * Q.inv_lip;
  if (fl & kRepeated) d = tmin(d, Q.rep_gap + b);
  if (fl & kPlaced) d *= Q.s;
  return d;
}

// XF: the scene has placed or modified primitives.  Scenes without them
// run kernels that never call placed_prim_sdf: a call in the sphere-tracing
// loop makes the caller keep its live values out of the registers the
// callee may use, which pushed the FP32 walk over its register budget.
template <typename T, bool XF>
__device__ __forceinline__ T prim_sdf(const SMCRT_K Prim<T>* P, int i, V3<T> p) {
  if constexpr (XF) {
    if (P[i].flags != 0) return placed_prim_sdf<T>(P, i, p);
  }
  return shape_sdf(P, i, p);
}

// region SDF from its primitives in order (CSG of Sec. 2.2): union (min),
// polynomial smooth union, intersection (max) or difference, the first
// primitive minus the others (max(d, -d_i)).  Intersection and difference
// are lower bounds of the distance with Lipschitz constant 1, so sphere
// tracing stays conservative.
template <typename T, bool XF>
__device__ __forceinline__ T region_sdf(JobRef a, RegRef R, V3<T> p) {
  const SMCRT_K Prim<T>* P = Tab<T>::prims(a);
  const int op = R.op;  // wave uniform: one loop, primitive SDFs inlined once
  T d = prim_sdf<T, XF>(P, R.first, p);
  for (int i = 1; i < R.count; ++i) {
    const T b = prim_sdf<T, XF>(P, R.first + i, p);
    if (op == kSmoothUnion) {
      const T h = tclamp(T(0.5) + T(0.5) * (b - d) * Tab<T>::inv_k(R), T(0), T(1));
      d = h * d + (T(1) - h) * b - Tab<T>::k(R) * h * (T(1) - h);
    } else {
      const T nb = op == kSubtract ? -b : b;
      d = op == kUnion ? tmin(d, nb) : tmax(d, nb);
    }
  }
  return d;
}

// capsule SDF from a compact record c = (a, b - a, 1/|b - a|^2, r): the
// capsule branch of shape_sdf, operation for operation
template <typename T>
__device__ __forceinline__ T cap_sdf(T a0, T a1, T a2, T e0, T e1, T e2, T inv, T r, V3<T> p) {
  const V3<T> q = p - mk(a0, a1, a2);
  const V3<T> e = mk(e0, e1, e2);
  const T t = tclamp(dot(q, e) * inv, T(0), T(1));
  const V3<T> d = q - t * e;
  return tsqrt(dot(d, d)) - r;
}

// Lower bound of the accelerated region's SDF at p in a cell that lists no
// primitive, from the cell's ring distance k (in cells) to the nearest cell
// that lists one: every surface point lies in such a cell, so the surface is
// at least k - 1 whole cells plus p's way to its own cell's faces away (the
// smallest side counted; cell coordinates cx, cy, cz of p and its cell
// ix, iy, iz).  Never below the margin; a relative 2^-20 less against
// rounding.
template <typename T>
__device__ __forceinline__ T ring_bound(JobRef a, const SMCRT_K Accel& A, int c, T cx, T cy, T cz, int ix, int iy,
                                        int iz) {
  const T m = Tab<T>::acc_margin(A);
  if (a.acc_rings == nullptr) return m;
  const uint32_t k = kptr(a.acc_rings)[c];
  const T fx = cx - T(ix), fy = cy - T(iy), fz = cz - T(iz);
  const T f = tmin(tmin(tmin(fx, T(1) - fx), tmin(fy, T(1) - fy)), tmin(fz, T(1) - fz));
  const T r = (T(k) - T(1) + tmax(f, T(0))) * Tab<T>::acc_cell_min(A) * (T(1) - T(0x1p-20));
  return tmax(m, r);
}

// SDF of the accelerated region through its uniform grid: min(margin, min
// over the primitives listed in p's cell).  Equal to the region SDF where
// that is below the margin, a lower bound elsewhere; outside the grid box
// (which is the primitives' box grown by the margin) the distance to the
// primitives' box is the lower bound.  Every index is checked.  Regions of
// plain capsules read their compact records: from the workgroup's LDS
// table when lds is given (FP32 staged walk), else from global memory.
template <typename T, bool XF>
__device__ __forceinline__ T accel_sdf(JobRef a, V3<T> p, LdsCaps lds = nullptr) {
  const SMCRT_K Accel& A = kptr(a.sc)->acc;
  const V3<T> lo = Tab<T>::acc_lo(A), ic = Tab<T>::acc_inv(A);
  const T cx = (p.x - lo.x) * ic.x, cy = (p.y - lo.y) * ic.y, cz = (p.z - lo.z) * ic.z;
  const int dx = A.dims[0], dy = A.dims[1], dz = A.dims[2];
  if (!(cx >= T(0) && cy >= T(0) && cz >= T(0) && cx < T(dx) && cy < T(dy) && cz < T(dz))) {
    const V3<T> bl = Tab<T>::acc_blo(A), bh = Tab<T>::acc_bhi(A);
    const V3<T> o = mk(tmax(tmax(bl.x - p.x, p.x - bh.x), T(0)), tmax(tmax(bl.y - p.y, p.y - bh.y), T(0)),
                       tmax(tmax(bl.z - p.z, p.z - bh.z), T(0)));
    return tsqrt(dot(o, o));
  }
  int ix = (int)cx, iy = (int)cy, iz = (int)cz;
  ix = ix < dx ? ix : dx - 1;
  iy = iy < dy ? iy : dy - 1;
  iz = iz < dz ? iz : dz - 1;
  const int c = ix + dx * (iy + dy * iz);
  const SMCRT_K uint32_t* offs = kptr(a.acc_offsets);
  const SMCRT_K uint32_t* ids = kptr(a.acc_ids);
  const uint32_t b = offs[c];
  uint64_t e = offs[c + 1];
  e = e < A.capacity ? e : A.capacity;
  const SMCRT_K Prim<T>* P = Tab<T>::prims(a);
  if (b >= e) return ring_bound<T>(a, A, c, cx, cy, cz, ix, iy, iz);
  const uint32_t lo_id = (uint32_t)A.first_prim, hi_id = (uint32_t)(A.first_prim + A.n_prims);
  T d = Tab<T>::acc_margin(A);
  if (A.caps) {
    if constexpr (sizeof(T) == 4) {
      if (lds) {
        for (uint64_t i = b; i < e; ++i) {
          const uint32_t id = ids[i];
          if (id >= lo_id && id < hi_id) {
            const uint32_t k = id - lo_id;
            const F4 x = lds[2 * k], y = lds[2 * k + 1];
            d = tmin(d, cap_sdf<T>(x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w, p));
          }
        }
        return d;
      }
    }
    const SMCRT_K T* C = Tab<T>::caps(a);
    for (uint64_t i = b; i < e; ++i) {
      const uint32_t id = ids[i];
      if (id >= lo_id && id < hi_id) {
        const SMCRT_K T* c = C + 8 * (size_t)(id - lo_id);
        d = tmin(d, cap_sdf<T>(c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7], p));
      }
    }
    return d;
  }
  for (uint64_t i = b; i < e; ++i) {
    const uint32_t id = ids[i];
    if (id >= lo_id && id < hi_id) d = tmin(d, prim_sdf<T, XF>(P, (int)id, p));
  }
  return d;
}

// SDF of region r (through the grid when r is the accelerated region)
template <typename T, bool XF>
__device__ __forceinline__ T region_dist(JobRef a, int r, V3<T> p, LdsCaps lds = nullptr) {
  if (r == a.acc_region) return accel_sdf<T, XF>(a, p, lds);
  return region_sdf<T, XF>(a, kptr(a.sc)->reg[r], p);
}

// owner of a point: the highest-index region with a negative SDF, else the
// ambient slot n_regions
template <typename T, bool XF>
__device__ __forceinline__ int region_of(JobRef a, V3<T> p) {
  ScP sc = kptr(a.sc);
  const int nr = sc->n_regions;
  int owner = nr;
  for (int r = nr - 1; r >= 0; --r) {
    if (region_dist<T, XF>(a, r, p) < T(0)) {
      owner = r;
      break;
    }
  }
  return owner;
}

// Outside the simulation volume (Sec. 2.3: escape when the volume's box
// SDF is positive).  The box SDF is positive exactly when the largest of
// |q_i| - h_i is, so the sign needs no square root; face = 2*axis + side of
// that largest component, the face the packet left through.
template <typename T>
__device__ __forceinline__ bool outside_volume(ScP sc, V3<T> p, int* face) {
  const V3<T> c = Tab<T>::bb_c(sc), h = Tab<T>::bb_h(sc);
  const V3<T> q = p - c;
  const T ex = tabs(q.x) - h.x, ey = tabs(q.y) - h.y, ez = tabs(q.z) - h.z;
  int ax = 0;
  T best = ex;
  if (ey > best) { best = ey; ax = 1; }
  if (ez > best) { best = ez; ax = 2; }
  const T qa = ax == 0 ? q.x : (ax == 1 ? q.y : q.z);
  *face = 2 * ax + (qa > T(0) ? 1 : 0);
  return best > T(0);
}

// Ambient skip: outside every region, the straight path from p along u
// cuts no surface before it enters the box of some region's surface; when
// it enters none inside the volume, only the volume's boundary lies ahead.
// Returns the path to the first such box, or delta past the boundary; 0
// when p is inside a box.  (u == 0 on an axis: the box is met only when p
// lies between its planes.)
template <typename T>
__device__ __forceinline__ T ambient_free(ScP sc, int nr, V3<T> p, V3<T> u, T delta) {
  const V3<T> c = Tab<T>::bb_c(sc), h = Tab<T>::bb_h(sc);
  const T pv[3] = {p.x, p.y, p.z}, uv[3] = {u.x, u.y, u.z};
  const T cv[3] = {c.x, c.y, c.z}, hv[3] = {h.x, h.y, h.z};
  T rv[3];
  T t = tinf<T>();
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    rv[i] = T(1) / uv[i];
    if (uv[i] != T(0)) t = tmin(t, ((uv[i] > T(0) ? cv[i] + hv[i] : cv[i] - hv[i]) - pv[i]) * rv[i]);
  }
  t += delta;
  for (int r = 0; r < nr; ++r) {
    T t0 = T(0), t1 = t;
    bool hit = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T lo = Tab<T>::amb_lo(sc, r, i), hi = Tab<T>::amb_hi(sc, r, i);
      if (uv[i] == T(0)) {
        hit = hit && pv[i] >= lo && pv[i] <= hi;
      } else {
        const T ta = (lo - pv[i]) * rv[i], tb = (hi - pv[i]) * rv[i];
        t0 = tmax(t0, tmin(ta, tb));
        t1 = tmin(t1, tmax(ta, tb));
      }
    }
    if (hit && t0 <= t1) t = t0;
  }
  return t;
}

// ---- segment tracing (Sec. 5 names it beside enhanced sphere tracing as a
// cure for the many small steps of rays that run along surfaces).  Outside
// a convex shape the exact distance along a ray, f(t) = d(p + t u), is a
// convex function of t and never falls below its tangent f(0) - c t, where
// c = -grad d . u is the rate at which the ray approaches the shape: the ray
// cannot reach the shape before f(0) / c, nor ever when c <= 0.  A union is
// reached when one member is (the smallest bound), an intersection only when
// every member is (the largest bound), a subtraction not before its first
// member.  Rounding: f(0) is taken less err, the scene's bound on the
// rounding of a distance, and c more err / f(0) (the gradient is the
// direction of a difference known to err) plus a few units in the last
// place.

// the length a ray runs before it can reach a convex shape at distance a
// that it approaches at rate c = -dv / l (dv = v . u for a vector v of
// length l > 0 from the nearest surface point towards p), with the rounding
// slack: (a - err) / (c + err / a + eps), taken as l a (a - err) / (l (err
// + eps a) - a dv), one division.  0 when a is within the rounding (or the
// rate is not a number), infinite when the ray moves away.
template <typename T>
__device__ __forceinline__ T tangent_bound(T a, T dv, T l, T err) {
  if (!(a > err)) return T(0);
  const T den = l * (err + Tab<T>::seg_eps() * a) - a * dv;
  if (den > T(0)) return tdiv(l * a * (a - err), den);
  return den <= T(0) ? tinf<T>() : T(0);
}

// distance of a plain convex primitive (sphere, box, capsule or capped
// cylinder, unplaced and unmodified) at p, computed as shape_sdf computes
// it, and the ray's rate of approach to it as -(*dv) / (*l): v points from
// the nearest surface point towards p (meaningful outside the shape)
template <typename T>
__device__ __forceinline__ T convex_sdf_rate(const SMCRT_K Prim<T>* P, int i, V3<T> p, V3<T> u, T* dv, T* l) {
  const int kind = P[i].kind;
  const SMCRT_K T* v = P[i].v;
  const V3<T> q = p - mk(v[0], v[1], v[2]);
  if (kind == kSphere) {
    *l = tsqrt(dot(q, q));
    *dv = dot(q, u);
    return *l - v[3];
  }
  if (kind == kBox) {
    const T ex = tabs(q.x) - v[3], ey = tabs(q.y) - v[4], ez = tabs(q.z) - v[5];
    const V3<T> o = mk(tmax(ex, T(0)), tmax(ey, T(0)), tmax(ez, T(0)));
    *l = tsqrt(dot(o, o));
    *dv = (q.x < T(0) ? -o.x : o.x) * u.x + (q.y < T(0) ? -o.y : o.y) * u.y + (q.z < T(0) ? -o.z : o.z) * u.z;
    return *l + tmin(tmax(ex, tmax(ey, ez)), T(0));
  }
  const V3<T> e = mk(v[3], v[4], v[5]);
  if (kind == kCapsule) {
    const T t = tclamp(dot(q, e) * v[6], T(0), T(1));
    const V3<T> d = q - t * e;
    *l = tsqrt(dot(d, d));
    *dv = dot(d, u);
    return *l - v[7];
  }
  // capped cylinder, in the half plane of (radial, axial) coordinates: v =
  // o1 rad / rho +/- o2 e, scaled by rho when o1 > 0
  const T x = dot(q, e);
  const V3<T> rad = q - x * e;
  const T rho = tsqrt(dot(rad, rad));
  const T q1 = rho - v[8];
  const T q2 = tabs(x - v[7]) - v[7];
  const T o1 = tmax(q1, T(0)), o2 = tmax(q2, T(0));
  const T len = tsqrt(o1 * o1 + o2 * o2);
  const T sc = o1 > T(0) ? rho : T(1);
  *l = sc * len;
  *dv = o1 * dot(rad, u) + (x > v[7] ? o2 : -o2) * sc * dot(e, u);
  return tmin(tmax(q1, q2), T(0)) + len;
}

// the accelerated region's distance (accel_sdf's value) and in *tb the
// way along u to its surface: inside the grid, the capsules listed in p's
// cell bound it by their tangents, and every other primitive lies farther
// than the margin; outside the grid (and for regions without a rule) the
// distance alone
template <typename T, bool XF>
__device__ __forceinline__ T accel_seg(JobRef a, V3<T> p, V3<T> u, T err, T* tb) {
  const SMCRT_K Accel& A = kptr(a.sc)->acc;
  const int rule = kptr(a.sc)->reg[A.region].seg;
  const V3<T> lo = Tab<T>::acc_lo(A), ic = Tab<T>::acc_inv(A);
  const T cx = (p.x - lo.x) * ic.x, cy = (p.y - lo.y) * ic.y, cz = (p.z - lo.z) * ic.z;
  const int dx = A.dims[0], dy = A.dims[1], dz = A.dims[2];
  if (rule != kSegUnion || !(cx >= T(0) && cy >= T(0) && cz >= T(0) && cx < T(dx) && cy < T(dy) && cz < T(dz))) {
    const T d = accel_sdf<T, XF>(a, p);
    *tb = tabs(d);
    return d;
  }
  int ix = (int)cx, iy = (int)cy, iz = (int)cz;
  ix = ix < dx ? ix : dx - 1;
  iy = iy < dy ? iy : dy - 1;
  iz = iz < dz ? iz : dz - 1;
  const int cell = ix + dx * (iy + dy * iz);
  const SMCRT_K uint32_t* offs = kptr(a.acc_offsets);
  const SMCRT_K uint32_t* ids = kptr(a.acc_ids);
  const uint32_t b = offs[cell];
  uint64_t e = offs[cell + 1];
  e = e < A.capacity ? e : A.capacity;
  if (b >= e) {
    const T d = ring_bound<T>(a, A, cell, cx, cy, cz, ix, iy, iz);
    *tb = d;
    return d;
  }
  const uint32_t lo_id = (uint32_t)A.first_prim, hi_id = (uint32_t)(A.first_prim + A.n_prims);
  T d = Tab<T>::acc_margin(A), t = d;
  if (A.caps) {
    const SMCRT_K T* C = Tab<T>::caps(a);
    for (uint64_t i = b; i < e; ++i) {
      const uint32_t id = ids[i];
      if (id >= lo_id && id < hi_id) {
        const SMCRT_K T* r = C + 8 * (size_t)(id - lo_id);
        const V3<T> q = p - mk(r[0], r[1], r[2]);
        const V3<T> ax = mk(r[3], r[4], r[5]);
        const T s = tclamp(dot(q, ax) * r[6], T(0), T(1));
        const V3<T> w = q - s * ax;
        const T l = tsqrt(dot(w, w));
        const T di = l - r[7];
        d = tmin(d, di);
        t = tmin(t, tangent_bound<T>(di, dot(w, u), l, err));
      }
    }
  } else {
    const SMCRT_K Prim<T>* P = Tab<T>::prims(a);
    for (uint64_t i = b; i < e; ++i) {
      const uint32_t id = ids[i];
      if (id >= lo_id && id < hi_id) {
        T dv, l;
        const T di = convex_sdf_rate<T>(P, (int)id, p, u, &dv, &l);
        d = tmin(d, di);
        t = tmin(t, tangent_bound<T>(di, dv, l, err));
      }
    }
  }
  *tb = d > T(0) ? tmax(d, t) : tabs(d);
  return d;
}

// distance of region r at p (region_dist's value) and in *tb a length the
// ray along u runs before it can meet the region's surface: from outside a
// region with a rule, the tangent bounds of its members; else the
// distance's magnitude
template <typename T, bool XF>
__device__ __forceinline__ T region_seg(JobRef a, int r, V3<T> p, V3<T> u, T err, T* tb) {
  if (r == a.acc_region) return accel_seg<T, XF>(a, p, u, err, tb);
  const SMCRT_K Region& R = kptr(a.sc)->reg[r];
  const int rule = R.seg;  // wave uniform
  if (rule == kSegNone) {
    const T d = region_sdf<T, XF>(a, R, p);
    *tb = tabs(d);
    return d;
  }
  const SMCRT_K Prim<T>* P = Tab<T>::prims(a);
  T dv, l;
  T d = convex_sdf_rate<T>(P, R.first, p, u, &dv, &l);
  T t = tangent_bound<T>(d, dv, l, err);
  if (rule == kSegSubtract) {
    for (int i = 1; i < R.count; ++i) d = tmax(d, -prim_sdf<T, XF>(P, R.first + i, p));
  } else {
    for (int i = 1; i < R.count; ++i) {
      const T di = convex_sdf_rate<T>(P, R.first + i, p, u, &dv, &l);
      const T ti = tangent_bound<T>(di, dv, l, err);
      if (rule == kSegUnion) {
        d = tmin(d, di);
        t = tmin(t, ti);
      } else {
        d = tmax(d, di);
        t = tmax(t, ti);
      }
    }
  }
  *tb = d > T(0) ? tmax(d, t) : tabs(d);
  return d;
}

// the way along u out of the simulation volume
template <typename T>
__device__ __forceinline__ T volume_exit(ScP sc, V3<T> p, V3<T> u) {
  const V3<T> c = Tab<T>::bb_c(sc), h = Tab<T>::bb_h(sc);
  const T pv[3] = {p.x, p.y, p.z}, uv[3] = {u.x, u.y, u.z};
  const T cv[3] = {c.x, c.y, c.z}, hv[3] = {h.x, h.y, h.z};
  T t = tinf<T>();
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (uv[i] != T(0)) t = tmin(t, tdiv((uv[i] > T(0) ? cv[i] + hv[i] : cv[i] - hv[i]) - pv[i], uv[i]));
  return t;
}

// unit outward normal of region R at p by central differences of step h
template <bool XF>
__device__ __forceinline__ V3<double> region_normal(JobRef a, int r, V3<double> p, double h) {
  V3<double> n;
  n.x = region_dist<double, XF>(a, r, mk(p.x + h, p.y, p.z)) - region_dist<double, XF>(a, r, mk(p.x - h, p.y, p.z));
  n.y = region_dist<double, XF>(a, r, mk(p.x, p.y + h, p.z)) - region_dist<double, XF>(a, r, mk(p.x, p.y - h, p.z));
  n.z = region_dist<double, XF>(a, r, mk(p.x, p.y, p.z + h)) - region_dist<double, XF>(a, r, mk(p.x, p.y, p.z - h));
  const double inv = 1.0 / __builtin_sqrt(dot(n, n));
  return inv * n;
}

// ------------------------------------------------------------------ tallies

struct LdsTallies {
  double absorbed[kMaxRegions];
  double escaped[6];
  double gain, loss, stalled;
  unsigned long long cnt[16];
};
enum CountSlot {
  kCInterfaces = 0, kCReflections, kCRefractions, kCCrossings, kCAdvances, kCKills, kCStalls, kCEscapes,
  kCLaunched, kCSteps, kCInteractions, kCPieces, kCAtomics
};

// per-lane run of equal voxels waiting to be added to the grid
struct Run {
  int v;
  double sum;
};

// Grid additions of one wave staged in LDS.  Runs end in the middle of
// divergent DDA loops, a few lanes at a time; staging them and draining the
// stage with every lane active issues the FP64 atomics as full 64-lane
// instructions, which keeps the memory-side atomic units fed steadily.
constexpr int kStage = 256;  // entries per wave
constexpr int kDrain = 64;   // entries that trigger a drain in the walk loop
struct WaveStage {
  double val[kStage];
  int v[kStage];
  int n;
};

struct Lane {
  Run run;
  WaveStage* stage; // this wave's staging area (LDS)
  double abs_sum;   // absorbed weight not yet added to the workgroup sums
  int abs_region;
  uint32_t n_steps, n_inter, n_pieces, n_atomics;
  // trace
  smcrt_event* rec;
  int n_rec;
};

__device__ __forceinline__ void grid_add(double* F, int v, double val) {
  __builtin_amdgcn_global_atomic_fadd_f64((SMCRT_G double*)F + v, val);
}

// Stages F[v] += val for the lanes active at the call (any subset of the
// wave); when the stage is full it adds directly.
__device__ __forceinline__ void stage_add(double* F, WaveStage& S, int v, double val) {
  const uint64_t m = __ballot(1);
  const int n = __popcll(m);
  const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  const int base = __builtin_amdgcn_readfirstlane(S.n);
  if (base + n <= kStage) {
    S.v[base + rank] = v;
    S.val[base + rank] = val;
    if (rank == 0) S.n = base + n;
  } else {
    grid_add(F, v, val);
  }
}

// Adds the staged entries to F once at least min_count are waiting.  Called
// with every lane of the wave active.
__device__ __forceinline__ void stage_drain(double* F, WaveStage& S, int min_count, int lane) {
  const int cnt = __builtin_amdgcn_readfirstlane(S.n);
  if (cnt > 0 && cnt >= min_count) {
    for (int i = lane; i < cnt; i += 64) grid_add(F, S.v[i], S.val[i]);
    if (lane == 0) S.n = 0;
  }
}

__device__ __forceinline__ void run_add(double* F, Lane& ln, int v, double val) {
  ++ln.n_pieces;
  if (v == ln.run.v) {
    ln.run.sum += val;
  } else {
    if (ln.run.v >= 0) {
      stage_add(F, *ln.stage, ln.run.v, ln.run.sum);
      ++ln.n_atomics;
    }
    ln.run.v = v;
    ln.run.sum = val;
  }
}

// Index of voxel (x, y, z) in a grid of 2x2x2 bricks ((nx+1)/2 by (ny+1)/2
// by (nz+1)/2 bricks, x fastest), a brick's eight voxels consecutive (x
// fastest inside): the neighbours of a path share 64-byte segments, so more
// of a wave's atomic adds travel in one request.
__device__ __forceinline__ int brick_index(int x, int y, int z, int nx, int ny) {
  const int bx = (nx + 1) >> 1, by = (ny + 1) >> 1;
  const int b = ((z >> 1) * by + (y >> 1)) * bx + (x >> 1);
  return (b << 3) | ((z & 1) << 2) | ((y & 1) << 1) | (x & 1);
}

template <typename T>
__device__ __forceinline__ T trcp(T x);
template <>
__device__ __forceinline__ float trcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double trcp<double>(double x) { return 1.0 / x; }
// 1/sqrt(x): one instruction (1 ulp) in FP32, correctly rounded in FP64
template <typename T>
__device__ __forceinline__ T trsqrt(T x);
template <>
__device__ __forceinline__ float trsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double trsqrt<double>(double x) { return 1.0 / __builtin_sqrt(x); }

// One axis of the voxel walk: voxel index, step (+1, -1 or 0), ray
// parameter of the next plane crossing, and the spacing of the crossings.
template <typename T>
struct DdaAxis {
  int i, s;
  T tn, dt;
};

// Narrows [t0, t1] to the part of the ray g + t*gu inside the slab [0, n]
// of one axis (grid units; r = 1/gu); false when the ray misses the slab.
template <typename T>
__device__ __forceinline__ bool clip_axis(T g, T gu, T r, int n, T& t0, T& t1) {
  if (gu == T(0)) return !(g < T(0) || g > T(n));
  const T ta = -g * r, tb = (T(n) - g) * r;
  t0 = tmax(t0, tmin(ta, tb));
  t1 = tmin(t1, tmax(ta, tb));
  return true;
}

// The voxel of one axis holding the ray at t0 (on a plane while moving down:
// the voxel below), clamped into the grid, and its next crossing.
template <typename T>
__device__ __forceinline__ DdaAxis<T> start_axis(T g, T gu, T r, int n, T t0) {
  DdaAxis<T> A;
  const T x = g + t0 * gu;
  T fl = floor(x);
  if (gu < T(0) && x == fl) fl -= T(1);
  fl = tclamp(fl, T(-1), T(n));
  int k = (int)fl;
  k = k < 0 ? 0 : (k >= n ? n - 1 : k);
  A.i = k;
  A.s = gu > T(0) ? 1 : (gu < T(0) ? -1 : 0);
  A.tn = gu > T(0) ? (T(k + 1) - g) * r : (gu < T(0) ? (T(k) - g) * r : tinf<T>());
  A.dt = gu != T(0) ? tabs(r) : tinf<T>();
  return A;
}

// Path-length estimator (Sec. 3.1): weight * length of the straight move
// p -> p + len*u credited to every voxel it crosses, by a 3-D DDA in voxel
// units.  Voxel i spans [lo + i*D, lo + (i+1)*D); indices are clamped on
// entry and the walk stops when it steps off the grid.  The axes are kept
// in named registers and the linear voxel index is stepped by the axis
// stride, so a crossing costs a few compares and selects.
template <typename T>
__device__ __forceinline__ void tally_move(JobRef a, V3<T> p, V3<T> u, T len, double w, Lane& ln) {
  ScP sc = kptr(a.sc);
  if (a.fluence == nullptr || !(len > T(0))) return;
  const int nx = sc->g_dims[0], ny = sc->g_dims[1], nz = sc->g_dims[2];
  const V3<T> inv = Tab<T>::g_inv(sc);
  const V3<T> lo = Tab<T>::g_lo(sc);
  const T gx = (p.x - lo.x) * inv.x, gy = (p.y - lo.y) * inv.y, gz = (p.z - lo.z) * inv.z;
  const T ux = u.x * inv.x, uy = u.y * inv.y, uz = u.z * inv.z;
  if (!__builtin_isfinite(gx + gy + gz + ux + uy + uz + len)) return;
  const T rx = trcp(ux), ry = trcp(uy), rz = trcp(uz);
  T t0 = T(0), t1 = len;
  if (!clip_axis(gx, ux, rx, nx, t0, t1) || !clip_axis(gy, uy, ry, ny, t0, t1) || !clip_axis(gz, uz, rz, nz, t0, t1))
    return;
  if (!(t1 > t0)) return;
  DdaAxis<T> X = start_axis(gx, ux, rx, nx, t0), Y = start_axis(gy, uy, ry, ny, t0),
             Z = start_axis(gz, uz, rz, nz, t0);
  int lin = X.i + nx * (Y.i + ny * Z.i);
  const int sy = Y.s * nx, sz = Z.s * (nx * ny);
  T t = t0;
  const int cap = nx + ny + nz + 3;
  for (int it = 0; it < cap; ++it) {
    const T tn = tmin(tmin(X.tn, Y.tn), tmin(Z.tn, t1));
    const T piece = tn - t;
    if (piece > T(0)) run_add(a.fluence, ln, a.brick ? brick_index(X.i, Y.i, Z.i, nx, ny) : lin, w * (double)piece);
    if (tn >= t1) break;
    // cross the nearest plane (ties: x before y before z)
    const bool bx = X.tn <= Y.tn && X.tn <= Z.tn;
    const bool by = !bx && Y.tn <= Z.tn;
    const bool bz = !bx && !by;
    X.i += bx ? X.s : 0;
    Y.i += by ? Y.s : 0;
    Z.i += bz ? Z.s : 0;
    X.tn = bx ? X.tn + X.dt : X.tn;
    Y.tn = by ? Y.tn + Y.dt : Y.tn;
    Z.tn = bz ? Z.tn + Z.dt : Z.tn;
    lin += bx ? X.s : (by ? sy : sz);
    if ((unsigned)X.i >= (unsigned)nx || (unsigned)Y.i >= (unsigned)ny || (unsigned)Z.i >= (unsigned)nz) break;
    t = tn;
  }
}

// Unpolarised Fresnel reflectance between indices n1 -> n2 at incidence
// cosine ci (Sec. 1); *ct receives the transmitted cosine.  Total internal
// reflection gives 1 (and *ct = 0).
__device__ __forceinline__ double fresnel(double n1, double n2, double ci, double* ct) {
  const double eta = n1 / n2;
  const double s2t = eta * eta * (1.0 - ci * ci);
  *ct = 0.0;
  if (s2t >= 1.0) return 1.0;
  const double c2 = __builtin_sqrt(1.0 - s2t);
  const double rs = (n1 * ci - n2 * c2) / (n1 * ci + n2 * c2);
  const double rp = (n1 * c2 - n2 * ci) / (n1 * c2 + n2 * ci);
  *ct = c2;
  return 0.5 * (rs * rs + rp * rp);
}

// ------------------------------------------------------------------ packet

enum State : int { kTransport = 0, kSurface = 1, kInteract = 2 };

template <typename T>
struct Packet {
  V3<T> p, u;
  // FP32 only: the part of the position that rounding left out of p
  // (compensated summation of the moves; zero after a jump of position)
  V3<T> pe;
  // remaining optical depth, FP64 in both transport precisions: it is used
  // up over many sphere-tracing steps, and along a grazing path (thousands
  // of steps of delta size) FP32 rounding would let it drift
  double tau;
  T mut, inv_mut;   // of the current region (0 and 0 in ambient)
  double w;
  uint64_t pid;
  uint32_t k;       // event index
  int region;       // n_regions = ambient
  int state;
  int steps;        // sphere-tracing steps in the current event
  T pend;           // straight path along u since the last tally, ending at p
  // previous sphere-tracing step of the current straight segment: surface
  // distance at its start (< 0: none yet) and its length, negated while an
  // over-relaxed step waits for its check at the next evaluation
  T pd, pl;
  // free-flight reuse: radius of a ball about p that holds no surface
  // (< 0: none known) and the interactions taken in it since the distance
  // was evaluated
  T safe;
  int links;
};

constexpr int kReuseLinks = 32;  // interactions per evaluation at most

// A packet still in flight when a resident-serving epoch ends (slot first,
// at the same offset in both precisions, for the host-side kernels that
// sort the records by slot).
template <typename T>
struct SavedPacket {
  int32_t slot;
  int32_t vx[3];
  Packet<T> pk;
};
static_assert(sizeof(SavedPacket<double>) <= kSavedPacketBytes, "saved packet record too large");
static_assert(sizeof(SavedPacket<float>) <= kSavedPacketBytes, "saved packet record too large");

// Writes the live packets of the calling lanes (all lanes of the wave
// active; live lanes save) to the launch's save slab.  The host sizes the
// slab for one packet per lane of every launch of the epoch; a record
// beyond it is counted but not written, and the host fails the epoch.
template <typename T>
__device__ __forceinline__ void save_live(const BatchArgs& B, JobRef a, bool live, const Packet<T>& pk,
                                          const int vx[3], int lane) {
  const uint64_t m = __ballot(live);
  const int n = __popcll(m);
  if (n == 0) return;
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(B.save_count, (unsigned int)n);
  base = __shfl(base, leader);
  if (!live) return;
  const unsigned int i = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
  if (i >= B.save_cap) return;
  SavedPacket<T>* s = reinterpret_cast<SavedPacket<T>*>(static_cast<char*>(B.save) + (size_t)i * kSavedPacketBytes);
  s->slot = a.slot;
  s->vx[0] = vx[0];
  s->vx[1] = vx[1];
  s->vx[2] = vx[2];
  s->pk = pk;
}

// Packet i of job a's resumed packets
template <typename T>
__device__ __forceinline__ void load_saved(JobRef a, unsigned int i, Packet<T>& pk, int vx[3]) {
  const SavedPacket<T>* s =
      reinterpret_cast<const SavedPacket<T>*>(static_cast<const char*>(a.resume) + (size_t)i * kSavedPacketBytes);
  pk = s->pk;
  vx[0] = s->vx[0];
  vx[1] = s->vx[1];
  vx[2] = s->vx[2];
}

template <typename T>
__device__ __forceinline__ void set_region(ScP sc, Packet<T>& pk, int r) {
  pk.region = r;
  pk.mut = Tab<T>::mut(sc->reg[r]);
  pk.inv_mut = Tab<T>::inv_mut(sc->reg[r]);
}

template <typename T, bool TRACE>
__device__ __forceinline__ void record(JobRef a, const Packet<T>& pk, Lane& ln, int type) {
  if constexpr (TRACE) {
    if (ln.n_rec < a.max_records) {
      smcrt_event e;
      e.event = pk.k;
      e.type = (uint32_t)type;
      e.region = pk.region == a.sc->n_regions ? -1 : pk.region;
      e.pad = 0;
      // FP32: the position with its compensation, as the walk carries it
      e.p[0] = (double)pk.p.x + (double)pk.pe.x;
      e.p[1] = (double)pk.p.y + (double)pk.pe.y;
      e.p[2] = (double)pk.p.z + (double)pk.pe.z;
      e.u[0] = pk.u.x; e.u[1] = pk.u.y; e.u[2] = pk.u.z;
      e.w = pk.w;
      e.tau = pk.tau;
      ln.rec[ln.n_rec] = e;
    }
    ++ln.n_rec;
  }
}

// Moves the packet len along u.  The tally is deferred: the straight path
// since the last change of direction collects in pend and is credited to
// the grid in one pass by flush_tally, which runs before the direction
// changes or the position jumps (interactions, interface events) and when
// the packet ends.  Collinear sphere-tracing steps thus share one DDA, and
// the lanes of a wave run it together.
//
// In FP32 the position is a compensated sum (2Sum per axis, exact for any
// magnitudes, also where a move is longer than the coordinate near the
// coordinate planes): pe keeps what rounding dropped from p and is added
// back on the next move.  A
// sphere-tracing step that runs nearly parallel to a face a few surface
// thresholds away moves p across that face by far less than p's ulp; a
// plain sum would drop every one of those moves, the packet would slide
// along the face at a fixed depth in steps of that depth, and a walk of
// 0.5 cm would take some 4e4 steps where the FP64 walk takes 2e3.
// s = fl(a + b) and *e = a + b - s exactly (Knuth's 2Sum; six additions,
// no condition on |a| and |b|)
template <typename T>
__device__ __forceinline__ T two_sum(T a, T b, T* e) {
  const T s = a + b;
  const T bb = s - a;
  *e = (a - (s - bb)) + (b - bb);
  return s;
}

// The packet is put at the FP64 point q: in FP32 as the float nearest q
// plus the float nearest the rest, so a re-placement at an interface keeps
// q to about 2^-48 of its size, as the compensated moves do.
template <typename T>
__device__ __forceinline__ void set_position(Packet<T>& pk, V3<double> q) {
  pk.p = from_d<T>(q);
  if constexpr (sizeof(T) == 4) pk.pe = from_d<T>(q - to_d(pk.p));
  else pk.pe = mk(T(0), T(0), T(0));
}

// The move itself: p (+ pe) += len u, compensated in FP32.
template <typename T>
__device__ __forceinline__ void shift(Packet<T>& pk, T len) {
  if constexpr (sizeof(T) == 4) {
    const V3<T> d = len * pk.u + pk.pe;
    V3<T> e;
    pk.p.x = two_sum(pk.p.x, d.x, &e.x);
    pk.p.y = two_sum(pk.p.y, d.y, &e.y);
    pk.p.z = two_sum(pk.p.z, d.z, &e.z);
    pk.pe = e;
  } else {
    pk.p = pk.p + len * pk.u;
  }
}

template <typename T>
__device__ __forceinline__ void advance(Packet<T>& pk, T len) {
  shift(pk, len);
  pk.pend += len;
}

// Sphere-tracing move of len along u (negative: back along u), charged to
// the pending path and the optical depth.  Returns the charged distance.
template <typename T>
__device__ __forceinline__ T step_along(Packet<T>& pk, T len) {
  advance(pk, len);
  pk.tau -= (double)pk.mut * (double)len;
  return len;
}

template <typename T>
__device__ __forceinline__ void flush_tally(JobRef a, Packet<T>& pk, Lane& ln) {
  if (pk.pend > T(0))
    tally_move<T>(a, pk.p - pk.pend * pk.u, pk.u, pk.pend, pk.w, ln);
  pk.pend = T(0);
}

// Escape image (Sec. 3.2 and Sec. 5: the light at a single plane of
// interest).  A packet leaving through the detector face adds its weight to
// the pixel holding the point where its straight path crosses the face's
// plane: traced back along u from its position when that lies beyond the
// plane and the packet moves outward, else its position.  The axis is a
// template argument: selecting a packet coordinate by a run-time axis lets
// the compiler index the packet in memory, which moves it to scratch.
template <int AX, typename T>
__device__ __forceinline__ void detect_on(JobRef a, ScP sc, V3<T> p, V3<T> u, double w, T sg, T plane) {
  const T pa = AX == 0 ? p.x : (AX == 1 ? p.y : p.z);
  const T ua = AX == 0 ? u.x : (AX == 1 ? u.y : u.z);
  const T over = (pa - plane) * sg, out = ua * sg;
  if (over > T(0) && out > T(0)) p = p - (over / out) * u;
  const T c1 = AX == 0 ? p.y : p.x, c2 = AX == 2 ? p.y : p.z;
  const T x = (c1 - (T)sc->det_lo[0]) / ((T)sc->det_hi[0] - (T)sc->det_lo[0]) * (T)sc->det_dims[0];
  const T y = (c2 - (T)sc->det_lo[1]) / ((T)sc->det_hi[1] - (T)sc->det_lo[1]) * (T)sc->det_dims[1];
  // bounds in floating point, before any conversion (NaN fails too)
  if (!(x >= T(0) && y >= T(0) && x < (T)sc->det_dims[0] && y < (T)sc->det_dims[1])) return;
  const int i = (int)floor(x), j = (int)floor(y);
  grid_add(a.detector, i + sc->det_dims[0] * j, w);
}

template <typename T>
__device__ __forceinline__ void detect(JobRef a, const Packet<T>& pk, int face, T plane) {
  if (a.detector == nullptr) return;
  ScP sc = kptr(a.sc);
  if (face != sc->det_face) return;
  const T sg = (face & 1) ? T(1) : T(-1);
  switch (face >> 1) {
    case 0: detect_on<0>(a, sc, pk.p, pk.u, pk.w, sg, plane); break;
    case 1: detect_on<1>(a, sc, pk.p, pk.u, pk.w, sg, plane); break;
    default: detect_on<2>(a, sc, pk.p, pk.u, pk.w, sg, plane); break;
  }
}

__device__ __forceinline__ void add_absorbed(LdsTallies& L, Lane& ln, int r, double dA) {
  if (r != ln.abs_region) {
    if (ln.abs_region >= 0) atomicAdd(&L.absorbed[ln.abs_region], ln.abs_sum);
    ln.abs_region = r;
    ln.abs_sum = 0.0;
  }
  ln.abs_sum += dA;
}

// emission, event 0 (Sec. 3.1 sources; Eq. 1)
template <typename T, bool TRACE, bool XF>
__device__ void emit(JobRef a, Packet<T>& pk, Lane& ln, LdsTallies& L) {
  ScP sc = kptr(a.sc);
  const U4 r = philox10(0u, (uint32_t)pk.pid, (uint32_t)(pk.pid >> 32), 0u, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
  const T x0 = xi_of<T>(r.w0), x1 = xi_of<T>(r.w1), x3 = xi_of<T>(r.w3);
  const SMCRT_K double* s = sc->src;
  // the emission point in FP64 (the source's place plus the sampled offset)
  V3<double> p = mk(s[0], s[1], s[2]);
  V3<T> u;
  const int kind = sc->src_kind;
  if (kind == kPoint) {
    const T ct = T(2) * x0 - T(1);
    const T st = T(2) * tsqrt(x0 * (T(1) - x0));  // sqrt(1 - ct^2) without cancellation
    T sp, cp;
    tsincos_2pi(x1, &sp, &cp);
    u = mk(st * cp, st * sp, ct);
  } else if (kind == kPencil) {
    u = mk((T)s[3], (T)s[4], (T)s[5]);
  } else if (kind == kDisc) {
    const T rr = (T)s[3] * tsqrt(x0);
    T sp, cp;
    tsincos_2pi(x1, &sp, &cp);
    p = mk(p.x + (double)(rr * cp), p.y + (double)(rr * sp), p.z);
    u = mk((T)s[4], (T)s[5], (T)s[6]);
  } else {
    p = mk(p.x + s[3] * (2.0 * (double)x0 - 1.0), p.y + s[4] * (2.0 * (double)x1 - 1.0), p.z);
    u = mk((T)s[5], (T)s[6], (T)s[7]);
  }
  const T il = T(1) / tsqrt(dot(u, u));
  set_position(pk, p);
  pk.u = il * u;
  pk.w = 1.0;
  pk.tau = (double)(-tlog(x3));
  pk.k = 0;
  pk.steps = 0;
  pk.pd = T(-1);
  pk.pl = T(0);
  pk.safe = T(-1);
  pk.links = 0;
  pk.pend = T(0);
  pk.state = kTransport;
  set_region(sc, pk, region_of<T, XF>(a, pk.p));
  atomicAdd(&L.cnt[kCLaunched], 1ull);
  record<T, TRACE>(a, pk, ln, SMCRT_EV_EMIT);
}

// absorption, Henyey-Greenstein scattering, roulette, next free path.
// Returns false when the packet ends.
template <typename T, bool TRACE>
__device__ bool interact(JobRef a, Packet<T>& pk, Lane& ln, LdsTallies& L) {
  ScP sc = kptr(a.sc);
  RegRef R = sc->reg[pk.region];
  pk.k += 1;
  ++ln.n_inter;
  const U4 r = philox10(pk.k, (uint32_t)pk.pid, (uint32_t)(pk.pid >> 32), 0u, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
  // implicit capture: the fraction mu_a/mu_t of the weight stays here
  const double dA = pk.w * R.mua / R.mut;
  add_absorbed(L, ln, pk.region, dA);
  pk.w -= dA;
  if (pk.w == 0.0) {
    record<T, TRACE>(a, pk, ln, SMCRT_EV_ABSORB);
    return false;
  }
  // scattering angle from the HG inverse CDF; azimuth uniform.  The CDF is
  // inverted for 1 - cos(theta) directly,
  //   1 - cos = (1 - g)(1 - xi)(f + 1 - g) / D,  D = 1 - g + 2 g xi,
  //   f = (1 - g^2) / D,
  // which has no cancellation near forward scattering, so FP32 keeps
  // sin(theta) = sqrt((1 - cos)(1 + cos)) to full relative precision.
  const T x0 = xi_of<T>(r.w0), x1 = xi_of<T>(r.w1);
  T omc;
  if (R.iso) {
    omc = T(2) * (T(1) - x0);
  } else if constexpr (sizeof(T) == 4) {
    const float D = R.hg_cf + R.hg_df * x0;
    const float f = tdiv(R.hg_bf, D);
    omc = tdiv(R.hg_cf * (1.0f - x0) * (f + R.hg_cf), D);
  } else {
    const double D = R.hg_c + R.hg_d * x0;
    const double f = R.hg_b / D;
    omc = R.hg_c * (1.0 - x0) * (f + R.hg_c) / D;
  }
  omc = tclamp(omc, T(0), T(2));
  const T ct = T(1) - omc;
  const T st = tsqrt(omc * (T(2) - omc));
  T sp, cp;
  tsincos_2pi(x1, &sp, &cp);
  const V3<T> u = pk.u;
  V3<T> v;
  if (tabs(u.z) > T(1) - T(1e-5)) {
    v = mk(st * cp, st * sp, (u.z >= T(0) ? ct : -ct));
  } else {
    // sqrt(1 - uz^2) from the other two components: no cancellation near the poles
    const T tt = tsqrt(u.x * u.x + u.y * u.y);
    const T itt = trcp(tt);
    v.x = st * (u.x * u.z * cp - u.y * sp) * itt + u.x * ct;
    v.y = st * (u.y * u.z * cp + u.x * sp) * itt + u.y * ct;
    v.z = -st * cp * tt + u.z * ct;
  }
  pk.u = trsqrt(dot(v, v)) * v;
  // Russian roulette on the weight
  if (pk.w < sc->w_threshold) {
    const double x2 = xi_of<double>(r.w2);
    if (x2 < sc->inv_m) {
      atomicAdd(&L.gain, (sc->m_d - 1.0) * pk.w);
      pk.w *= sc->m_d;
    } else {
      atomicAdd(&L.loss, pk.w);
      atomicAdd(&L.cnt[kCKills], 1ull);
      record<T, TRACE>(a, pk, ln, SMCRT_EV_KILL);
      return false;
    }
  }
  pk.tau = (double)(-tlog(xi_of<T>(r.w3)));
  pk.steps = 0;
  pk.pd = T(-1);
  record<T, TRACE>(a, pk, ln, SMCRT_EV_SCATTER);
  return true;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// First job of the launch's geometry, scanning from `start`, whose packet
// counter has not reached its packet count; -1 when every such job is handed
// out.  Wave uniform.
__device__ __forceinline__ int pick_job(const SMCRT_K WalkArgs* jobs, const BatchArgs& B, int start) {
  for (int i = 0; i < B.n_jobs; ++i) {
    const int j = (start + i) % B.n_jobs;
    JobRef J = jobs[j];
    if (J.geometry != B.geometry) continue;
    const unsigned long long c = __hip_atomic_load(J.counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t cu = ((uint64_t)__builtin_amdgcn_readfirstlane((unsigned)(c >> 32)) << 32) |
                        (uint64_t)__builtin_amdgcn_readfirstlane((unsigned)c);
    if (cu < J.n) return j;
    if (J.resume_n > 0) {  // packets of an earlier epoch left to resume
      const unsigned int r = __hip_atomic_load(J.resume_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__builtin_amdgcn_readfirstlane(r) < J.resume_n) return j;
    }
  }
  return -1;
}

// Copies job a's FP32 capsule records into the workgroup's LDS table (two
// float4 per capsule); false, with nothing copied, when the job has none or
// more than the table holds.  Called by every thread of the workgroup; the
// caller's barrier makes the table visible.
__device__ __forceinline__ bool stage_caps(JobRef a, F4* dst) {
  const SMCRT_K Accel& A = kptr(a.sc)->acc;
  if (A.region < 0 || !A.caps || A.n_prims > kStageCaps || a.acc_capf == nullptr) return false;
  const F4* src = reinterpret_cast<const F4*>(a.acc_capf);
  const int n = 2 * A.n_prims;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  return true;
}

// Adds a wave's pending sums to job a's outputs and clears them.  Called with
// every lane of the wave active.
__device__ __forceinline__ void flush_wave(JobRef a, Lane& ln, LdsTallies& L, int lane) {
  if (a.fluence != nullptr) stage_drain(a.fluence, *ln.stage, 1, lane);
  if (ln.run.v >= 0) {
    grid_add(a.fluence, ln.run.v, ln.run.sum);
    ++ln.n_atomics;
  }
  if (ln.abs_region >= 0) atomicAdd(&L.absorbed[ln.abs_region], ln.abs_sum);
  atomicAdd(&L.cnt[kCSteps], (unsigned long long)ln.n_steps);
  atomicAdd(&L.cnt[kCInteractions], (unsigned long long)ln.n_inter);
  atomicAdd(&L.cnt[kCPieces], (unsigned long long)ln.n_pieces);
  atomicAdd(&L.cnt[kCAtomics], (unsigned long long)ln.n_atomics);
  ln.run.v = -1;
  ln.run.sum = 0.0;
  ln.abs_region = -1;
  ln.abs_sum = 0.0;
  ln.n_steps = ln.n_inter = ln.n_pieces = ln.n_atomics = 0;
  __threadfence_block();
  if (lane == 0) {
    const int nr = a.sc->n_regions;
    if (a.absorbed != nullptr)
      for (int r = 0; r < nr; ++r) unsafeAtomicAdd(a.absorbed + r, L.absorbed[r]);
    smcrt_tallies* G = reinterpret_cast<smcrt_tallies*>(a.tallies);
    if (G != nullptr) {
      for (int f = 0; f < 6; ++f) unsafeAtomicAdd(&G->escaped_face[f], L.escaped[f]);
      unsafeAtomicAdd(&G->launched, (double)L.cnt[kCLaunched]);
      unsafeAtomicAdd(&G->roulette_gain, L.gain);
      unsafeAtomicAdd(&G->roulette_loss, L.loss);
      unsafeAtomicAdd(&G->stalled, L.stalled);
      atomicAdd((unsigned long long*)&G->events, L.cnt[kCInteractions] + L.cnt[kCInterfaces]);
      atomicAdd((unsigned long long*)&G->steps, L.cnt[kCSteps]);
      atomicAdd((unsigned long long*)&G->interactions, L.cnt[kCInteractions]);
      atomicAdd((unsigned long long*)&G->interfaces, L.cnt[kCInterfaces]);
      atomicAdd((unsigned long long*)&G->reflections, L.cnt[kCReflections]);
      atomicAdd((unsigned long long*)&G->refractions, L.cnt[kCRefractions]);
      atomicAdd((unsigned long long*)&G->crossings, L.cnt[kCCrossings]);
      atomicAdd((unsigned long long*)&G->advances, L.cnt[kCAdvances]);
      atomicAdd((unsigned long long*)&G->voxel_pieces, L.cnt[kCPieces]);
      atomicAdd((unsigned long long*)&G->kills, L.cnt[kCKills]);
      atomicAdd((unsigned long long*)&G->stalls, L.cnt[kCStalls]);
      atomicAdd((unsigned long long*)&G->escapes, L.cnt[kCEscapes]);
      atomicAdd((unsigned long long*)&G->grid_atomics, L.cnt[kCAtomics]);
    }
    for (int r = 0; r < kMaxRegions; ++r) L.absorbed[r] = 0.0;
    for (int f = 0; f < 6; ++f) L.escaped[f] = 0.0;
    for (int c = 0; c < 16; ++c) L.cnt[c] = 0ull;
    L.gain = L.loss = L.stalled = 0.0;
  }
  __threadfence_block();
}

}  // namespace smcrt
