// api.cpp -- host side of libsmcrt: scene building and validation, packing of
// the device tables, engines, and the C entry points declared in smcrt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/smcrt.h"
#include "launch.h"
#include "layout.h"

using namespace smcrt;

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

static smcrt_status fail(smcrt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

static smcrt_status hip_fail(hipError_t e, const char* what) {
  return fail(SMCRT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                  \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

extern "C" const char* smcrt_last_error(void) { return g_last_error.c_str(); }
extern "C" int smcrt_abi_version(void) { return SMCRT_ABI_VERSION; }

// ------------------------------------------------------------------ scenes

struct HostPrim {
  int kind;
  double p[8];
  // placement x = s R x_local + t, rounding, onion shell, twist (local frame)
  bool placed = false;
  double rot[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double t[3] = {0, 0, 0}, s = 1.0;
  double round_r = 0.0, onion_t = 0.0, twist_k = 0.0;
  double bend_k = 0.0;  // turn by bend_k * x about the local z axis (exclusive with twist_k)
  double elong[3] = {0, 0, 0};
  double disp_a = 0.0, disp_f = 0.0;
  double rep_c[3] = {1, 1, 1};
  int32_t rep_n[3] = {1, 1, 1};
};
static bool repeated(const HostPrim& p);
static double repetition_gap(const HostPrim& p);

struct HostRegion {
  std::vector<int32_t> prims;
  int op;
  double k, mua, mus, g, n;
};

struct smcrt_scene {
  double n_ambient = 1.0, delta = 1e-5, pad = 1e-4;
  double relax = 1.0;  // over-relaxation factor of sphere-tracing steps
  bool segment = false;  // segment-traced steps
  std::vector<HostPrim> prims;
  std::vector<HostRegion> regions;
  bool has_source = false;
  int src_kind = 0;
  double src[8] = {0};
  bool grid_set = false;
  double g_lo[3] = {0}, g_hi[3] = {0};
  int32_t g_dims[3] = {1, 1, 1};
  double w_threshold = 1e-4;
  int32_t m_survive = 10;
  int32_t max_steps = 100000;
  int64_t max_events = 1000000;
  int32_t accel_region = -1;
  int32_t accel_cells[3] = {0, 0, 0};
  int32_t geometry = kGeomSdf;
  int32_t det_face = -1;
  int32_t det_dims[2] = {0, 0};
  double det_lo[2] = {0, 0}, det_hi[2] = {0, 0};
  // packed device tables (rebuilt when dirty)
  bool dirty = true;
  std::vector<unsigned char> blob;
};

static bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

extern "C" smcrt_status smcrt_scene_create(smcrt_scene** out, double n_ambient, double delta, double pad) {
  if (!out) return fail(SMCRT_E_INVALID, "scene_create: out is NULL");
  if (!(n_ambient > 0) || !std::isfinite(n_ambient)) return fail(SMCRT_E_INVALID, "scene_create: n_ambient must be > 0");
  if (!(delta > 0) || !std::isfinite(delta)) return fail(SMCRT_E_INVALID, "scene_create: delta must be > 0");
  if (!(pad >= 0) || !std::isfinite(pad)) return fail(SMCRT_E_INVALID, "scene_create: pad must be >= 0");
  smcrt_scene* s = new (std::nothrow) smcrt_scene();
  if (!s) return fail(SMCRT_E_NOMEM, "scene_create: out of host memory");
  s->n_ambient = n_ambient;
  s->delta = delta;
  s->pad = pad;
  *out = s;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_destroy(smcrt_scene* s) {
  delete s;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_add_primitive(smcrt_scene* s, int kind, const double* params, int n_params,
                                                  int32_t* out_prim) {
  if (!s || !params) return fail(SMCRT_E_INVALID, "add_primitive: NULL argument");
  static const int need[9] = {4, 6, 7, 7, 8, 8, 4, 5, 6};
  if (kind < 0 || kind > 8) return fail(SMCRT_E_INVALID, "add_primitive: unknown kind %d", kind);
  if (n_params != need[kind]) return fail(SMCRT_E_INVALID, "add_primitive: kind %d takes %d params, got %d", kind, need[kind], n_params);
  for (int i = 0; i < n_params; ++i)
    if (!std::isfinite(params[i])) return fail(SMCRT_E_INVALID, "add_primitive: param %d is not finite", i);
  if ((int)s->prims.size() >= kMaxPrims) return fail(SMCRT_E_INVALID, "add_primitive: more than %d primitives", kMaxPrims);
  HostPrim p;
  p.kind = kind;
  std::memset(p.p, 0, sizeof(p.p));
  std::memcpy(p.p, params, sizeof(double) * n_params);
  if (kind == kSphere && !(p.p[3] > 0)) return fail(SMCRT_E_INVALID, "add_primitive: sphere radius must be > 0");
  if (kind == kBox && !(p.p[3] > 0 && p.p[4] > 0 && p.p[5] > 0))
    return fail(SMCRT_E_INVALID, "add_primitive: box half extents must be > 0");
  if (kind == kCapsule || kind == kCylinder) {
    double d[3] = {p.p[3] - p.p[0], p.p[4] - p.p[1], p.p[5] - p.p[2]};
    if (!(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > 0)) return fail(SMCRT_E_INVALID, "add_primitive: segment ends must differ");
    if (!(p.p[6] > 0)) return fail(SMCRT_E_INVALID, "add_primitive: radius must be > 0");
  }
  if (kind == kCone) {
    double d[3] = {p.p[3] - p.p[0], p.p[4] - p.p[1], p.p[5] - p.p[2]};
    if (!(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > 0)) return fail(SMCRT_E_INVALID, "add_primitive: cone ends must differ");
    if (!(p.p[6] >= 0 && p.p[7] >= 0 && p.p[6] + p.p[7] > 0))
      return fail(SMCRT_E_INVALID, "add_primitive: cone radii must be >= 0, not both 0");
  }
  if (kind == kOctahedron && !(p.p[3] > 0)) return fail(SMCRT_E_INVALID, "add_primitive: octahedron size must be > 0");
  if (kind == kHexPrism && !(p.p[3] > 0 && p.p[4] > 0))
    return fail(SMCRT_E_INVALID, "add_primitive: hexagonal prism apothem and half height must be > 0");
  if (kind == kEllipsoid && !(p.p[3] > 0 && p.p[4] > 0 && p.p[5] > 0))
    return fail(SMCRT_E_INVALID, "add_primitive: ellipsoid radii must be > 0");
  if (kind == kTorus) {
    if (!(p.p[3] * p.p[3] + p.p[4] * p.p[4] + p.p[5] * p.p[5] > 0)) return fail(SMCRT_E_INVALID, "add_primitive: torus axis must be non-zero");
    if (!(p.p[6] >= 0 && p.p[7] > 0)) return fail(SMCRT_E_INVALID, "add_primitive: torus needs R >= 0 and tube radius r > 0");
  }
  s->prims.push_back(p);
  s->dirty = true;
  if (out_prim) *out_prim = (int32_t)s->prims.size() - 1;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_add_region(smcrt_scene* s, const int32_t* prims, int n_prims, int op, double k_cm,
                                               double mu_a, double mu_s, double g, double n, int32_t* out_region) {
  if (!s || !prims) return fail(SMCRT_E_INVALID, "add_region: NULL argument");
  if ((int)s->regions.size() >= kMaxRegions) return fail(SMCRT_E_INVALID, "add_region: at most %d regions", kMaxRegions);
  if (n_prims < 1) return fail(SMCRT_E_INVALID, "add_region: needs at least one primitive");
  for (int i = 0; i < n_prims; ++i)
    if (prims[i] < 0 || prims[i] >= (int32_t)s->prims.size())
      return fail(SMCRT_E_INVALID, "add_region: primitive index %d out of range", prims[i]);
  if (op < SMCRT_OP_UNION || op > SMCRT_OP_SUBTRACT) return fail(SMCRT_E_INVALID, "add_region: unknown op %d", op);
  if (op == SMCRT_OP_SMOOTH_UNION && !(k_cm > 0 && std::isfinite(k_cm)))
    return fail(SMCRT_E_INVALID, "add_region: smooth union needs k > 0");
  if (!(mu_a >= 0 && std::isfinite(mu_a)) || !(mu_s >= 0 && std::isfinite(mu_s)) || !(mu_a + mu_s > 0))
    return fail(SMCRT_E_INVALID, "add_region: need mu_a >= 0, mu_s >= 0, mu_a + mu_s > 0");
  if (!(g > -1 && g < 1)) return fail(SMCRT_E_INVALID, "add_region: need -1 < g < 1");
  if (!(n > 0 && std::isfinite(n))) return fail(SMCRT_E_INVALID, "add_region: need n > 0");
  HostRegion r;
  r.prims.assign(prims, prims + n_prims);
  r.op = op;
  r.k = op == SMCRT_OP_SMOOTH_UNION ? k_cm : 0.0;
  r.mua = mu_a;
  r.mus = mu_s;
  r.g = g;
  r.n = n;
  s->regions.push_back(r);
  s->dirty = true;
  if (out_region) *out_region = (int32_t)s->regions.size() - 1;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_source(smcrt_scene* s, int kind, const double* params, int n_params) {
  if (!s || !params) return fail(SMCRT_E_INVALID, "set_source: NULL argument");
  static const int need[4] = {3, 6, 7, 8};
  if (kind < 0 || kind > 3) return fail(SMCRT_E_INVALID, "set_source: unknown kind %d", kind);
  if (n_params != need[kind]) return fail(SMCRT_E_INVALID, "set_source: kind %d takes %d params, got %d", kind, need[kind], n_params);
  for (int i = 0; i < n_params; ++i)
    if (!std::isfinite(params[i])) return fail(SMCRT_E_INVALID, "set_source: param %d is not finite", i);
  double v[8] = {0};
  std::memcpy(v, params, sizeof(double) * n_params);
  int du = kind == kPencil ? 3 : kind == kDisc ? 4 : kind == kRect ? 5 : -1;
  if (kind == kDisc && !(v[3] > 0)) return fail(SMCRT_E_INVALID, "set_source: disc radius must be > 0");
  if (kind == kRect && !(v[3] > 0 && v[4] > 0)) return fail(SMCRT_E_INVALID, "set_source: rectangle half sides must be > 0");
  if (du >= 0) {
    double l = std::sqrt(v[du] * v[du] + v[du + 1] * v[du + 1] + v[du + 2] * v[du + 2]);
    if (!(l > 0)) return fail(SMCRT_E_INVALID, "set_source: direction must be non-zero");
    for (int i = 0; i < 3; ++i) v[du + i] /= l;
  }
  s->src_kind = kind;
  std::memcpy(s->src, v, sizeof(v));
  s->has_source = true;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_grid(smcrt_scene* s, const double lo[3], const double hi[3], const int32_t dims[3]) {
  if (!s || !lo || !hi || !dims) return fail(SMCRT_E_INVALID, "set_grid: NULL argument");
  if (!finite3(lo) || !finite3(hi)) return fail(SMCRT_E_INVALID, "set_grid: bounds must be finite");
  for (int i = 0; i < 3; ++i) {
    if (!(hi[i] > lo[i])) return fail(SMCRT_E_INVALID, "set_grid: need lo < hi on every axis");
    if (dims[i] < 0 || dims[i] > 4096) return fail(SMCRT_E_INVALID, "set_grid: dims must be in [0, 4096]");
  }
  if ((double)dims[0] * dims[1] * dims[2] > 2147483647.0) return fail(SMCRT_E_INVALID, "set_grid: more than 2^31-1 voxels");
  std::memcpy(s->g_lo, lo, sizeof(s->g_lo));
  std::memcpy(s->g_hi, hi, sizeof(s->g_hi));
  std::memcpy(s->g_dims, dims, sizeof(s->g_dims));
  s->grid_set = true;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_roulette(smcrt_scene* s, double w_threshold, int32_t m_survive) {
  if (!s) return fail(SMCRT_E_INVALID, "set_roulette: NULL scene");
  if (!(w_threshold >= 0 && w_threshold < 1)) return fail(SMCRT_E_INVALID, "set_roulette: need 0 <= w_threshold < 1");
  if (m_survive < 1) return fail(SMCRT_E_INVALID, "set_roulette: need m_survive >= 1");
  s->w_threshold = w_threshold;
  s->m_survive = m_survive;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_limits(smcrt_scene* s, int32_t max_steps, int64_t max_events) {
  if (!s) return fail(SMCRT_E_INVALID, "set_limits: NULL scene");
  if (max_steps < 1 || max_events < 1) return fail(SMCRT_E_INVALID, "set_limits: limits must be >= 1");
  if (max_events > 0xFFFFFFF0LL) return fail(SMCRT_E_INVALID, "set_limits: max_events must fit the 32-bit event counter");
  s->max_steps = max_steps;
  s->max_events = max_events;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_primitive_placement(smcrt_scene* s, int32_t prim, const double rot[9],
                                                            double scale, const double trans[3]) {
  if (!s || !rot || !trans) return fail(SMCRT_E_INVALID, "set_primitive_placement: NULL argument");
  if (prim < 0 || prim >= (int32_t)s->prims.size()) return fail(SMCRT_E_INVALID, "set_primitive_placement: no primitive %d", prim);
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(rot[i])) return fail(SMCRT_E_INVALID, "set_primitive_placement: rotation not finite");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(trans[i])) return fail(SMCRT_E_INVALID, "set_primitive_placement: translation not finite");
  if (!(scale > 0.0 && std::isfinite(scale))) return fail(SMCRT_E_INVALID, "set_primitive_placement: scale must be > 0");
  for (int i = 0; i < 3; ++i)  // rows orthonormal
    for (int j = 0; j < 3; ++j) {
      const double d = rot[3 * i] * rot[3 * j] + rot[3 * i + 1] * rot[3 * j + 1] + rot[3 * i + 2] * rot[3 * j + 2];
      if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-9)
        return fail(SMCRT_E_INVALID, "set_primitive_placement: rotation must be orthonormal (to 1e-9)");
    }
  const double det = rot[0] * (rot[4] * rot[8] - rot[5] * rot[7]) - rot[1] * (rot[3] * rot[8] - rot[5] * rot[6]) +
                     rot[2] * (rot[3] * rot[7] - rot[4] * rot[6]);
  if (!(det > 0.0)) return fail(SMCRT_E_INVALID, "set_primitive_placement: rotation must have determinant +1");
  HostPrim& p = s->prims[prim];
  p.placed = true;
  std::memcpy(p.rot, rot, sizeof(p.rot));
  std::memcpy(p.t, trans, sizeof(p.t));
  p.s = scale;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_primitive_modifiers(smcrt_scene* s, int32_t prim, double round_r, double onion_t,
                                                            double twist_k) {
  if (!s) return fail(SMCRT_E_INVALID, "set_primitive_modifiers: NULL scene");
  if (prim < 0 || prim >= (int32_t)s->prims.size()) return fail(SMCRT_E_INVALID, "set_primitive_modifiers: no primitive %d", prim);
  if (!(round_r >= 0.0 && std::isfinite(round_r)) || !(onion_t >= 0.0 && std::isfinite(onion_t)))
    return fail(SMCRT_E_INVALID, "set_primitive_modifiers: rounding and shell must be finite and >= 0");
  if (!std::isfinite(twist_k)) return fail(SMCRT_E_INVALID, "set_primitive_modifiers: twist must be finite");
  if (twist_k != 0.0 && s->prims[prim].bend_k != 0.0)
    return fail(SMCRT_E_INVALID, "set_primitive_modifiers: primitive %d is bent; a primitive is either twisted or bent", prim);
  HostPrim& p = s->prims[prim];
  p.round_r = round_r;
  p.onion_t = onion_t;
  p.twist_k = twist_k;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_primitive_bend(smcrt_scene* s, int32_t prim, double bend_k) {
  if (!s) return fail(SMCRT_E_INVALID, "set_primitive_bend: NULL scene");
  if (prim < 0 || prim >= (int32_t)s->prims.size()) return fail(SMCRT_E_INVALID, "set_primitive_bend: no primitive %d", prim);
  if (!std::isfinite(bend_k)) return fail(SMCRT_E_INVALID, "set_primitive_bend: bend must be finite");
  if (bend_k != 0.0 && s->prims[prim].twist_k != 0.0)
    return fail(SMCRT_E_INVALID, "set_primitive_bend: primitive %d is twisted; a primitive is either twisted or bent", prim);
  s->prims[prim].bend_k = bend_k;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_primitive_elongation(smcrt_scene* s, int32_t prim, const double h[3]) {
  if (!s || !h) return fail(SMCRT_E_INVALID, "set_primitive_elongation: NULL argument");
  if (prim < 0 || prim >= (int32_t)s->prims.size()) return fail(SMCRT_E_INVALID, "set_primitive_elongation: no primitive %d", prim);
  for (int i = 0; i < 3; ++i)
    if (!(h[i] >= 0.0 && std::isfinite(h[i]))) return fail(SMCRT_E_INVALID, "set_primitive_elongation: h must be finite and >= 0");
  std::memcpy(s->prims[prim].elong, h, sizeof(double) * 3);
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_primitive_displacement(smcrt_scene* s, int32_t prim, double amplitude, double frequency) {
  if (!s) return fail(SMCRT_E_INVALID, "set_primitive_displacement: NULL scene");
  if (prim < 0 || prim >= (int32_t)s->prims.size()) return fail(SMCRT_E_INVALID, "set_primitive_displacement: no primitive %d", prim);
  if (!(amplitude >= 0.0 && std::isfinite(amplitude)) || !(frequency >= 0.0 && std::isfinite(frequency)))
    return fail(SMCRT_E_INVALID, "set_primitive_displacement: amplitude and frequency must be finite and >= 0");
  s->prims[prim].disp_a = amplitude;
  s->prims[prim].disp_f = frequency;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_primitive_repetition(smcrt_scene* s, int32_t prim, const double spacing[3],
                                                             const int32_t counts[3]) {
  if (!s || !spacing || !counts) return fail(SMCRT_E_INVALID, "set_primitive_repetition: NULL argument");
  if (prim < 0 || prim >= (int32_t)s->prims.size()) return fail(SMCRT_E_INVALID, "set_primitive_repetition: no primitive %d", prim);
  for (int i = 0; i < 3; ++i) {
    if (counts[i] < 1 || counts[i] > 4096) return fail(SMCRT_E_INVALID, "set_primitive_repetition: counts must be in [1, 4096]");
    if (!(spacing[i] > 0.0 && std::isfinite(spacing[i]))) return fail(SMCRT_E_INVALID, "set_primitive_repetition: spacing must be > 0");
  }
  HostPrim p = s->prims[prim];
  std::memcpy(p.rep_c, spacing, sizeof(double) * 3);
  std::memcpy(p.rep_n, counts, sizeof(int32_t) * 3);
  if (repeated(p) && !(repetition_gap(p) > 0.0))
    return fail(SMCRT_E_INVALID, "set_primitive_repetition: copies must fit their cells (set the other modifiers first)");
  s->prims[prim] = p;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_relaxation(smcrt_scene* s, double omega) {
  if (!s) return fail(SMCRT_E_INVALID, "set_relaxation: NULL scene");
  if (!(omega >= 1.0 && omega < 2.0)) return fail(SMCRT_E_INVALID, "set_relaxation: omega must be in [1, 2)");
  if (omega > 1.0 && s->segment)
    return fail(SMCRT_E_INVALID, "set_relaxation: the scene takes segment-traced steps; relaxed steps exclude them");
  s->relax = omega;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_segment_tracing(smcrt_scene* s, int32_t on) {
  if (!s) return fail(SMCRT_E_INVALID, "set_segment_tracing: NULL scene");
  if (on != 0 && on != 1) return fail(SMCRT_E_INVALID, "set_segment_tracing: on must be 0 or 1");
  if (on && s->relax > 1.0)
    return fail(SMCRT_E_INVALID, "set_segment_tracing: the scene takes relaxed steps; segment-traced steps exclude them");
  s->segment = on != 0;
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_accel(smcrt_scene* s, int32_t region, const int32_t cells[3]) {
  if (!s) return fail(SMCRT_E_INVALID, "set_accel: NULL scene");
  if (region < 0) {
    s->accel_region = -1;
    s->dirty = true;
    return SMCRT_OK;
  }
  if (!cells) return fail(SMCRT_E_INVALID, "set_accel: NULL cells");
  if (region >= (int32_t)s->regions.size()) return fail(SMCRT_E_INVALID, "set_accel: region %d does not exist", region);
  if (s->regions[region].op != SMCRT_OP_UNION) return fail(SMCRT_E_INVALID, "set_accel: only union regions can be accelerated");
  for (int i = 0; i < 3; ++i)
    if (cells[i] < 1 || cells[i] > 256) return fail(SMCRT_E_INVALID, "set_accel: cells must be in [1, 256] per axis");
  s->accel_region = region;
  std::memcpy(s->accel_cells, cells, sizeof(s->accel_cells));
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_detector(smcrt_scene* s, int face, const double lo[2], const double hi[2],
                                                 const int32_t dims[2]) {
  if (!s || !lo || !hi || !dims) return fail(SMCRT_E_INVALID, "set_detector: NULL argument");
  if (dims[0] < 0 || dims[1] < 0) return fail(SMCRT_E_INVALID, "set_detector: negative dims");
  if (dims[0] == 0 || dims[1] == 0) {
    s->det_face = -1;
    s->dirty = true;
    return SMCRT_OK;
  }
  if (face < 0 || face > 5) return fail(SMCRT_E_INVALID, "set_detector: face %d outside 0..5", face);
  if ((double)dims[0] * dims[1] > 2147483647.0) return fail(SMCRT_E_INVALID, "set_detector: more than 2^31-1 pixels");
  for (int i = 0; i < 2; ++i)
    if (!(std::isfinite(lo[i]) && std::isfinite(hi[i]) && lo[i] < hi[i]))
      return fail(SMCRT_E_INVALID, "set_detector: need finite lo < hi");
  s->det_face = face;
  for (int i = 0; i < 2; ++i) {
    s->det_dims[i] = dims[i];
    s->det_lo[i] = lo[i];
    s->det_hi[i] = hi[i];
  }
  s->dirty = true;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_set_geometry(smcrt_scene* s, int mode) {
  if (!s) return fail(SMCRT_E_INVALID, "set_geometry: NULL scene");
  if (mode != SMCRT_GEOM_SDF && mode != SMCRT_GEOM_VOXEL) return fail(SMCRT_E_INVALID, "set_geometry: unknown mode %d", mode);
  s->geometry = mode == SMCRT_GEOM_VOXEL ? kGeomVoxel : kGeomSdf;
  s->dirty = true;
  return SMCRT_OK;
}

// conservative box of a primitive's shape in its own frame
static void local_box(const HostPrim& p, double lo[3], double hi[3]) {
  for (int i = 0; i < 3; ++i) {
    switch (p.kind) {
      case kSphere: lo[i] = p.p[i] - p.p[3]; hi[i] = p.p[i] + p.p[3]; break;
      case kBox: lo[i] = p.p[i] - p.p[3 + i]; hi[i] = p.p[i] + p.p[3 + i]; break;
      case kTorus: {  // the ring's box grown by the tube radius
        const double al = std::sqrt(p.p[3] * p.p[3] + p.p[4] * p.p[4] + p.p[5] * p.p[5]);
        const double e = p.p[3 + i] / al;
        const double ext = p.p[6] * std::sqrt(std::max(1.0 - e * e, 0.0)) + p.p[7];
        lo[i] = p.p[i] - ext;
        hi[i] = p.p[i] + ext;
        break;
      }
      case kCone: {  // the end points' box grown by the larger radius
        const double r = std::max(p.p[6], p.p[7]);
        lo[i] = std::min(p.p[i], p.p[3 + i]) - r;
        hi[i] = std::max(p.p[i], p.p[3 + i]) + r;
        break;
      }
      case kOctahedron: lo[i] = p.p[i] - p.p[3]; hi[i] = p.p[i] + p.p[3]; break;
      case kHexPrism: {  // circumradius 2h/sqrt(3) in x, apothem h in y
        const double e = i == 0 ? 2.0 * p.p[3] / std::sqrt(3.0) : (i == 1 ? p.p[3] : p.p[4]);
        lo[i] = p.p[i] - e;
        hi[i] = p.p[i] + e;
        break;
      }
      case kEllipsoid: lo[i] = p.p[i] - p.p[3 + i]; hi[i] = p.p[i] + p.p[3 + i]; break;
      default:
        lo[i] = std::min(p.p[i], p.p[3 + i]) - p.p[6];
        hi[i] = std::max(p.p[i], p.p[3 + i]) + p.p[6];
    }
  }
}

// box of one copy of the modified shape in the primitive's frame: the local
// box grown by the elongation per axis and by rounding, shell and
// displacement amplitude on every side
static void modified_box(const HostPrim& p, double lo[3], double hi[3]) {
  local_box(p, lo, hi);
  const double g = p.round_r + p.onion_t + p.disp_a;
  for (int i = 0; i < 3; ++i) {
    lo[i] -= p.elong[i] + g;
    hi[i] += p.elong[i] + g;
  }
}

// turn rate of a twisted or bent primitive (0: neither)
static double turn_k(const HostPrim& p) { return p.twist_k != 0.0 ? p.twist_k : p.bend_k; }

// bounding cylinder about the local z axis of a twisted or bent primitive
// (a turn about z keeps the distance from the axis): radius 1.001 x the
// largest distance from the axis of its modified box, z range that box's
// grown by 0.1 % of its length at each end
static void twist_cylinder(const HostPrim& p, double* rho, double* zlo, double* zhi) {
  double lo[3], hi[3];
  modified_box(p, lo, hi);
  double r2 = 0.0;
  for (double x : {lo[0], hi[0]})
    for (double y : {lo[1], hi[1]}) r2 = std::max(r2, x * x + y * y);
  const double m = 1e-3 * (hi[2] - lo[2]);
  *rho = 1.001 * std::sqrt(r2);
  *zlo = lo[2] - m;
  *zhi = hi[2] + m;
}

// box of one copy: the modified box, or the twist's or bend's bounding
// cylinder's box
static void copy_box(const HostPrim& p, double a[3], double b[3]) {
  modified_box(p, a, b);
  if (turn_k(p) != 0.0) {
    double rho, z0, z1;
    twist_cylinder(p, &rho, &z0, &z1);
    a[0] = a[1] = -rho;
    b[0] = b[1] = rho;
    a[2] = z0;
    b[2] = z1;
  }
}

static bool repeated(const HostPrim& p) { return p.rep_n[0] > 1 || p.rep_n[1] > 1 || p.rep_n[2] > 1; }

// smallest distance from a copy's box to a face of its cell that another
// copy lies behind (<= 0: the copies do not fit their cells)
static double repetition_gap(const HostPrim& p) {
  double a[3], b[3];
  copy_box(p, a, b);
  double gap = 1e300;
  for (int i = 0; i < 3; ++i)
    if (p.rep_n[i] > 1) gap = std::min(gap, 0.5 * p.rep_c[i] - std::max(std::fabs(a[i]), std::fabs(b[i])));
  return gap;
}

// conservative world box of a primitive: the box of one copy over the
// repeated array, with the 8 corners placed in the world
static void prim_box(const HostPrim& p, double lo[3], double hi[3]) {
  double a[3], b[3];
  copy_box(p, a, b);
  for (int i = 0; i < 3; ++i) {
    const double ext = 0.5 * (p.rep_n[i] - 1) * p.rep_c[i];
    a[i] -= ext;
    b[i] += ext;
  }
  if (!p.placed) {
    for (int i = 0; i < 3; ++i) { lo[i] = a[i]; hi[i] = b[i]; }
    return;
  }
  for (int i = 0; i < 3; ++i) { lo[i] = 1e300; hi[i] = -1e300; }
  for (int c = 0; c < 8; ++c) {
    const double x[3] = {(c & 1) ? b[0] : a[0], (c & 2) ? b[1] : a[1], (c & 4) ? b[2] : a[2]};
    for (int i = 0; i < 3; ++i) {
      const double w = p.s * (p.rot[3 * i] * x[0] + p.rot[3 * i + 1] * x[1] + p.rot[3 * i + 2] * x[2]) + p.t[i];
      lo[i] = std::min(lo[i], w);
      hi[i] = std::max(hi[i], w);
    }
  }
}

// emission points of the source (for the simulation volume)
static void source_box(const smcrt_scene* s, double lo[3], double hi[3]) {
  const double* v = s->src;
  for (int i = 0; i < 3; ++i) lo[i] = hi[i] = v[i];
  if (s->src_kind == kDisc) {
    for (int i = 0; i < 2; ++i) { lo[i] -= v[3]; hi[i] += v[3]; }
  } else if (s->src_kind == kRect) {
    for (int i = 0; i < 2; ++i) { lo[i] -= v[3 + i]; hi[i] += v[3 + i]; }
  }
}

static void scene_bbox(const smcrt_scene* s, double lo[3], double hi[3], bool with_source, double pad) {
  for (int i = 0; i < 3; ++i) { lo[i] = 1e300; hi[i] = -1e300; }
  for (const HostPrim& p : s->prims) {
    double a[3], b[3];
    prim_box(p, a, b);
    for (int i = 0; i < 3; ++i) { lo[i] = std::min(lo[i], a[i]); hi[i] = std::max(hi[i], b[i]); }
  }
  if (with_source) {
    double a[3], b[3];
    source_box(s, a, b);
    for (int i = 0; i < 3; ++i) { lo[i] = std::min(lo[i], a[i]); hi[i] = std::max(hi[i], b[i]); }
  }
  for (int i = 0; i < 3; ++i) { lo[i] -= pad; hi[i] += pad; }
}

// a primitive as given: one of the basic shapes, unplaced and unmodified
static bool plain_shape(const HostPrim& hp) {
  return hp.kind < kCone && !hp.placed && turn_k(hp) == 0.0 && hp.round_r == 0.0 && hp.onion_t == 0.0 &&
         hp.disp_a == 0.0 && !repeated(hp) && hp.elong[0] == 0.0 && hp.elong[1] == 0.0 && hp.elong[2] == 0.0;
}

static smcrt_status check_complete(const smcrt_scene* s) {
  if (s->regions.empty()) return fail(SMCRT_E_INVALID, "scene has no region");
  if (!s->has_source) return fail(SMCRT_E_INVALID, "scene has no source");
  double lo[3], hi[3];
  scene_bbox(s, lo, hi, true, s->pad);
  const double* v = s->src;
  for (int i = 0; i < 3; ++i)
    if (!(v[i] >= lo[i] && v[i] <= hi[i])) return fail(SMCRT_E_INVALID, "source outside the simulation volume");
  if (s->geometry == kGeomVoxel && !(s->grid_set && s->g_dims[0] > 0 && s->g_dims[1] > 0 && s->g_dims[2] > 0))
    return fail(SMCRT_E_INVALID, "the voxel geometry needs a fluence grid with dims >= 1 in every axis");
  for (size_t i = 0; i < s->prims.size(); ++i)
    if (repeated(s->prims[i]) && !(repetition_gap(s->prims[i]) > 0.0))
      return fail(SMCRT_E_INVALID, "primitive %d: repeated copies no longer fit their cells", (int)i);
  if (s->segment && s->geometry != kGeomSdf)
    return fail(SMCRT_E_INVALID, "segment-traced steps need the SDF geometry, not the voxel model");
  if (s->segment)
    for (size_t i = 0; i < s->prims.size(); ++i)
      if (!plain_shape(s->prims[i]))
        return fail(SMCRT_E_INVALID, "segment-traced steps: primitive %d is placed, modified or of a further shape", (int)i);
  return SMCRT_OK;
}

// the segment-tracing rule of a region (the rounding-free argument needs
// exact distances of convex shapes): a union or intersection of plain
// convex primitives, or a subtraction from a plain convex one
static int seg_rule(const smcrt_scene* s, const HostRegion& r) {
  auto convex = [&](int32_t id) {
    const HostPrim& hp = s->prims[id];
    return plain_shape(hp) && hp.kind != kTorus;
  };
  switch (r.op) {
    case kUnion:
    case kIntersect:
      for (int32_t id : r.prims)
        if (!convex(id)) return kSegNone;
      return r.op == kUnion ? kSegUnion : kSegIntersect;
    case kSubtract:
      return convex(r.prims[0]) ? kSegSubtract : kSegNone;
    default:
      return kSegNone;
  }
}

template <typename T>
static void pack_prim(const HostPrim& h, Prim<T>& o) {
  std::memset(&o, 0, sizeof(o));
  o.kind = h.kind;
  const double* p = h.p;
  switch (h.kind) {
    case kSphere:
      for (int i = 0; i < 4; ++i) o.v[i] = (T)p[i];
      break;
    case kBox:
      for (int i = 0; i < 6; ++i) o.v[i] = (T)p[i];
      break;
    case kCapsule: {
      double ba[3] = {p[3] - p[0], p[4] - p[1], p[5] - p[2]};
      double bb = ba[0] * ba[0] + ba[1] * ba[1] + ba[2] * ba[2];
      for (int i = 0; i < 3; ++i) { o.v[i] = (T)p[i]; o.v[3 + i] = (T)ba[i]; }
      o.v[6] = (T)(1.0 / bb);
      o.v[7] = (T)p[6];
      break;
    }
    case kCylinder: {
      double ba[3] = {p[3] - p[0], p[4] - p[1], p[5] - p[2]};
      double L = std::sqrt(ba[0] * ba[0] + ba[1] * ba[1] + ba[2] * ba[2]);
      for (int i = 0; i < 3; ++i) { o.v[i] = (T)p[i]; o.v[3 + i] = (T)(ba[i] / L); }
      o.v[6] = (T)L;
      o.v[7] = (T)(0.5 * L);
      o.v[8] = (T)p[6];
      break;
    }
    case kTorus: {
      const double al = std::sqrt(p[3] * p[3] + p[4] * p[4] + p[5] * p[5]);
      for (int i = 0; i < 3; ++i) { o.v[i] = (T)p[i]; o.v[3 + i] = (T)(p[3 + i] / al); }
      o.v[6] = (T)p[6];
      o.v[7] = (T)p[7];
      break;
    }
    case kCone: {
      double ba[3] = {p[3] - p[0], p[4] - p[1], p[5] - p[2]};
      const double L = std::sqrt(ba[0] * ba[0] + ba[1] * ba[1] + ba[2] * ba[2]);
      for (int i = 0; i < 3; ++i) { o.v[i] = (T)p[i]; o.v[3 + i] = (T)(ba[i] / L); }
      o.v[6] = (T)L;
      o.v[7] = (T)p[6];
      o.v[8] = (T)p[7];
      break;
    }
    case kOctahedron:
      for (int i = 0; i < 4; ++i) o.v[i] = (T)p[i];
      break;
    case kHexPrism:
      for (int i = 0; i < 5; ++i) o.v[i] = (T)p[i];
      o.v[5] = (T)(2.0 * p[3] / std::sqrt(3.0));
      break;
    case kEllipsoid:
      for (int i = 0; i < 3; ++i) { o.v[i] = (T)p[i]; o.v[3 + i] = (T)(1.0 / p[3 + i]); }
      o.v[6] = (T)std::min(p[3], std::min(p[4], p[5]));
      break;
  }
  // placement and modifiers
  const bool elongated = h.elong[0] != 0.0 || h.elong[1] != 0.0 || h.elong[2] != 0.0;
  o.flags = (h.placed ? kPlaced : 0) | (turn_k(h) != 0.0 ? kTwisted : 0) | (h.bend_k != 0.0 ? kBent : 0) |
            ((h.round_r != 0.0 || h.onion_t != 0.0 || elongated || h.disp_a != 0.0) ? kModified : 0) |
            (repeated(h) ? kRepeated : 0) | (h.kind >= kCone ? kFurtherShape : 0);
  for (int i = 0; i < 3; ++i) {
    o.elong[i] = (T)h.elong[i];
    o.rep_c[i] = (T)h.rep_c[i];
    o.rep_n[i] = h.rep_n[i];
  }
  o.disp_a = (T)h.disp_a;
  o.disp_f = (T)h.disp_f;
  o.disp_inv_lip = (T)(1.0 / (1.0 + h.disp_a * h.disp_f * std::sqrt(3.0)));
  o.rep_gap = repeated(h) ? (T)repetition_gap(h) : T(0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) o.m[3 * i + j] = (T)(h.rot[3 * j + i] / h.s);
  for (int i = 0; i < 3; ++i) o.t[i] = (T)h.t[i];
  o.s = (T)h.s;
  o.round_r = (T)h.round_r;
  o.onion_t = (T)h.onion_t;
  if (turn_k(h) != 0.0) {
    double rho, z0, z1;
    twist_cylinder(h, &rho, &z0, &z1);
    o.twist_k = (T)turn_k(h);
    o.twist_rho = (T)rho;
    o.twist_zc = (T)(0.5 * (z0 + z1));
    o.twist_zh = (T)(0.5 * (z1 - z0));
    // Lipschitz bound of the untwist (unbend) map within radius rho: the
    // largest singular value of its Jacobian, (k rho + sqrt((k rho)^2 + 4))
    // / 2 (at most 1 + k rho)
    const double kr = std::fabs(turn_k(h)) * rho;
    o.inv_lip = (T)(h.bend_k != 0.0 ? 1.0 / (1.0 + kr) : 2.0 / (kr + std::sqrt(kr * kr + 4.0)));
  }
  prim_box(h, o.box_lo, o.box_hi);
}

static void fill_region(Region& r, double mua, double mus, double g, double n, double k, int op, int first, int count) {
  std::memset(&r, 0, sizeof(r));
  r.first = first;
  r.count = count;
  r.op = op;
  r.k = k;
  r.inv_k = k > 0 ? 1.0 / k : 0.0;
  r.mua = mua;
  r.mus = mus;
  r.mut = mua + mus;
  r.inv_mut = r.mut > 0 ? 1.0 / r.mut : 0.0;
  r.absorb = r.mut > 0 ? mua / r.mut : 0.0;
  r.g = g;
  r.n = n;
  r.iso = std::fabs(g) < 1e-6;
  r.hg_a = 1 + g * g;
  r.hg_b = 1 - g * g;
  r.hg_c = 1 - g;
  r.hg_d = 2 * g;
  r.hg_e = r.iso ? 0.0 : 1.0 / (2 * g);
  r.kf = (float)r.k;
  r.inv_kf = (float)r.inv_k;
  r.mutf = (float)r.mut;
  r.inv_mutf = (float)r.inv_mut;
  r.gf = (float)g;
  r.hg_af = (float)r.hg_a;
  r.hg_bf = (float)r.hg_b;
  r.hg_cf = (float)r.hg_c;
  r.hg_df = (float)r.hg_d;
  r.hg_ef = (float)r.hg_e;
}

// grid of the accelerated region: the primitives' box grown by a margin of
// one cell (the largest cell edge of the ungrown box), cut into the requested
// cells; capacity bounds the list entries from above (each primitive's cell
// range widened by one cell per side)
static smcrt_status pack_accel(const smcrt_scene* s, SceneHeader* h, const std::vector<int>& order) {
  Accel& A = h->acc;
  std::memset(&A, 0, sizeof(A));
  A.region = -1;
  if (s->accel_region < 0) return SMCRT_OK;
  const HostRegion& R = s->regions[s->accel_region];
  if (R.op != SMCRT_OP_UNION) return fail(SMCRT_E_INVALID, "accelerated region must be a union");
  int first = 0;
  for (int r = 0; r < s->accel_region; ++r) first += (int)s->regions[r].prims.size();
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int id : R.prims) {
    double a[3], b[3];
    prim_box(s->prims[id], a, b);
    for (int i = 0; i < 3; ++i) { lo[i] = std::min(lo[i], a[i]); hi[i] = std::max(hi[i], b[i]); }
  }
  double margin = 0.0;
  for (int i = 0; i < 3; ++i) margin = std::max(margin, (hi[i] - lo[i]) / s->accel_cells[i]);
  if (!(margin > 0)) return fail(SMCRT_E_INVALID, "accelerated region has an empty box");
  A.region = s->accel_region;
  A.first_prim = first;
  A.n_prims = (int32_t)R.prims.size();
  A.margin = margin;
  A.marginf = (float)margin;
  {
    double cmin = 1e300;
    for (int i = 0; i < 3; ++i) cmin = std::min(cmin, (hi[i] - lo[i] + 2.0 * margin) / s->accel_cells[i]);
    A.cell_min = cmin;
    A.cell_minf = std::nextafter((float)cmin, 0.0f);  // rounded down
  }
  int64_t cells = 1;
  for (int i = 0; i < 3; ++i) {
    A.dims[i] = s->accel_cells[i];
    cells *= A.dims[i];
    A.lo[i] = lo[i] - margin;
    A.inv_cell[i] = A.dims[i] / (hi[i] - lo[i] + 2.0 * margin);
    A.box_lo[i] = lo[i];
    A.box_hi[i] = hi[i];
    A.lof[i] = (float)A.lo[i];
    A.inv_cellf[i] = (float)A.inv_cell[i];
    A.box_lof[i] = (float)lo[i];
    A.box_hif[i] = (float)hi[i];
  }
  A.n_cells = (int32_t)cells;
  uint64_t cap = 0;
  for (int id : R.prims) {
    double a[3], b[3];
    prim_box(s->prims[id], a, b);
    uint64_t c = 1;
    for (int i = 0; i < 3; ++i) {
      int x0 = (int)std::floor((a[i] - margin - A.lo[i]) * A.inv_cell[i]) - 1;
      int x1 = (int)std::floor((b[i] + margin - A.lo[i]) * A.inv_cell[i]) + 1;
      x0 = std::max(x0, 0);
      x1 = std::min(x1, A.dims[i] - 1);
      c *= (uint64_t)std::max(x1 - x0 + 1, 1);
    }
    cap += c;
  }
  A.capacity = cap;
  (void)order;
  return SMCRT_OK;
}

static smcrt_status pack(smcrt_scene* s) {
  if (!s->dirty) return SMCRT_OK;
  smcrt_status st = check_complete(s);
  if (st != SMCRT_OK) return st;
  // primitives in region order, each region's list contiguous
  std::vector<int> order;
  for (const HostRegion& r : s->regions) order.insert(order.end(), r.prims.begin(), r.prims.end());
  size_t np = order.size();
  size_t off_d = (sizeof(SceneHeader) + 255) & ~size_t(255);
  size_t off_f = (off_d + np * sizeof(PrimD) + 255) & ~size_t(255);
  size_t bytes = off_f + np * sizeof(PrimF);
  // compact capsule records of the accelerated region when it holds plain
  // capsules only (the grid queries then read 32 or 64 bytes per capsule)
  size_t n_caps = 0, cap_d = 0, cap_f = 0;
  if (s->accel_region >= 0 && s->accel_region < (int)s->regions.size()) {
    bool plain = true;
    for (int32_t id : s->regions[s->accel_region].prims) {
      const HostPrim& hp = s->prims[id];
      if (hp.kind != kCapsule || hp.placed || turn_k(hp) != 0.0 || hp.round_r != 0.0 || hp.onion_t != 0.0 ||
          hp.disp_a != 0.0 || repeated(hp) || hp.elong[0] != 0.0 || hp.elong[1] != 0.0 || hp.elong[2] != 0.0)
        plain = false;
    }
    if (plain) {
      n_caps = s->regions[s->accel_region].prims.size();
      cap_d = (bytes + 255) & ~size_t(255);
      cap_f = (cap_d + n_caps * 8 * sizeof(double) + 255) & ~size_t(255);
      bytes = cap_f + n_caps * 8 * sizeof(float);
    }
  }
  s->blob.assign(bytes, 0);
  SceneHeader* h = reinterpret_cast<SceneHeader*>(s->blob.data());
  PrimD* pd = reinterpret_cast<PrimD*>(s->blob.data() + off_d);
  PrimF* pf = reinterpret_cast<PrimF*>(s->blob.data() + off_f);
  for (size_t i = 0; i < np; ++i) {
    pack_prim(s->prims[order[i]], pd[i]);
    pack_prim(s->prims[order[i]], pf[i]);
  }
  h->n_prims = (int32_t)np;
  h->n_regions = (int32_t)s->regions.size();
  int first = 0;
  for (size_t r = 0; r < s->regions.size(); ++r) {
    const HostRegion& hr = s->regions[r];
    fill_region(h->reg[r], hr.mua, hr.mus, hr.g, hr.n, hr.k, hr.op, first, (int)hr.prims.size());
    h->reg[r].seg = s->segment ? seg_rule(s, hr) : kSegNone;
    first += (int)hr.prims.size();
  }
  fill_region(h->reg[s->regions.size()], 0.0, 0.0, 0.0, s->n_ambient, 0.0, kUnion, 0, 0);
  h->delta = s->delta;
  h->deltaf = (float)s->delta;
  h->relax = s->relax;
  h->relax_k = 2.0 - s->relax;
  h->relaxf = (float)s->relax;
  h->relax_kf = (float)h->relax_k;
  h->segment = s->segment ? 1 : 0;
  h->h_normal = 1e-2 * s->delta;
  h->snap_cos = 0.1;
  h->offset = 2.0 * s->delta;
  double lo[3], hi[3];
  scene_bbox(s, lo, hi, true, s->pad);
  for (int i = 0; i < 3; ++i) {
    h->bb_c[i] = 0.5 * (lo[i] + hi[i]);
    h->bb_h[i] = 0.5 * (hi[i] - lo[i]);
    h->bb_cf[i] = (float)h->bb_c[i];
    h->bb_hf[i] = (float)h->bb_h[i];
  }
  {
    // rounding of a distance: 16 units in the last place of the largest
    // coordinate the computation meets (the volume's and the primitives')
    double big = 0.0;
    for (int i = 0; i < 3; ++i) big = std::max(big, std::fabs(h->bb_c[i]) + h->bb_h[i]);
    for (const HostPrim& hp : s->prims) {
      double a[3], b[3];
      prim_box(hp, a, b);
      for (int i = 0; i < 3; ++i) big = std::max(big, std::max(std::fabs(a[i]), std::fabs(b[i])));
    }
    h->seg_err = 16.0 * 0x1p-53 * big;
    h->seg_errf = (float)(16.0 * 0x1p-24 * big);
  }
  for (size_t r = 0; r < s->regions.size(); ++r) {
    // the surface of a region lies in its primitives' boxes; a smooth union
    // reaches at most k/4 beyond them
    const HostRegion& hr = s->regions[r];
    double rlo[3] = {1e300, 1e300, 1e300}, rhi[3] = {-1e300, -1e300, -1e300};
    for (int32_t id : hr.prims) {
      double a[3], b[3];
      prim_box(s->prims[id], a, b);
      for (int i = 0; i < 3; ++i) { rlo[i] = std::min(rlo[i], a[i]); rhi[i] = std::max(rhi[i], b[i]); }
    }
    const double grow = (hr.op == kSmoothUnion ? hr.k : 0.0) + 0.5 * s->delta;
    for (int i = 0; i < 3; ++i) {
      h->amb_lo[r][i] = rlo[i] - grow;
      h->amb_hi[r][i] = rhi[i] + grow;
      float fl = (float)h->amb_lo[r][i], fh = (float)h->amb_hi[r][i];
      if ((double)fl > h->amb_lo[r][i]) fl = std::nextafter(fl, -INFINITY);
      if ((double)fh < h->amb_hi[r][i]) fh = std::nextafter(fh, INFINITY);
      h->amb_lof[r][i] = fl;
      h->amb_hif[r][i] = fh;
    }
  }
  double glo[3], ghi[3];
  int32_t gd[3];
  if (s->grid_set) {
    std::memcpy(glo, s->g_lo, sizeof(glo));
    std::memcpy(ghi, s->g_hi, sizeof(ghi));
    std::memcpy(gd, s->g_dims, sizeof(gd));
  } else {
    scene_bbox(s, glo, ghi, false, 0.0);
    gd[0] = gd[1] = gd[2] = 1;
  }
  h->has_grid = gd[0] > 0 && gd[1] > 0 && gd[2] > 0;
  for (int i = 0; i < 3; ++i) {
    h->g_dims[i] = gd[i];
    h->g_lo[i] = glo[i];
    h->g_d[i] = gd[i] > 0 ? (ghi[i] - glo[i]) / gd[i] : 1.0;
    h->g_inv_d[i] = gd[i] > 0 ? gd[i] / (ghi[i] - glo[i]) : 1.0;
    h->g_hi[i] = ghi[i];
    h->g_lof[i] = (float)glo[i];
    h->g_inv_df[i] = (float)h->g_inv_d[i];
    h->g_df[i] = (float)h->g_d[i];
    h->g_hif[i] = (float)ghi[i];
  }
  h->geometry = s->geometry;
  h->xf = 0;
  for (const HostPrim& hp : s->prims)
    if (hp.kind >= kCone || hp.placed || turn_k(hp) != 0.0 || hp.round_r != 0.0 || hp.onion_t != 0.0 || hp.disp_a != 0.0 || repeated(hp) ||
        hp.elong[0] != 0.0 || hp.elong[1] != 0.0 || hp.elong[2] != 0.0)
      h->xf = 1;
  h->src_kind = s->src_kind;
  std::memcpy(h->src, s->src, sizeof(h->src));
  h->det_face = s->det_face;
  for (int i = 0; i < 2; ++i) {
    h->det_dims[i] = s->det_face >= 0 ? s->det_dims[i] : 0;
    h->det_lo[i] = s->det_lo[i];
    h->det_hi[i] = s->det_hi[i];
  }
  h->w_threshold = s->w_threshold;
  h->m_survive = s->m_survive;
  h->m_d = (double)s->m_survive;
  h->inv_m = 1.0 / (double)s->m_survive;
  h->max_steps = s->max_steps;
  h->max_events = s->max_events;
  st = pack_accel(s, h, order);
  if (st != SMCRT_OK) return st;
  if (n_caps && h->acc.region >= 0) {
    double* cd = reinterpret_cast<double*>(s->blob.data() + cap_d);
    float* cf = reinterpret_cast<float*>(s->blob.data() + cap_f);
    for (size_t i = 0; i < n_caps; ++i)
      for (int k = 0; k < 8; ++k) {
        cd[8 * i + k] = pd[h->acc.first_prim + i].v[k];
        cf[8 * i + k] = pf[h->acc.first_prim + i].v[k];
      }
    h->acc.caps = 1;
    h->acc.cap_offset_d = cap_d;
    h->acc.cap_offset_f = cap_f;
  }
  h->prim_offset_d = off_d;
  h->prim_offset_f = off_f;
  h->blob_bytes = bytes;
  s->dirty = false;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_scene_info(const smcrt_scene* s, int32_t* n_regions, int32_t* n_prims, double bb_lo[3],
                                         double bb_hi[3]) {
  if (!s) return fail(SMCRT_E_INVALID, "scene_info: NULL scene");
  if (n_regions) *n_regions = (int32_t)s->regions.size();
  if (n_prims) *n_prims = (int32_t)s->prims.size();
  if (bb_lo || bb_hi) {
    if (!s->has_source) return fail(SMCRT_E_STATE, "scene_info: set a source before asking for the volume");
    double lo[3], hi[3];
    scene_bbox(s, lo, hi, true, s->pad);
    if (bb_lo) std::memcpy(bb_lo, lo, sizeof(lo));
    if (bb_hi) std::memcpy(bb_hi, hi, sizeof(hi));
  }
  return SMCRT_OK;
}

// ------------------------------------------------------------------ engines

struct smcrt_engine {
  int device = 0;
  int n_cu = 0;
  smcrt_opts opts;
  // one device arena per engine: scene tables, job table, per-job packet
  // counters and the uniform-grid buffers, laid out afresh at every launch
  void* d_arena = nullptr;
  size_t arena_cap = 0;
  std::vector<unsigned char> image;  // host copy of the arena's uploaded prefix
  // pinned staging of that prefix; stage_done marks when the last upload
  // from it has been consumed by the device
  void* h_stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t stage_done = nullptr;
  bool stage_pending = false;
  // captured kernel sequence of the last launch shape (grid builds, counter
  // reset, walk), replayed while the arena layout and options are unchanged
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uint64_t> graph_key;
  uint64_t graph_replays = 0;
};

static void default_opts(smcrt_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->precision = SMCRT_PREC_F32;
  o->block = 256;
  o->blocks_per_cu = 0;  // 0 = as many as fit
  o->refill_min = 4;
  o->surface_min = 8;
}

static smcrt_status check_opts(const smcrt_opts* o) {
  if (o->precision != SMCRT_PREC_F32 && o->precision != SMCRT_PREC_F64)
    return fail(SMCRT_E_INVALID, "opts: unknown precision %d", o->precision);
  if (o->block < 64 || o->block > 256 || o->block % 64) return fail(SMCRT_E_INVALID, "opts: block must be 64, 128, 192 or 256");
  if (o->blocks_per_cu < 0 || o->blocks_per_cu > 32) return fail(SMCRT_E_INVALID, "opts: blocks_per_cu must be in [0, 32]");
  if (o->refill_min < 1 || o->refill_min > 64) return fail(SMCRT_E_INVALID, "opts: refill_min must be in [1, 64]");
  if (o->surface_min < 1 || o->surface_min > 64) return fail(SMCRT_E_INVALID, "opts: surface_min must be in [1, 64]");
  if (o->tally_layout != 0 && o->tally_layout != 1) return fail(SMCRT_E_INVALID, "opts: tally_layout must be 0 or 1");
  if (o->no_stage != 0 && o->no_stage != 1) return fail(SMCRT_E_INVALID, "opts: no_stage must be 0 or 1");
  return SMCRT_OK;
}

// Whether a job tallies into a grid of 2x2x2 bricks (tally_layout 0): FP32
// SDF walks on cubic voxels, up to 2^27 voxels.  Measured: on cubes the
// shared segments save more atomic requests than the brick index costs; on
// the flat voxels of the layered slab they do not.
static bool brick_tally(const smcrt_opts& o, const SceneHeader* h) {
  if (o.tally_layout != 0 || o.precision != SMCRT_PREC_F32 || h->geometry != kGeomSdf || !h->has_grid)
    return false;
  const double n = (double)h->g_dims[0] * h->g_dims[1] * h->g_dims[2];
  if (n > (double)(1 << 27)) return false;
  for (int i = 1; i < 3; ++i)
    if (std::fabs(h->g_d[i] - h->g_d[0]) > 1e-9 * h->g_d[0]) return false;
  return true;
}

// Launch class of a job (the kernel that runs it): its geometry model, plus
// kLaunchXf for placed or modified primitives; FP32 SDF jobs whose
// accelerated region is plain capsules that fit the LDS table run in the
// staged-capsule kernel (not for traces, which run one packet per thread);
// scenes with segment-traced steps (plain SDF scenes: the packer checks) in
// the segment kernel.
static int job_class(const smcrt_opts& o, const SceneHeader* h, bool trace) {
  if (h->segment) return kLaunchSegment;
  const int c = h->geometry + (h->xf ? kLaunchXf : 0);
  if (!trace && !o.no_stage && c == kGeomSdf && o.precision == SMCRT_PREC_F32 && h->acc.region >= 0 && h->acc.caps &&
      h->acc.n_prims <= kStageCaps)
    return kLaunchStaged;
  return c;
}

// voxels of the 2x2x2-brick grid of a scene's fluence grid (partial bricks
// at the far faces are whole)
static size_t brick_voxels(const SceneHeader* h) {
  return 8ull * (size_t)((h->g_dims[0] + 1) / 2) * (size_t)((h->g_dims[1] + 1) / 2) * (size_t)((h->g_dims[2] + 1) / 2);
}

extern "C" smcrt_status smcrt_engine_create(smcrt_engine** out, int device) {
  if (!out) return fail(SMCRT_E_INVALID, "engine_create: out is NULL");
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count), "hipGetDeviceCount");
  if (device < 0 || device >= count) return fail(SMCRT_E_INVALID, "engine_create: device %d not present (%d devices)", device, count);
  HIP_TRY(hipSetDevice(device), "hipSetDevice");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
  smcrt_engine* e = new (std::nothrow) smcrt_engine();
  if (!e) return fail(SMCRT_E_NOMEM, "engine_create: out of host memory");
  e->device = device;
  e->n_cu = prop.multiProcessorCount;
  default_opts(&e->opts);
  *out = e;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_engine_destroy(smcrt_engine* e) {
  if (!e) return SMCRT_OK;
  // best effort: the engine is going away whatever these return
  (void)hipSetDevice(e->device);
  (void)hipDeviceSynchronize();
  if (e->d_arena) (void)hipFree(e->d_arena);
  if (e->graph_exec) (void)hipGraphExecDestroy(e->graph_exec);
  if (e->capture_stream) (void)hipStreamDestroy(e->capture_stream);
  if (e->h_stage) (void)hipHostFree(e->h_stage);
  if (e->stage_done) (void)hipEventDestroy(e->stage_done);
  delete e;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_engine_get_opts(const smcrt_engine* e, smcrt_opts* out) {
  if (!e || !out) return fail(SMCRT_E_INVALID, "engine_get_opts: NULL argument");
  *out = e->opts;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_engine_set_opts(smcrt_engine* e, const smcrt_opts* o) {
  if (!e || !o) return fail(SMCRT_E_INVALID, "engine_set_opts: NULL argument");
  smcrt_status st = check_opts(o);
  if (st != SMCRT_OK) return st;
  e->opts = *o;
  return SMCRT_OK;
}

static LaunchCfg launch_cfg(smcrt_engine* e, int launch_class) {
  LaunchCfg c;
  c.block = launch_class == kLaunchStaged ? 1024 : e->opts.block;
  int per_cu = launch_class == kLaunchStaged ? 0 : e->opts.blocks_per_cu;
  if (per_cu <= 0) per_cu = walk_max_blocks_per_cu(e->opts.precision, c.block, launch_class);
  if (per_cu <= 0) per_cu = 1;
  c.grid = e->n_cu * per_cu;
  c.refill_min = e->opts.refill_min;
  c.surface_min = e->opts.surface_min;
  return c;
}

struct JobSpec {
  smcrt_scene* s;
  uint64_t seed, first, n;
  double* fluence;
  double* absorbed;
  smcrt_tallies* tallies;
  double* detector = nullptr;
};

struct TraceSpec {
  const uint64_t* ids;
  smcrt_event* out;
  int32_t* count;
  int n_ids, max_records;
};

// a point query (smcrt_scene_distance) of one job's scene
struct DistSpec {
  const double* points;
  uint64_t n;
  int accelerated;
  double* dist;
  int32_t* owner;
  double* normals;
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Lays the jobs' scenes, the job table, the per-job counters, the uniform
// grids and the voxel grids out in the engine arena, uploads the tables,
// builds the uniform grids, voxelises the voxel-model scenes, zeroes the
// counters and launches the walk of each geometry present -- all on `st`.
// With vox_out (one job) it stops after voxelising that scene into vox_out.
static smcrt_status launch_jobs(smcrt_engine* e, const std::vector<JobSpec>& jobs, const TraceSpec* tr, hipStream_t st,
                                uint8_t* vox_out = nullptr, const DistSpec* dq = nullptr) {
  if (jobs.empty()) return SMCRT_OK;
  std::vector<smcrt_scene*> uniq;
  std::vector<int> job_scene(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) {
    smcrt_status r = pack(jobs[j].s);
    if (r != SMCRT_OK) return r;
    int k = -1;
    for (size_t u = 0; u < uniq.size(); ++u)
      if (uniq[u] == jobs[j].s) k = (int)u;
    if (k < 0) {
      k = (int)uniq.size();
      uniq.push_back(jobs[j].s);
    }
    job_scene[j] = k;
  }
  // layout
  std::vector<size_t> blob_off(uniq.size()), acc_off(uniq.size(), 0), vox_off(uniq.size(), 0), vox_n(uniq.size(), 0);
  size_t off = 0;
  for (size_t u = 0; u < uniq.size(); ++u) {
    blob_off[u] = off;
    off = align256(off + uniq[u]->blob.size());
  }
  const size_t jobs_off = off;
  off = align256(off + jobs.size() * sizeof(WalkArgs));
  const size_t image_bytes = off;
  const size_t counters_off = off;
  off = align256(off + jobs.size() * sizeof(unsigned long long));
  for (size_t u = 0; u < uniq.size(); ++u) {
    const Accel& A = reinterpret_cast<const SceneHeader*>(uniq[u]->blob.data())->acc;
    if (A.region < 0) continue;
    acc_off[u] = off;
    off += 3 * align256(sizeof(uint32_t) * ((size_t)A.n_cells + 1)) + align256(sizeof(uint32_t) * A.capacity);
  }
  for (size_t u = 0; u < uniq.size(); ++u) {
    const SceneHeader* h = reinterpret_cast<const SceneHeader*>(uniq[u]->blob.data());
    if (dq || (h->geometry != kGeomVoxel && !vox_out)) continue;
    vox_n[u] = (size_t)h->g_dims[0] * h->g_dims[1] * h->g_dims[2];
    if (vox_out) continue;
    vox_off[u] = off;
    off = align256(off + vox_n[u]);
  }
  // brick grids of the jobs that tally into one
  std::vector<size_t> brick_off(jobs.size(), 0), brick_n(jobs.size(), 0);
  for (size_t j = 0; j < jobs.size(); ++j) {
    const SceneHeader* h = reinterpret_cast<const SceneHeader*>(uniq[job_scene[j]]->blob.data());
    if (tr || vox_out || dq || !jobs[j].fluence || !brick_tally(e->opts, h)) continue;
    brick_n[j] = brick_voxels(h);
    brick_off[j] = off;
    off = align256(off + sizeof(double) * brick_n[j]);
  }
  const size_t total = off;
  if (total > e->arena_cap) {
    if (e->d_arena) {
      HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
      HIP_TRY(hipFree(e->d_arena), "hipFree(arena)");
      e->d_arena = nullptr;
      e->arena_cap = 0;
    }
    const size_t cap = total + total / 4;
    HIP_TRY(hipMalloc(&e->d_arena, cap), "hipMalloc(arena)");
    e->arena_cap = cap;
  }
  char* base = static_cast<char*>(e->d_arena);
  // host image: scene tables and the job table
  e->image.assign(image_bytes, 0);
  for (size_t u = 0; u < uniq.size(); ++u) std::memcpy(e->image.data() + blob_off[u], uniq[u]->blob.data(), uniq[u]->blob.size());
  WalkArgs* table = reinterpret_cast<WalkArgs*>(e->image.data() + jobs_off);
  for (size_t j = 0; j < jobs.size(); ++j) {
    const int u = job_scene[j];
    const SceneHeader* h = reinterpret_cast<const SceneHeader*>(uniq[u]->blob.data());
    WalkArgs& a = table[j];
    std::memset(&a, 0, sizeof(a));
    char* sc = base + blob_off[u];
    a.sc = reinterpret_cast<const SceneHeader*>(sc);
    a.pd = reinterpret_cast<const PrimD*>(sc + h->prim_offset_d);
    a.pf = reinterpret_cast<const PrimF*>(sc + h->prim_offset_f);
    a.seed = jobs[j].seed;
    a.first = jobs[j].first;
    a.n = jobs[j].n;
    a.counter = reinterpret_cast<unsigned long long*>(base + counters_off) + j;
    a.fluence = h->has_grid ? jobs[j].fluence : nullptr;
    a.absorbed = jobs[j].absorbed;
    a.detector = h->det_face >= 0 ? jobs[j].detector : nullptr;
    a.tallies = jobs[j].tallies;
    a.acc_region = h->acc.region;
    a.geometry = tr ? job_class(e->opts, h, true) : job_class(e->opts, h, false);
    if (h->acc.region >= 0 && h->acc.caps) {
      a.acc_capd = reinterpret_cast<const double*>(sc + h->acc.cap_offset_d);
      a.acc_capf = reinterpret_cast<const float*>(sc + h->acc.cap_offset_f);
    }
    if (vox_n[u]) a.vox = vox_out ? vox_out : reinterpret_cast<uint8_t*>(base + vox_off[u]);
    if (brick_n[j]) {
      a.fluence = reinterpret_cast<double*>(base + brick_off[j]);
      a.brick = 1;
    }
    if (h->acc.region >= 0) {
      const size_t cb = align256(sizeof(uint32_t) * ((size_t)h->acc.n_cells + 1));
      a.acc_offsets = reinterpret_cast<const uint32_t*>(base + acc_off[u] + 2 * cb);
      a.acc_ids = reinterpret_cast<const uint32_t*>(base + acc_off[u] + 3 * cb);
      a.acc_rings = reinterpret_cast<const uint32_t*>(base + acc_off[u]);
    }
    if (tr) {
      a.trace_ids = tr->ids;
      a.trace_out = tr->out;
      a.trace_count = tr->count;
      a.n_trace = tr->n_ids;
      a.max_records = tr->max_records;
      a.fluence = nullptr;
      a.detector = nullptr;
    }
  }
  // upload through pinned staging; wait until the previous upload left it
  if (e->stage_pending) {
    HIP_TRY(hipEventSynchronize(e->stage_done), "hipEventSynchronize(stage)");
    e->stage_pending = false;
  }
  if (image_bytes > e->stage_cap) {
    if (e->h_stage) HIP_TRY(hipHostFree(e->h_stage), "hipHostFree");
    e->h_stage = nullptr;
    e->stage_cap = 0;
    HIP_TRY(hipHostMalloc(&e->h_stage, image_bytes + image_bytes / 4, hipHostMallocDefault), "hipHostMalloc(stage)");
    e->stage_cap = image_bytes + image_bytes / 4;
  }
  if (!e->stage_done) HIP_TRY(hipEventCreateWithFlags(&e->stage_done, hipEventDisableTiming), "hipEventCreate");
  std::memcpy(e->h_stage, e->image.data(), image_bytes);
  HIP_TRY(hipMemcpyAsync(e->d_arena, e->h_stage, image_bytes, hipMemcpyHostToDevice, st), "hipMemcpyAsync(tables)");
  HIP_TRY(hipEventRecord(e->stage_done, st), "hipEventRecord(stage)");
  e->stage_pending = true;
  BatchArgs B;
  std::memset(&B, 0, sizeof(B));
  B.jobs = reinterpret_cast<const WalkArgs*>(base + jobs_off);
  B.n_jobs = (int32_t)jobs.size();
  B.refill_min = e->opts.refill_min;
  B.surface_min = e->opts.surface_min;
  bool has_geom[kLaunchClasses] = {};
  for (size_t j = 0; j < jobs.size(); ++j) has_geom[table[j].geometry] = true;
  LaunchCfg cg[kLaunchClasses];
  for (int g = 0; g < kLaunchClasses; ++g) cg[g] = launch_cfg(e, g);
  if (tr) {
    for (LaunchCfg& c : cg) {
      c.block = 64;
      c.grid = (tr->n_ids + 63) / 64;
    }
  }
  // the device-side sequence after the upload
  auto enqueue = [&](hipStream_t q) -> smcrt_status {
    for (size_t u = 0; u < uniq.size(); ++u) {
      const SceneHeader* h = reinterpret_cast<const SceneHeader*>(uniq[u]->blob.data());
      if (h->acc.region < 0) continue;
      const size_t cb = align256(sizeof(uint32_t) * ((size_t)h->acc.n_cells + 1));
      char* ab = base + acc_off[u];
      char* sc = base + blob_off[u];
      HIP_TRY(launch_accel_build(reinterpret_cast<const SceneHeader*>(sc), reinterpret_cast<const PrimD*>(sc + h->prim_offset_d),
                                 h->acc.n_prims, h->acc.n_cells, reinterpret_cast<uint32_t*>(ab),
                                 reinterpret_cast<uint32_t*>(ab + cb), reinterpret_cast<uint32_t*>(ab + 2 * cb),
                                 reinterpret_cast<uint32_t*>(ab + 3 * cb), q),
              "accel build");
    }
    for (size_t u = 0; u < uniq.size(); ++u) {
      if (!vox_n[u]) continue;
      int j0 = 0;
      while (job_scene[j0] != (int)u) ++j0;
      uint8_t* vb = vox_out ? vox_out : reinterpret_cast<uint8_t*>(base + vox_off[u]);
      HIP_TRY(launch_voxelize(B.jobs, j0, vb, vox_n[u], q), "voxelize");
    }
    if (vox_out) return SMCRT_OK;
    if (dq) {
      HIP_TRY(launch_distance(e->opts.precision, B.jobs, 0, dq->points, dq->n, dq->accelerated, dq->dist, dq->owner,
                              dq->normals, q),
              "distance kernel");
      return SMCRT_OK;
    }
    HIP_TRY(launch_zero_u64_n(reinterpret_cast<unsigned long long*>(base + counters_off), (int)jobs.size(), q), "zero counters");
    for (size_t j = 0; j < jobs.size(); ++j)
      if (brick_n[j]) HIP_TRY(launch_zero_f64(reinterpret_cast<double*>(base + brick_off[j]), brick_n[j], q), "zero brick grid");
    for (int g = 0; g < kLaunchClasses; ++g) {
      if (!has_geom[g]) continue;
      BatchArgs Bg = B;
      Bg.geometry = g;
      HIP_TRY(launch_walk(e->opts.precision, tr != nullptr, cg[g], Bg, q), "walk kernel");
    }
    for (size_t j = 0; j < jobs.size(); ++j) {
      if (!brick_n[j]) continue;
      const int32_t* d = reinterpret_cast<const SceneHeader*>(uniq[job_scene[j]]->blob.data())->g_dims;
      HIP_TRY(launch_brick_add(reinterpret_cast<const double*>(base + brick_off[j]), jobs[j].fluence, d[0], d[1], d[2], q),
              "add brick grid");
    }
    return SMCRT_OK;
  };
  if (!e->opts.use_graph || tr || vox_out || dq) return enqueue(st);
  // replay the captured sequence when the launch shape is the same
  std::vector<uint64_t> key = {(uint64_t)(uintptr_t)base, image_bytes, total, jobs.size(), (uint64_t)cg[0].block,
                               (uint64_t)e->opts.precision, (uint64_t)B.refill_min, (uint64_t)B.surface_min};
  for (int g = 0; g < kLaunchClasses; ++g) {
    key.push_back((uint64_t)cg[g].grid);
    key.push_back((uint64_t)has_geom[g]);
  }
  for (size_t j = 0; j < jobs.size(); ++j) {
    key.push_back(brick_off[j]);
    key.push_back(brick_n[j]);
    key.push_back((uint64_t)(uintptr_t)jobs[j].fluence);
  }
  for (size_t u = 0; u < uniq.size(); ++u) {
    const Accel& A = reinterpret_cast<const SceneHeader*>(uniq[u]->blob.data())->acc;
    key.push_back(blob_off[u]);
    key.push_back((uint64_t)A.region);
    key.push_back((uint64_t)A.n_prims);
    key.push_back((uint64_t)A.n_cells);
    key.push_back(vox_off[u]);
    key.push_back(vox_n[u]);
  }
  if (!e->graph_exec || key != e->graph_key) {
    if (e->graph_exec) {
      HIP_TRY(hipGraphExecDestroy(e->graph_exec), "hipGraphExecDestroy");
      e->graph_exec = nullptr;
    }
    if (!e->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&e->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
    HIP_TRY(hipStreamBeginCapture(e->capture_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    smcrt_status r = enqueue(e->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(e->capture_stream, &g);
    if (r != SMCRT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&e->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      e->graph_exec = nullptr;
      return hip_fail(ie, "hipGraphInstantiate");
    }
    e->graph_key = key;
  } else {
    ++e->graph_replays;
  }
  HIP_TRY(hipGraphLaunch(e->graph_exec, st), "hipGraphLaunch");
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_run_ex(smcrt_engine* e, const smcrt_scene* scene, uint64_t seed, uint64_t first_packet,
                                     uint64_t n_packets, const smcrt_outputs* out, void* hip_stream) {
  if (!e || !scene || !out) return fail(SMCRT_E_INVALID, "run: NULL engine, scene or outputs");
  if (!out->absorbed || !out->tallies) return fail(SMCRT_E_INVALID, "run: absorbed and tallies are required");
  if (n_packets == 0) return SMCRT_OK;
  if (first_packet + n_packets < first_packet) return fail(SMCRT_E_INVALID, "run: packet range overflows 64 bits");
  HIP_TRY(hipSetDevice(e->device), "hipSetDevice");
  std::vector<JobSpec> jobs(1);
  jobs[0] = JobSpec{const_cast<smcrt_scene*>(scene), seed, first_packet, n_packets, out->fluence_raw, out->absorbed,
                    out->tallies, out->detector};
  return launch_jobs(e, jobs, nullptr, (hipStream_t)hip_stream);
}

extern "C" smcrt_status smcrt_run(smcrt_engine* e, const smcrt_scene* scene, uint64_t seed, uint64_t first_packet,
                                  uint64_t n_packets, double* d_fluence_raw, double* d_absorbed, smcrt_tallies* d_tallies,
                                  void* hip_stream) {
  const smcrt_outputs out{d_fluence_raw, d_absorbed, d_tallies, nullptr};
  return smcrt_run_ex(e, scene, seed, first_packet, n_packets, &out, hip_stream);
}

// smcrt_run_ex without device allocation: the scene tables, the job record,
// the packet counter, the uniform-grid build buffers and the voxel grid are
// laid out in the library's fixed device scratch (static_run.hip), and the
// walk tallies straight into the caller's grid (no brick grid).  Device
// work: the table upload (from the scene's own packed tables), then kernels
// only (job record, counter reset, grid builds, walk).
extern "C" smcrt_status smcrt_run_ex_static(smcrt_engine* e, const smcrt_scene* scene, uint64_t seed,
                                            uint64_t first_packet, uint64_t n_packets, const smcrt_outputs* out,
                                            void* hip_stream) {
  if (!e || !scene || !out) return fail(SMCRT_E_INVALID, "run_ex_static: NULL engine, scene or outputs");
  if (!out->absorbed || !out->tallies) return fail(SMCRT_E_INVALID, "run_ex_static: absorbed and tallies are required");
  if (n_packets == 0) return SMCRT_OK;
  if (first_packet + n_packets < first_packet) return fail(SMCRT_E_INVALID, "run_ex_static: packet range overflows 64 bits");
  smcrt_scene* s = const_cast<smcrt_scene*>(scene);
  smcrt_status st = pack(s);
  if (st != SMCRT_OK) return st;
  const SceneHeader* h = reinterpret_cast<const SceneHeader*>(s->blob.data());
  // layout in the scratch: tables, job record, counter, grid-build buffers, voxels
  const size_t jobs_off = align256(s->blob.size());
  const size_t counter_off = align256(jobs_off + sizeof(WalkArgs));
  size_t off = align256(counter_off + sizeof(unsigned long long));
  size_t acc_off = 0, cb = 0, vox_off = 0, vox_n = 0;
  if (h->acc.region >= 0) {
    acc_off = off;
    cb = align256(sizeof(uint32_t) * ((size_t)h->acc.n_cells + 1));
    off = acc_off + 3 * cb + align256(sizeof(uint32_t) * h->acc.capacity);
  }
  if (h->geometry == kGeomVoxel) {
    vox_n = (size_t)h->g_dims[0] * h->g_dims[1] * h->g_dims[2];
    vox_off = off;
    off = align256(off + vox_n);
  }
  if (off > kStaticScratchBytes)
    return fail(SMCRT_E_INVALID, "run_ex_static: the scene needs %zu bytes of device scratch, the static scratch holds %zu",
                off, kStaticScratchBytes);
  HIP_TRY(hipSetDevice(e->device), "hipSetDevice");
  void* base_v = nullptr;
  HIP_TRY(static_scratch(e->device, &base_v), "static scratch address");
  char* base = static_cast<char*>(base_v);
  const hipStream_t q = (hipStream_t)hip_stream;
  WalkArgs a;
  std::memset(&a, 0, sizeof(a));
  a.sc = reinterpret_cast<const SceneHeader*>(base);
  a.pd = reinterpret_cast<const PrimD*>(base + h->prim_offset_d);
  a.pf = reinterpret_cast<const PrimF*>(base + h->prim_offset_f);
  a.seed = seed;
  a.first = first_packet;
  a.n = n_packets;
  a.counter = reinterpret_cast<unsigned long long*>(base + counter_off);
  a.fluence = h->has_grid ? out->fluence_raw : nullptr;
  a.absorbed = out->absorbed;
  a.detector = h->det_face >= 0 ? out->detector : nullptr;
  a.tallies = out->tallies;
  a.acc_region = h->acc.region;
  a.geometry = job_class(e->opts, h, false);
  if (h->acc.region >= 0 && h->acc.caps) {
    a.acc_capd = reinterpret_cast<const double*>(base + h->acc.cap_offset_d);
    a.acc_capf = reinterpret_cast<const float*>(base + h->acc.cap_offset_f);
  }
  if (vox_n) a.vox = reinterpret_cast<uint8_t*>(base + vox_off);
  if (h->acc.region >= 0) {
    a.acc_offsets = reinterpret_cast<const uint32_t*>(base + acc_off + 2 * cb);
    a.acc_ids = reinterpret_cast<const uint32_t*>(base + acc_off + 3 * cb);
    a.acc_rings = reinterpret_cast<const uint32_t*>(base + acc_off);
  }
  WalkArgs* d_job = reinterpret_cast<WalkArgs*>(base + jobs_off);
  HIP_TRY(hipMemcpyAsync(base, s->blob.data(), s->blob.size(), hipMemcpyHostToDevice, q), "hipMemcpyAsync(tables)");
  HIP_TRY(launch_write_job(a, d_job, q), "job record");
  if (h->acc.region >= 0)
    HIP_TRY(launch_accel_build(a.sc, a.pd, h->acc.n_prims, h->acc.n_cells, reinterpret_cast<uint32_t*>(base + acc_off),
                               reinterpret_cast<uint32_t*>(base + acc_off + cb),
                               reinterpret_cast<uint32_t*>(base + acc_off + 2 * cb),
                               reinterpret_cast<uint32_t*>(base + acc_off + 3 * cb), q),
            "accel build");
  if (vox_n) HIP_TRY(launch_voxelize(d_job, 0, a.vox, vox_n, q), "voxelize");
  HIP_TRY(launch_zero_u64(a.counter, q), "zero counter");
  BatchArgs B;
  std::memset(&B, 0, sizeof(B));
  B.jobs = d_job;
  B.n_jobs = 1;
  B.refill_min = e->opts.refill_min;
  B.surface_min = e->opts.surface_min;
  B.geometry = a.geometry;
  HIP_TRY(launch_walk(e->opts.precision, false, launch_cfg(e, a.geometry), B, q), "walk kernel");
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_run_batch_ex(smcrt_engine* e, int n, const smcrt_scene* const* scenes, const uint64_t* seeds,
                                           const uint64_t* first_packets, const uint64_t* n_packets,
                                           const smcrt_outputs* outs, void* hip_stream) {
  if (!e || n < 1 || !scenes || !seeds || !n_packets || !outs)
    return fail(SMCRT_E_INVALID, "run_batch: NULL argument or n < 1");
  std::vector<JobSpec> jobs;
  for (int j = 0; j < n; ++j) {
    if (!scenes[j]) return fail(SMCRT_E_INVALID, "run_batch: scene %d is NULL", j);
    if (!outs[j].absorbed || !outs[j].tallies) return fail(SMCRT_E_INVALID, "run_batch: job %d lacks absorbed or tallies", j);
    const uint64_t first = first_packets ? first_packets[j] : 0;
    if (first + n_packets[j] < first) return fail(SMCRT_E_INVALID, "run_batch: job %d packet range overflows", j);
    if (n_packets[j] == 0) continue;
    jobs.push_back(JobSpec{const_cast<smcrt_scene*>(scenes[j]), seeds[j], first, n_packets[j], outs[j].fluence_raw,
                           outs[j].absorbed, outs[j].tallies, outs[j].detector});
  }
  if (jobs.empty()) return SMCRT_OK;
  HIP_TRY(hipSetDevice(e->device), "hipSetDevice");
  return launch_jobs(e, jobs, nullptr, (hipStream_t)hip_stream);
}

extern "C" smcrt_status smcrt_run_batch(smcrt_engine* e, int n, const smcrt_scene* const* scenes, const uint64_t* seeds,
                                        const uint64_t* first_packets, const uint64_t* n_packets, double* const* d_fluence_raw,
                                        double* const* d_absorbed, smcrt_tallies* const* d_tallies, void* hip_stream) {
  if (!e || n < 1 || !scenes || !seeds || !n_packets || !d_fluence_raw || !d_absorbed || !d_tallies)
    return fail(SMCRT_E_INVALID, "run_batch: NULL argument or n < 1");
  std::vector<smcrt_outputs> outs((size_t)n);
  for (int j = 0; j < n; ++j) outs[j] = smcrt_outputs{d_fluence_raw[j], d_absorbed[j], d_tallies[j], nullptr};
  return smcrt_run_batch_ex(e, n, scenes, seeds, first_packets, n_packets, outs.data(), hip_stream);
}

// The autotuner over one launch of the given scenes (n_trial packets each):
// the launch-shape grid, then the tally layout and the capsule staging where
// a scene gives that choice.  Scratch outputs are shared by the jobs (their
// sums are not read).
static smcrt_status autotune_jobs(smcrt_engine* e, const std::vector<smcrt_scene*>& scenes, uint64_t n_trial,
                                  smcrt_opts* out_best, double* out_packets_per_s) {
  if (n_trial < 1000) return fail(SMCRT_E_INVALID, "autotune: n_trial must be >= 1000");
  std::vector<const SceneHeader*> hs;
  size_t nvox = 0;
  for (smcrt_scene* s : scenes) {
    smcrt_status st = pack(s);
    if (st != SMCRT_OK) return st;
    const SceneHeader* h = reinterpret_cast<const SceneHeader*>(s->blob.data());
    hs.push_back(h);
    if (h->has_grid) nvox = std::max(nvox, (size_t)h->g_dims[0] * h->g_dims[1] * h->g_dims[2]);
  }
  HIP_TRY(hipSetDevice(e->device), "hipSetDevice");
  // scratch outputs and a private stream
  double *f = nullptr, *ab = nullptr;
  smcrt_tallies* t = nullptr;
  hipStream_t q = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (q) (void)hipStreamSynchronize(q);
    if (f) (void)hipFree(f);
    if (ab) (void)hipFree(ab);
    if (t) (void)hipFree(t);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (q) (void)hipStreamDestroy(q);
  };
  hipError_t err = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
  if (err == hipSuccess && nvox) err = hipMalloc(&f, sizeof(double) * nvox);
  if (err == hipSuccess) err = hipMalloc(&ab, sizeof(double) * kMaxRegions);
  if (err == hipSuccess) err = hipMalloc(&t, sizeof(smcrt_tallies));
  if (err == hipSuccess) err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  if (err != hipSuccess) {
    cleanup();
    return hip_fail(err, "autotune set-up");
  }
  const smcrt_opts base = e->opts;
  const int max_per_cu = walk_max_blocks_per_cu(base.precision, 256, kGeomSdf);
  struct Shape { int block, per_cu; };
  std::vector<Shape> shapes = {{256, 0}, {128, 0}};
  if (max_per_cu > 1) shapes.push_back({256, max_per_cu - 1});
  const int refills[3] = {1, 4, 16}, surfaces[3] = {4, 8, 16};
  smcrt_opts best = base;
  double best_rate = -1.0;
  smcrt_status r = SMCRT_OK;
  std::vector<JobSpec> jobs(scenes.size());
  for (size_t j = 0; j < scenes.size(); ++j) jobs[j] = JobSpec{scenes[j], 0x5eedull + j, 0, n_trial, f, ab, t};
  const double packets = (double)n_trial * (double)scenes.size();
  // one warm run and one timed run under o; false on an error (in r or err)
  auto trial = [&](const smcrt_opts& o) {
    e->opts = o;
    e->opts.use_graph = 0;
    r = launch_jobs(e, jobs, nullptr, q);  // warm
    if (r != SMCRT_OK) return false;
    if ((err = hipEventRecord(e0, q)) != hipSuccess) return false;
    r = launch_jobs(e, jobs, nullptr, q);
    if (r != SMCRT_OK) return false;
    if ((err = hipEventRecord(e1, q)) != hipSuccess || (err = hipEventSynchronize(e1)) != hipSuccess) return false;
    float ms = 0.f;
    if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return false;
    const double rate = packets / (ms * 1e-3);
    if (rate > best_rate) {
      best_rate = rate;
      best = o;
    }
    return true;
  };
  bool ok = true;
  for (const Shape& sh : shapes)
    for (int rf : refills)
      for (int sf : surfaces) {
        if (!ok) break;
        smcrt_opts o = base;
        o.block = sh.block;
        o.blocks_per_cu = sh.per_cu;
        o.refill_min = rf;
        o.surface_min = sf;
        ok = trial(o);
      }
  // then, from the best shape, the tally layout and the capsule staging
  // where the scene gives a choice (the brick grid, the LDS capsule table)
  if (ok) {
    smcrt_opts o = best;
    o.tally_layout = 0;
    bool choice = false;
    for (const SceneHeader* h : hs) choice = choice || brick_tally(o, h);
    if (choice) {
      o.tally_layout = 1 - best.tally_layout;
      ok = trial(o);
    }
  }
  if (ok) {
    smcrt_opts o = best;
    o.no_stage = 0;
    bool choice = false;
    for (const SceneHeader* h : hs) choice = choice || job_class(o, h, false) == kLaunchStaged;
    if (choice) {
      o.no_stage = 1 - best.no_stage;
      ok = trial(o);
    }
  }
  best.use_graph = base.use_graph;
  cleanup();
  e->opts = (r == SMCRT_OK && err == hipSuccess) ? best : base;
  if (r != SMCRT_OK) return r;
  if (err != hipSuccess) return hip_fail(err, "autotune timing");
  if (out_best) *out_best = best;
  if (out_packets_per_s) *out_packets_per_s = best_rate;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_engine_autotune(smcrt_engine* e, const smcrt_scene* scene, uint64_t n_trial,
                                              smcrt_opts* out_best, double* out_packets_per_s) {
  if (!e || !scene) return fail(SMCRT_E_INVALID, "autotune: NULL engine or scene");
  return autotune_jobs(e, {const_cast<smcrt_scene*>(scene)}, n_trial, out_best, out_packets_per_s);
}

extern "C" smcrt_status smcrt_engine_autotune_batch(smcrt_engine* e, int n, const smcrt_scene* const* scenes,
                                                    uint64_t n_trial, smcrt_opts* out_best, double* out_packets_per_s) {
  if (!e || n < 1 || !scenes) return fail(SMCRT_E_INVALID, "autotune_batch: NULL engine or scenes, or n < 1");
  std::vector<smcrt_scene*> v((size_t)n);
  for (int j = 0; j < n; ++j) {
    if (!scenes[j]) return fail(SMCRT_E_INVALID, "autotune_batch: NULL scene %d", j);
    v[j] = const_cast<smcrt_scene*>(scenes[j]);
  }
  return autotune_jobs(e, v, n_trial, out_best, out_packets_per_s);
}

extern "C" smcrt_status smcrt_trace(smcrt_engine* e, const smcrt_scene* scene, uint64_t seed, const uint64_t* d_packet_ids,
                                    int n_ids, int max_events, smcrt_event* d_out, int32_t* d_count, void* hip_stream) {
  if (!e || !scene || !d_packet_ids || !d_out || !d_count) return fail(SMCRT_E_INVALID, "trace: NULL argument");
  if (n_ids < 1 || max_events < 1) return fail(SMCRT_E_INVALID, "trace: need n_ids >= 1 and max_events >= 1");
  if ((int64_t)n_ids * max_events > (1LL << 31)) return fail(SMCRT_E_INVALID, "trace: too many records");
  HIP_TRY(hipSetDevice(e->device), "hipSetDevice");
  std::vector<JobSpec> jobs(1);
  jobs[0] = JobSpec{const_cast<smcrt_scene*>(scene), seed, 0, 0, nullptr, nullptr, nullptr};
  TraceSpec tr{d_packet_ids, d_out, d_count, n_ids, max_events};
  return launch_jobs(e, jobs, &tr, (hipStream_t)hip_stream);
}

extern "C" smcrt_status smcrt_voxelize(smcrt_engine* e, const smcrt_scene* scene, uint8_t* d_out, void* hip_stream) {
  if (!e || !scene || !d_out) return fail(SMCRT_E_INVALID, "voxelize: NULL engine, scene or output");
  if (!(scene->grid_set && scene->g_dims[0] > 0 && scene->g_dims[1] > 0 && scene->g_dims[2] > 0))
    return fail(SMCRT_E_INVALID, "voxelize: the scene needs a fluence grid with dims >= 1 in every axis");
  HIP_TRY(hipSetDevice(e->device), "hipSetDevice");
  std::vector<JobSpec> jobs(1);
  jobs[0] = JobSpec{const_cast<smcrt_scene*>(scene), 0, 0, 0, nullptr, nullptr, nullptr};
  return launch_jobs(e, jobs, nullptr, (hipStream_t)hip_stream, d_out);
}

extern "C" smcrt_status smcrt_scene_distance(smcrt_engine* e, const smcrt_scene* scene, const double* d_points, uint64_t n,
                                             int32_t accelerated, double* d_dist, int32_t* d_owner, double* d_normals,
                                             void* hip_stream) {
  if (!e || !scene) return fail(SMCRT_E_INVALID, "scene_distance: NULL engine or scene");
  if (accelerated != 0 && accelerated != 1) return fail(SMCRT_E_INVALID, "scene_distance: accelerated must be 0 or 1");
  if (n == 0) return SMCRT_OK;
  if (!d_points || !d_dist) return fail(SMCRT_E_INVALID, "scene_distance: NULL points or distances");
  HIP_TRY(hipSetDevice(e->device), "hipSetDevice");
  std::vector<JobSpec> jobs(1);
  jobs[0] = JobSpec{const_cast<smcrt_scene*>(scene), 0, 0, 0, nullptr, nullptr, nullptr};
  const DistSpec dq{d_points, n, (int)accelerated, d_dist, d_owner, d_normals};
  return launch_jobs(e, jobs, nullptr, (hipStream_t)hip_stream, nullptr, &dq);
}

extern "C" smcrt_status smcrt_normalize_fluence(const smcrt_scene* scene, const double* d_raw, double launched,
                                                double* d_phi, void* hip_stream) {
  if (!scene || !d_raw || !d_phi) return fail(SMCRT_E_INVALID, "normalize_fluence: NULL argument");
  if (!(launched > 0)) return fail(SMCRT_E_INVALID, "normalize_fluence: launched must be > 0");
  smcrt_scene* s = const_cast<smcrt_scene*>(scene);
  smcrt_status st = pack(s);
  if (st != SMCRT_OK) return st;
  const SceneHeader* h = reinterpret_cast<const SceneHeader*>(s->blob.data());
  if (!h->has_grid) return fail(SMCRT_E_INVALID, "normalize_fluence: the scene has no grid");
  size_t n = (size_t)h->g_dims[0] * h->g_dims[1] * h->g_dims[2];
  double vol = h->g_d[0] * h->g_d[1] * h->g_d[2];
  HIP_TRY(launch_scale(d_raw, d_phi, n, 1.0 / (launched * vol), (hipStream_t)hip_stream), "scale kernel");
  return SMCRT_OK;
}

// ------------------------------------------------------------------ serving
//
// Continuous batching with device-resident state.  A worker thread admits
// queued requests in arrival order into slots while their device
// footprint fits the budget: each admitted request gets its scene tables,
// grid-build buffers and voxel grid on the device and a packet-id counter
// that persists while it is resident.  The device runs epochs of a fixed
// length of device time: every resident request is a job of one batched
// launch per kernel class; waves first resume the packets the previous
// epoch left in flight, then take new ids, and at the epoch's deadline the
// packets still in flight are written to an HBM slab (their whole state)
// instead of being run to their end.  Between epochs the slab is sorted by
// slot, new requests join, finished ones leave: arrivals never wait for the
// longest packet of an epoch, and the device stays busy.  A request is done
// when all its ids are handed out and none of its packets is in flight.
// Packets are keyed by (seed, packet id, event) and tallies add, so its
// result equals its run alone up to FP64 summation order.  Dry runs (no
// device) keep a packet-chunk scheduler, for admission and cancellation.

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace {

struct Request {
  uint64_t id = 0;
  smcrt_scene* scene = nullptr;
  uint64_t seed = 0, n = 0, next = 0;
  double* fluence = nullptr;
  double* absorbed = nullptr;
  smcrt_tallies* tallies = nullptr;
  uint64_t footprint = 0;
  int state = SMCRT_REQ_QUEUED;
  bool cancel = false;
  double t_submit = 0, t_admit = -1, t_done = -1;
  std::string error;
};

}  // namespace

struct Resident;

struct smcrt_server {
  smcrt_engine* engine = nullptr;  // NULL: dry run (scheduling only)
  smcrt_opts opts;                 // launch options (the engine's, also in a dry run)
  uint64_t budget = 0, used = 0, epoch_packets = 0, min_chunk = 0;
  uint64_t epoch_us = 20000;       // device epochs: length in microseconds of device time
  Resident* res = nullptr;         // device state of a device server
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::map<uint64_t, Request*> all;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  hipStream_t stream = nullptr;
  std::chrono::steady_clock::time_point t0;
  uint64_t epochs = 0, packets_done = 0, in_flight = 0, saved_total = 0;
  double busy_s = 0;
};

static double server_now(const smcrt_server* sv) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - sv->t0).count();
}

// device bytes a request holds while admitted: its outputs, its scene
// tables, the grid buffers of its accelerated region and its voxel grid
// (served requests tally straight into their output grid: no brick grid)
static uint64_t request_footprint(const smcrt_scene* s) {
  const SceneHeader* h = reinterpret_cast<const SceneHeader*>(s->blob.data());
  uint64_t b = s->blob.size() + sizeof(WalkArgs) + sizeof(smcrt_tallies) + 8 * kMaxRegions + 256;
  if (h->has_grid) b += 8ull * h->g_dims[0] * h->g_dims[1] * h->g_dims[2];
  if (h->acc.region >= 0) b += 12ull * ((uint64_t)h->acc.n_cells + 1) + 4ull * h->acc.capacity + 3 * 256;
  if (h->geometry == kGeomVoxel) b += (uint64_t)h->g_dims[0] * h->g_dims[1] * h->g_dims[2] + 256;
  return b;
}

// Dry run (no device): epochs in which every admitted request takes its
// next chunk of packet ids and completes at once.
static void dry_loop(smcrt_server* sv) {
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // admit in arrival order while the budget allows
    while (!sv->queue.empty()) {
      Request* r = sv->queue.front();
      if (r->cancel) {
        sv->queue.pop_front();
        r->state = SMCRT_REQ_CANCELLED;
        r->t_done = server_now(sv);
        sv->cv_done.notify_all();
        continue;
      }
      if (sv->used + r->footprint > sv->budget) break;
      sv->queue.pop_front();
      sv->used += r->footprint;
      r->state = SMCRT_REQ_RUNNING;
      r->t_admit = server_now(sv);
      sv->active.push_back(r);
    }
    if (sv->active.empty()) {
      if (sv->stop) return;
      sv->cv_work.wait(lk);
      continue;
    }
    // one epoch over every admitted request
    std::vector<std::pair<Request*, uint64_t>> taken;
    const uint64_t share = std::max<uint64_t>(sv->min_chunk, sv->epoch_packets / sv->active.size());
    for (Request* r : sv->active) {
      if (r->cancel) continue;
      const uint64_t chunk = std::min<uint64_t>(r->n - r->next, share);
      if (chunk == 0) continue;
      taken.push_back({r, chunk});
    }
    lk.unlock();
    const double t_start = server_now(sv);
    const smcrt_status st = SMCRT_OK;
    std::string err;
    lk.lock();
    sv->busy_s += server_now(sv) - t_start;
    ++sv->epochs;
    for (auto& rc : taken) {
      rc.first->next += rc.second;
      if (st == SMCRT_OK) sv->packets_done += rc.second;
    }
    const double t = server_now(sv);
    std::vector<Request*> keep;
    for (Request* r : sv->active) {
      bool finished = false;
      if (st != SMCRT_OK) {
        r->state = SMCRT_REQ_FAILED;
        r->error = err;
        finished = true;
      } else if (r->cancel) {
        r->state = SMCRT_REQ_CANCELLED;
        finished = true;
      } else if (r->next >= r->n) {
        r->state = SMCRT_REQ_DONE;
        finished = true;
      }
      if (finished) {
        r->t_done = t;
        sv->used -= r->footprint;
      } else {
        keep.push_back(r);
      }
    }
    sv->active.swap(keep);
    sv->cv_done.notify_all();
  }
}

// ---- device servers

namespace {

constexpr int kMaxSlots = 128;

// a resident request and its device allocation: scene tables, the
// accelerated region's grid buffers, the voxel model's region grid
struct Slot {
  Request* r = nullptr;
  char* dev = nullptr;
  size_t acc_off = 0, acc_cb = 0, vox_off = 0, vox_n = 0;
  uint64_t handed = 0;     // packet ids handed out so far
  uint32_t saved = 0;      // packets in flight at the end of the last epoch
  bool draining = false;   // left with packets saved (cancelled): idle for one epoch before reuse
};

}  // namespace

struct Resident {
  Slot slots[kMaxSlots];
  int n_used = 0;  // slots 0..n_used-1 appear in the job table
  // device state (persistent across epochs)
  WalkArgs* d_jobs = nullptr;
  unsigned long long* d_counters = nullptr;  // ids handed out, per slot
  unsigned int* d_resume_next = nullptr;     // resumed packets taken, per slot
  unsigned int* d_counts = nullptr;          // packets saved, per slot
  unsigned int* d_cursors = nullptr;         // scatter cursors, per slot
  unsigned int* d_offsets = nullptr;         // resume segment of each slot
  unsigned int* d_save_count = nullptr;      // records in the save slab
  unsigned char* d_save = nullptr;           // packets saved at the end of an epoch
  unsigned char* d_resume = nullptr;         // the same, sorted by slot, resumed by the next epoch
  uint32_t cap = 0;                          // records each slab holds
  // pinned host mirrors
  WalkArgs* h_jobs = nullptr;
  unsigned long long* h_counters = nullptr;
  unsigned int* h_counts = nullptr;
  unsigned int* h_offsets = nullptr;
  unsigned int* h_save_count = nullptr;
  LaunchCfg cfg[kLaunchClasses];
  uint64_t ticks_per_us = 0;
  unsigned int prev_saved = 0;               // records the last epoch saved
};

static void resident_free(smcrt_server* sv) {
  Resident* R = sv->res;
  if (!R) return;
  for (Slot& sl : R->slots)
    if (sl.dev) (void)hipFree(sl.dev);
  void* dev[] = {R->d_jobs, R->d_counters, R->d_resume_next, R->d_counts, R->d_cursors, R->d_offsets, R->d_save_count,
                 R->d_save, R->d_resume};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  void* host[] = {R->h_jobs, R->h_counters, R->h_counts, R->h_offsets, R->h_save_count};
  for (void* p : host)
    if (p) (void)hipHostFree(p);
  delete R;
  sv->res = nullptr;
}

// Device state of a server: per-slot counters and job table, the two
// packet slabs (one record per lane of every kernel class of an epoch),
// pinned mirrors, the launch shapes and the wall-clock rate.
static smcrt_status resident_init(smcrt_server* sv) {
  Resident* R = new (std::nothrow) Resident();
  if (!R) return fail(SMCRT_E_NOMEM, "server_create: out of host memory");
  sv->res = R;
  smcrt_engine* e = sv->engine;
  uint64_t lanes = 0;
  for (int g = 0; g < kLaunchClasses; ++g) {
    R->cfg[g] = launch_cfg(e, g);
    if (g == kLaunchStaged && e->opts.precision != SMCRT_PREC_F32) continue;
    lanes += (uint64_t)R->cfg[g].grid * R->cfg[g].block;
  }
  if (lanes > 0xffffffffull) return fail(SMCRT_E_INVALID, "server_create: too many resident lanes");
  R->cap = (uint32_t)lanes;
  int khz = 0;
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, e->device), "wall clock rate");
  if (khz <= 0) return fail(SMCRT_E_HIP, "server_create: the device reports no wall-clock rate");
  R->ticks_per_us = (uint64_t)khz / 1000 ? (uint64_t)khz / 1000 : 1;
  HIP_TRY(hipMalloc(&R->d_jobs, sizeof(WalkArgs) * kMaxSlots), "hipMalloc(server jobs)");
  HIP_TRY(hipMalloc(&R->d_counters, sizeof(unsigned long long) * kMaxSlots), "hipMalloc(server counters)");
  HIP_TRY(hipMalloc(&R->d_resume_next, sizeof(unsigned int) * kMaxSlots), "hipMalloc(server resume)");
  HIP_TRY(hipMalloc(&R->d_counts, sizeof(unsigned int) * kMaxSlots), "hipMalloc(server counts)");
  HIP_TRY(hipMalloc(&R->d_cursors, sizeof(unsigned int) * kMaxSlots), "hipMalloc(server cursors)");
  HIP_TRY(hipMalloc(&R->d_offsets, sizeof(unsigned int) * kMaxSlots), "hipMalloc(server offsets)");
  HIP_TRY(hipMalloc(&R->d_save_count, sizeof(unsigned int)), "hipMalloc(server save count)");
  HIP_TRY(hipMalloc(&R->d_save, (size_t)R->cap * kSavedPacketBytes), "hipMalloc(server save slab)");
  HIP_TRY(hipMalloc(&R->d_resume, (size_t)R->cap * kSavedPacketBytes), "hipMalloc(server resume slab)");
  HIP_TRY(hipHostMalloc(&R->h_jobs, sizeof(WalkArgs) * kMaxSlots, hipHostMallocDefault), "hipHostMalloc(jobs)");
  HIP_TRY(hipHostMalloc(&R->h_counters, sizeof(unsigned long long) * kMaxSlots, hipHostMallocDefault), "hipHostMalloc");
  HIP_TRY(hipHostMalloc(&R->h_counts, sizeof(unsigned int) * kMaxSlots, hipHostMallocDefault), "hipHostMalloc");
  HIP_TRY(hipHostMalloc(&R->h_offsets, sizeof(unsigned int) * kMaxSlots, hipHostMallocDefault), "hipHostMalloc");
  HIP_TRY(hipHostMalloc(&R->h_save_count, sizeof(unsigned int), hipHostMallocDefault), "hipHostMalloc");
  std::memset(R->h_counts, 0, sizeof(unsigned int) * kMaxSlots);
  HIP_TRY(launch_zero_u32(R->d_save_count, 1, sv->stream), "zero");
  HIP_TRY(hipStreamSynchronize(sv->stream), "hipStreamSynchronize");
  return SMCRT_OK;
}

// Job record of slot s for the next epoch (an empty one for a free slot)
static void resident_job(smcrt_server* sv, int s, WalkArgs& a) {
  Resident* R = sv->res;
  Slot& sl = R->slots[s];
  std::memset(&a, 0, sizeof(a));
  a.counter = R->d_counters + s;
  a.resume_next = R->d_resume_next + s;
  a.slot = s;
  a.geometry = -1;  // in no launch class
  if (!sl.r) return;
  const Request* r = sl.r;
  const SceneHeader* h = reinterpret_cast<const SceneHeader*>(r->scene->blob.data());
  a.sc = reinterpret_cast<const SceneHeader*>(sl.dev);
  a.pd = reinterpret_cast<const PrimD*>(sl.dev + h->prim_offset_d);
  a.pf = reinterpret_cast<const PrimF*>(sl.dev + h->prim_offset_f);
  a.seed = r->seed;
  a.first = 0;
  a.n = r->cancel ? std::min(sl.handed, r->n) : r->n;  // a cancelled request takes no new ids
  a.fluence = h->has_grid ? r->fluence : nullptr;
  a.absorbed = r->absorbed;
  a.tallies = r->tallies;
  a.acc_region = h->acc.region;
  a.geometry = job_class(sv->opts, h, false);
  if (h->acc.region >= 0) {
    a.acc_offsets = reinterpret_cast<const uint32_t*>(sl.dev + sl.acc_off + 2 * sl.acc_cb);
    a.acc_ids = reinterpret_cast<const uint32_t*>(sl.dev + sl.acc_off + 3 * sl.acc_cb);
    a.acc_rings = reinterpret_cast<const uint32_t*>(sl.dev + sl.acc_off);
    if (h->acc.caps) {
      a.acc_capd = reinterpret_cast<const double*>(sl.dev + h->acc.cap_offset_d);
      a.acc_capf = reinterpret_cast<const float*>(sl.dev + h->acc.cap_offset_f);
    }
  }
  if (sl.vox_n) a.vox = reinterpret_cast<uint8_t*>(sl.dev + sl.vox_off);
  if (!r->cancel && R->h_counts[s] > 0) {
    a.resume = R->d_resume + (size_t)R->h_offsets[s] * kSavedPacketBytes;
    a.resume_n = R->h_counts[s];
  }
}

// Puts request r in free slot s: its tables, grid buffers and voxel grid on
// the device, the grids built, its id counter zeroed.  Synchronous.
static smcrt_status resident_admit(smcrt_server* sv, int s, Request* r) {
  Resident* R = sv->res;
  Slot& sl = R->slots[s];
  const SceneHeader* h = reinterpret_cast<const SceneHeader*>(r->scene->blob.data());
  size_t off = align256(r->scene->blob.size());
  sl.acc_off = sl.acc_cb = sl.vox_off = sl.vox_n = 0;
  if (h->acc.region >= 0) {
    sl.acc_cb = align256(sizeof(uint32_t) * ((size_t)h->acc.n_cells + 1));
    sl.acc_off = off;
    off += 3 * sl.acc_cb + align256(sizeof(uint32_t) * h->acc.capacity);
  }
  if (h->geometry == kGeomVoxel) {
    sl.vox_n = (size_t)h->g_dims[0] * h->g_dims[1] * h->g_dims[2];
    sl.vox_off = off;
    off = align256(off + sl.vox_n);
  }
  HIP_TRY(hipMalloc(&sl.dev, off), "hipMalloc(request tables)");
  sl.r = r;
  sl.handed = 0;
  sl.saved = 0;
  R->h_counts[s] = 0;
  HIP_TRY(hipMemcpy(sl.dev, r->scene->blob.data(), r->scene->blob.size(), hipMemcpyHostToDevice), "upload tables");
  resident_job(sv, s, R->h_jobs[s]);
  HIP_TRY(hipMemcpyAsync(R->d_jobs + s, R->h_jobs + s, sizeof(WalkArgs), hipMemcpyHostToDevice, sv->stream),
          "upload job");
  HIP_TRY(launch_zero_u64(R->d_counters + s, sv->stream), "zero counter");
  if (h->acc.region >= 0) {
    char* ab = sl.dev + sl.acc_off;
    HIP_TRY(launch_accel_build(reinterpret_cast<const SceneHeader*>(sl.dev),
                               reinterpret_cast<const PrimD*>(sl.dev + h->prim_offset_d), h->acc.n_prims, h->acc.n_cells,
                               reinterpret_cast<uint32_t*>(ab), reinterpret_cast<uint32_t*>(ab + sl.acc_cb),
                               reinterpret_cast<uint32_t*>(ab + 2 * sl.acc_cb), reinterpret_cast<uint32_t*>(ab + 3 * sl.acc_cb),
                               sv->stream),
            "accel build");
  }
  if (sl.vox_n)
    HIP_TRY(launch_voxelize(R->d_jobs, s, reinterpret_cast<uint8_t*>(sl.dev + sl.vox_off), sl.vox_n, sv->stream),
            "voxelize");
  HIP_TRY(hipStreamSynchronize(sv->stream), "hipStreamSynchronize(admit)");
  return SMCRT_OK;
}

static void resident_release(smcrt_server* sv, int s) {
  Slot& sl = sv->res->slots[s];
  if (sl.dev) (void)hipFree(sl.dev);
  sl.dev = nullptr;
  sl.r = nullptr;
  sl.draining = sl.saved > 0;
  sl.handed = 0;
  sl.saved = 0;
}

// The next epoch's job table and resume segments (the last epoch's
// counts, in slot order) in the pinned mirrors; has[g]: class g has jobs.
// Under the server's lock.
static void resident_prepare(smcrt_server* sv, bool has[kLaunchClasses]) {
  Resident* R = sv->res;
  unsigned int acc = 0;
  for (int s = 0; s < R->n_used; ++s) {
    R->h_offsets[s] = acc;
    acc += R->h_counts[s];
  }
  for (int g = 0; g < kLaunchClasses; ++g) has[g] = false;
  for (int s = 0; s < R->n_used; ++s) {
    resident_job(sv, s, R->h_jobs[s]);
    const int g = R->h_jobs[s].geometry;
    if (g >= 0 && g < kLaunchClasses) has[g] = true;
  }
}

// One epoch on the device: job table, the previous epoch's packets sorted
// by slot, one deadline-bounded launch per kernel class with jobs, the
// packets not resumed carried over, the new slab counted by slot, counters
// and counts copied back.  Synchronous.
static smcrt_status resident_epoch(smcrt_server* sv, const bool has[kLaunchClasses]) {
  Resident* R = sv->res;
  smcrt_engine* e = sv->engine;
  const hipStream_t q = sv->stream;
  const int n = R->n_used;
  HIP_TRY(hipMemcpyAsync(R->d_jobs, R->h_jobs, sizeof(WalkArgs) * n, hipMemcpyHostToDevice, q), "upload jobs");
  HIP_TRY(hipMemcpyAsync(R->d_offsets, R->h_offsets, sizeof(unsigned int) * n, hipMemcpyHostToDevice, q), "offsets");
  if (R->prev_saved > 0) {
    HIP_TRY(launch_zero_u32(R->d_cursors, n, q), "zero cursors");
    HIP_TRY(launch_saved_scatter(R->d_save, R->d_save_count, R->cap, R->d_offsets, R->d_cursors, R->d_resume, n, q),
            "sort saved packets");
  }
  HIP_TRY(launch_zero_u32(R->d_resume_next, n, q), "zero resume cursors");
  HIP_TRY(launch_zero_u32(R->d_save_count, 1, q), "zero save count");
  BatchArgs B;
  std::memset(&B, 0, sizeof(B));
  B.jobs = R->d_jobs;
  B.n_jobs = n;
  B.refill_min = e->opts.refill_min;
  B.surface_min = e->opts.surface_min;
  B.deadline = sv->epoch_us * R->ticks_per_us;
  B.save = R->d_save;
  B.save_count = R->d_save_count;
  B.save_cap = R->cap;
  for (int g = 0; g < kLaunchClasses; ++g) {
    if (!has[g]) continue;
    B.geometry = g;
    HIP_TRY(launch_walk(e->opts.precision, false, R->cfg[g], B, q), "walk kernel (epoch)");
  }
  HIP_TRY(launch_saved_carry(R->d_jobs, n, R->d_save, R->d_save_count, R->cap, q), "carry saved packets");
  HIP_TRY(launch_zero_u32(R->d_counts, n, q), "zero counts");
  HIP_TRY(launch_saved_count(R->d_save, R->d_save_count, R->cap, R->d_counts, n, q), "count saved packets");
  HIP_TRY(hipMemcpyAsync(R->h_counters, R->d_counters, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, q), "read");
  HIP_TRY(hipMemcpyAsync(R->h_counts, R->d_counts, sizeof(unsigned int) * n, hipMemcpyDeviceToHost, q), "read");
  HIP_TRY(hipMemcpyAsync(R->h_save_count, R->d_save_count, sizeof(unsigned int), hipMemcpyDeviceToHost, q), "read");
  HIP_TRY(hipStreamSynchronize(q), "hipStreamSynchronize(epoch)");
  if (*R->h_save_count > R->cap)
    return fail(SMCRT_E_HIP, "epoch: %u packets in flight, the slab holds %u", *R->h_save_count, R->cap);
  R->prev_saved = *R->h_save_count;
  return SMCRT_OK;
}

static void resident_loop(smcrt_server* sv) {
  Resident* R = sv->res;
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    if (sv->stop)  // shutting down: what runs is cancelled at the end of this epoch
      for (int s = 0; s < R->n_used; ++s)
        if (R->slots[s].r) R->slots[s].r->cancel = true;
    // admit in arrival order while the budget and a slot allow
    while (!sv->queue.empty()) {
      Request* r = sv->queue.front();
      if (r->cancel) {
        sv->queue.pop_front();
        r->state = SMCRT_REQ_CANCELLED;
        r->t_done = server_now(sv);
        sv->cv_done.notify_all();
        continue;
      }
      if (sv->used + r->footprint > sv->budget) break;
      int s = -1;
      for (int k = 0; k < kMaxSlots && s < 0; ++k)
        if (!R->slots[k].r && !R->slots[k].draining) s = k;
      if (s < 0) break;
      sv->queue.pop_front();
      sv->used += r->footprint;
      r->state = SMCRT_REQ_RUNNING;
      r->t_admit = server_now(sv);
      lk.unlock();
      const smcrt_status st = resident_admit(sv, s, r);
      const std::string err = st == SMCRT_OK ? std::string() : std::string(smcrt_last_error());
      lk.lock();
      if (st != SMCRT_OK) {
        resident_release(sv, s);
        R->slots[s].draining = false;
        sv->used -= r->footprint;
        r->state = SMCRT_REQ_FAILED;
        r->error = err;
        r->t_done = server_now(sv);
        sv->cv_done.notify_all();
        continue;
      }
      R->n_used = std::max(R->n_used, s + 1);
    }
    bool any = false, draining = false;
    for (int s = 0; s < R->n_used; ++s) {
      any = any || R->slots[s].r != nullptr;
      draining = draining || R->slots[s].draining;
    }
    if (!any && !draining) {
      R->n_used = 0;
      if (sv->stop) return;
      sv->cv_work.wait(lk);
      continue;
    }
    bool has[kLaunchClasses];
    resident_prepare(sv, has);
    lk.unlock();
    const double t_start = server_now(sv);
    const smcrt_status st = resident_epoch(sv, has);
    const std::string err = st == SMCRT_OK ? std::string() : std::string(smcrt_last_error());
    lk.lock();
    sv->busy_s += server_now(sv) - t_start;
    ++sv->epochs;
    if (st == SMCRT_OK) {
      sv->in_flight = R->prev_saved;
      sv->saved_total += R->prev_saved;
    }
    const double t = server_now(sv);
    for (int s = 0; s < R->n_used; ++s) {
      Slot& sl = R->slots[s];
      if (!sl.r) {
        sl.draining = false;  // its saved packets were neither resumed nor carried: gone
        continue;
      }
      Request* r = sl.r;
      const uint64_t was_done = sl.handed - sl.saved;
      if (st == SMCRT_OK) {
        sl.handed = std::min<uint64_t>(R->h_counters[s], r->n);
        sl.saved = R->h_counts[s];
        r->next = sl.handed;
        sv->packets_done += (sl.handed - sl.saved) - was_done;
      }
      bool finished = true;
      if (st != SMCRT_OK) {
        r->state = SMCRT_REQ_FAILED;
        r->error = err;
      } else if (r->cancel) {
        r->state = SMCRT_REQ_CANCELLED;
      } else if (sl.handed >= r->n && sl.saved == 0) {
        r->state = SMCRT_REQ_DONE;
      } else {
        finished = false;
      }
      if (finished) {
        r->t_done = t;
        sv->used -= r->footprint;
        resident_release(sv, s);
      }
    }
    if (st != SMCRT_OK) {  // a failed epoch leaves no trustworthy packet state
      R->prev_saved = 0;
      for (int s = 0; s < kMaxSlots; ++s) {
        R->slots[s].draining = false;
        R->h_counts[s] = 0;
      }
    }
    sv->cv_done.notify_all();
  }
}

static void server_loop(smcrt_server* sv) {
  if (sv->engine) resident_loop(sv);
  else dry_loop(sv);
}

extern "C" smcrt_status smcrt_server_create(smcrt_server** out, int device, uint64_t hbm_budget_bytes,
                                            uint64_t epoch_packets, const smcrt_opts* opts) {
  if (!out) return fail(SMCRT_E_INVALID, "server_create: out is NULL");
  if (hbm_budget_bytes == 0) return fail(SMCRT_E_INVALID, "server_create: budget must be > 0");
  if (opts) {
    smcrt_status st = check_opts(opts);
    if (st != SMCRT_OK) return st;
  }
  smcrt_server* sv = new (std::nothrow) smcrt_server();
  if (!sv) return fail(SMCRT_E_NOMEM, "server_create: out of host memory");
  sv->budget = hbm_budget_bytes;
  sv->epoch_packets = epoch_packets ? epoch_packets : 2000000;
  sv->min_chunk = std::max<uint64_t>(1, std::min<uint64_t>(10000, sv->epoch_packets));
  sv->t0 = std::chrono::steady_clock::now();
  default_opts(&sv->opts);
  if (opts) sv->opts = *opts;
  if (device >= 0) {
    smcrt_status st = smcrt_engine_create(&sv->engine, device);
    if (st != SMCRT_OK) {
      delete sv;
      return st;
    }
    sv->engine->opts = sv->opts;
    hipError_t e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      smcrt_engine_destroy(sv->engine);
      delete sv;
      return hip_fail(e, "server stream");
    }
    st = resident_init(sv);
    if (st != SMCRT_OK) {
      const std::string msg = smcrt_last_error();
      resident_free(sv);
      (void)hipStreamDestroy(sv->stream);
      smcrt_engine_destroy(sv->engine);
      delete sv;
      return fail(st, "%s", msg.c_str());
    }
  }
  sv->worker = std::thread([sv]() {
    if (sv->engine) (void)hipSetDevice(sv->engine->device);
    server_loop(sv);
  });
  *out = sv;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_server_destroy(smcrt_server* sv) {
  if (!sv) return SMCRT_OK;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
    for (Request* r : sv->queue) r->cancel = true;
  }
  sv->cv_work.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  for (auto& kv : sv->all) delete kv.second;
  if (sv->engine) {
    (void)hipSetDevice(sv->engine->device);
    if (sv->stream) (void)hipStreamSynchronize(sv->stream);
    resident_free(sv);
  }
  if (sv->stream) (void)hipStreamDestroy(sv->stream);
  if (sv->engine) smcrt_engine_destroy(sv->engine);
  delete sv;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_submit(smcrt_server* sv, const smcrt_scene* scene, uint64_t seed, uint64_t n_packets,
                                     double* d_fluence_raw, double* d_absorbed, smcrt_tallies* d_tallies,
                                     uint64_t* out_request) {
  if (!sv || !scene || !out_request) return fail(SMCRT_E_INVALID, "submit: NULL argument");
  if (n_packets == 0) return fail(SMCRT_E_INVALID, "submit: n_packets must be >= 1");
  smcrt_scene* s = const_cast<smcrt_scene*>(scene);
  uint64_t fp;
  {
    std::lock_guard<std::mutex> g(sv->mu);  // the worker packs scenes under this lock's protection too
    smcrt_status st = pack(s);
    if (st != SMCRT_OK) return st;
    if (sv->engine && (!d_absorbed || !d_tallies))
      return fail(SMCRT_E_INVALID, "submit: output buffers missing");
    fp = request_footprint(s);
    if (fp > sv->budget)
      return fail(SMCRT_E_BUDGET, "submit: request needs %llu bytes, budget is %llu", (unsigned long long)fp,
                  (unsigned long long)sv->budget);
    if (sv->stop) return fail(SMCRT_E_STATE, "submit: server is shutting down");
    Request* r = new (std::nothrow) Request();
    if (!r) return fail(SMCRT_E_NOMEM, "submit: out of host memory");
    r->id = sv->next_id++;
    r->scene = s;
    r->seed = seed;
    r->n = n_packets;
    r->fluence = d_fluence_raw;
    r->absorbed = d_absorbed;
    r->tallies = d_tallies;
    r->footprint = fp;
    r->t_submit = server_now(sv);
    sv->all[r->id] = r;
    sv->queue.push_back(r);
    *out_request = r->id;
  }
  sv->cv_work.notify_all();
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_poll(smcrt_server* sv, uint64_t req, int* out_state, double* out_t_submit,
                                   double* out_t_admit, double* out_t_done) {
  if (!sv) return fail(SMCRT_E_INVALID, "poll: NULL server");
  std::lock_guard<std::mutex> g(sv->mu);
  auto it = sv->all.find(req);
  if (it == sv->all.end()) return fail(SMCRT_E_INVALID, "poll: unknown request %llu", (unsigned long long)req);
  const Request* r = it->second;
  if (out_state) *out_state = r->state;
  if (out_t_submit) *out_t_submit = r->t_submit;
  if (out_t_admit) *out_t_admit = r->t_admit;
  if (out_t_done) *out_t_done = r->t_done;
  if (r->state == SMCRT_REQ_FAILED) g_last_error = r->error;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_wait(smcrt_server* sv, uint64_t req, double timeout_s) {
  if (!sv) return fail(SMCRT_E_INVALID, "wait: NULL server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(req);
  if (it == sv->all.end()) return fail(SMCRT_E_INVALID, "wait: unknown request %llu", (unsigned long long)req);
  Request* r = it->second;
  auto done = [r]() { return r->state == SMCRT_REQ_DONE || r->state == SMCRT_REQ_FAILED || r->state == SMCRT_REQ_CANCELLED; };
  if (timeout_s < 0) {
    sv->cv_done.wait(lk, done);
  } else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return fail(SMCRT_E_STATE, "wait: request %llu not finished after %.3f s", (unsigned long long)req, timeout_s);
  }
  if (r->state == SMCRT_REQ_FAILED) return fail(SMCRT_E_HIP, "request failed: %s", r->error.c_str());
  if (r->state == SMCRT_REQ_CANCELLED) return fail(SMCRT_E_CANCELLED, "request %llu was cancelled", (unsigned long long)req);
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_cancel(smcrt_server* sv, uint64_t req) {
  if (!sv) return fail(SMCRT_E_INVALID, "cancel: NULL server");
  {
    std::lock_guard<std::mutex> g(sv->mu);
    auto it = sv->all.find(req);
    if (it == sv->all.end()) return fail(SMCRT_E_INVALID, "cancel: unknown request %llu", (unsigned long long)req);
    it->second->cancel = true;
  }
  sv->cv_work.notify_all();
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_server_set_epoch_us(smcrt_server* sv, uint64_t epoch_us) {
  if (!sv) return fail(SMCRT_E_INVALID, "server_set_epoch_us: NULL server");
  if (epoch_us < 100 || epoch_us > 10000000) return fail(SMCRT_E_INVALID, "server_set_epoch_us: epoch must be 100 us to 10 s");
  std::lock_guard<std::mutex> g(sv->mu);
  sv->epoch_us = epoch_us;
  return SMCRT_OK;
}

extern "C" smcrt_status smcrt_server_stats(smcrt_server* sv, smcrt_server_info* out) {
  if (!sv || !out) return fail(SMCRT_E_INVALID, "server_stats: NULL argument");
  std::lock_guard<std::mutex> g(sv->mu);
  out->epochs = sv->epochs;
  out->packets_done = sv->packets_done;
  out->queued = sv->queue.size();
  out->active = sv->active.size();
  if (sv->res) {
    out->active = 0;
    for (const Slot& sl : sv->res->slots) out->active += sl.r != nullptr;
  }
  out->bytes_in_use = sv->used;
  out->busy_s = sv->busy_s;
  out->uptime_s = server_now(sv);
  out->in_flight = sv->in_flight;
  out->saved_total = sv->saved_total;
  return SMCRT_OK;
}
