// voxel_model.h -- device functions of the voxelised-geometry model, the
// comparison model of Sec. 3: the scene is replaced by the region of each
// fluence-grid voxel centre (voxelize_kernel in voxel.hip), and a packet
// moves from voxel face to voxel face.  Emission, interactions, the random
// stream and the tallies are the SDF walk's own (walk_common.h); only the
// geometry differs:
//   - beyond the grid lies the ambient medium; a packet born outside the
//     grid travels to it unattenuated and untallied, or escapes if it misses;
//   - a face between voxels of equal refractive index is crossed without an
//     event (the region, hence mu_a and mu_s, may still change there);
//   - a face where the index changes, the grid faces included, is an
//     interface event with the axis as normal: Fresnel in FP64, reflection
//     or vector Snell refraction, next event index, variate word 0;
//   - transmission through a grid face is an escape through that face.
#pragma once
#include "walk_common.h"

namespace smcrt {

__device__ __forceinline__ int vox_index(ScP sc, const int v[3]) {
  return v[0] + sc->g_dims[0] * (v[1] + sc->g_dims[1] * v[2]);
}

template <typename T>
__device__ __forceinline__ T comp(const V3<T>& a, int i) {
  return i == 0 ? a.x : (i == 1 ? a.y : a.z);
}
template <typename T>
__device__ __forceinline__ void set_comp(V3<T>& a, int i, T x) {
  if (i == 0) a.x = x;
  else if (i == 1) a.y = x;
  else a.z = x;
}

// escape through grid face `face`; on_grid: the packet is on that face (it
// reached the grid), so it is seen by the escape image
template <typename T, bool TRACE>
__device__ __forceinline__ void escape_face(JobRef a, Packet<T>& pk, Lane& ln, LdsTallies& L, int face, bool on_grid) {
  ScP sc = kptr(a.sc);
  pk.region = sc->n_regions;
  atomicAdd(&L.escaped[face], pk.w);
  atomicAdd(&L.cnt[kCEscapes], 1ull);
  if (on_grid) detect<T>(a, pk, face, (face & 1) ? Tab<T>::g_hi(sc, face >> 1) : Tab<T>::g_lo(sc, face >> 1));
  record<T, TRACE>(a, pk, ln, SMCRT_EV_ESCAPE);
}

// Interface event at the face of axis ax between the packet's medium and
// region r2 (n_regions = ambient).  FP64 Fresnel with the axis as normal.
// Returns true when the packet passed into r2, false when it reflected.
template <typename T, bool TRACE>
__device__ bool voxel_interface(JobRef a, Packet<T>& pk, Lane& ln, LdsTallies& L, int ax, int r2, double n1,
                                double n2) {
  ScP sc = kptr(a.sc);
  pk.k += 1;
  pk.steps = 0;
  atomicAdd(&L.cnt[kCInterfaces], 1ull);
  const U4 rr = philox10(pk.k, (uint32_t)pk.pid, (uint32_t)(pk.pid >> 32), 0u, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
  const double x0 = xi_of<double>(rr.w0);
  V3<double> u = to_d(pk.u);
  const double ua = comp(u, ax);
  const double ci = __builtin_fabs(ua);
  double ct;
  const double R = fresnel(n1, n2, ci, &ct);
  if (x0 < R) {  // specular reflection: the axis component flips
    set_comp(pk.u, ax, -comp(pk.u, ax));
    atomicAdd(&L.cnt[kCReflections], 1ull);
    record<T, TRACE>(a, pk, ln, SMCRT_EV_REFLECT);
    return false;
  }
  const double eta = n1 / n2, sg = ua > 0.0 ? 1.0 : -1.0;
  u = eta * u;
  set_comp(u, ax, comp(u, ax) + (ct - eta * ci) * sg);
  u = (1.0 / __builtin_sqrt(dot(u, u))) * u;
  pk.u = from_d<T>(u);
  set_region(sc, pk, r2);
  atomicAdd(&L.cnt[kCRefractions], 1ull);
  record<T, TRACE>(a, pk, ln, SMCRT_EV_REFRACT);
  return true;
}

// After emission: place the packet in its voxel v, entering the grid from
// outside if it was born there.  Returns false when the packet has ended
// (it missed the grid, or reflected off the grid face it arrived at).
template <typename T, bool TRACE>
__device__ bool enter_grid(JobRef a, Packet<T>& pk, int v[3], Lane& ln, LdsTallies& L) {
  ScP sc = kptr(a.sc);
  const int nr = sc->n_regions;
  const V3<T> p = pk.p, u = pk.u;
  bool inside = true;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (comp(p, i) < Tab<T>::g_lo(sc, i) || comp(p, i) > Tab<T>::g_hi(sc, i)) inside = false;
  int entry = -1;
  if (!inside) {  // slab test against the grid box
    T t0 = T(0), t1 = tinf<T>();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T pi = comp(p, i), ui = comp(u, i), lo = Tab<T>::g_lo(sc, i), hi = Tab<T>::g_hi(sc, i);
      if (ui == T(0)) {
        if (pi < lo || pi > hi) t1 = T(-1);
      } else {
        const T ta = (lo - pi) / ui, tb = (hi - pi) / ui;
        const T tn = tmin(ta, tb), tx = tmax(ta, tb);
        if (tn > t0) {
          t0 = tn;
          entry = i;
        }
        t1 = tmin(t1, tx);
      }
    }
    if (!(t1 > t0) || entry < 0) {  // misses the grid: out through the nearest box face
      int face = 0;
      T best = -tinf<T>();
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T lo = Tab<T>::g_lo(sc, i), hi = Tab<T>::g_hi(sc, i);
        const T c = T(0.5) * (lo + hi), e = tabs(comp(p, i) - c) - T(0.5) * (hi - lo);
        if (e > best) {
          best = e;
          face = 2 * i + (comp(p, i) > c ? 1 : 0);
        }
      }
      escape_face<T, TRACE>(a, pk, ln, L, face, false);
      return false;
    }
    shift(pk, t0);
    set_region(sc, pk, nr);  // in the ambient medium, on the grid face
  }
  // voxel holding the point; on a voxel face, the one the packet moves into
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int n = sc->g_dims[i];
    const T x = (comp(pk.p, i) - Tab<T>::g_lo(sc, i)) / Tab<T>::g_d(sc, i);
    const T fl = floor(x);
    int k = (int)tclamp(fl, T(-1), T(n));
    if (comp(u, i) < T(0) && x == fl) k -= 1;
    if (i == entry) k = comp(u, i) > T(0) ? 0 : n - 1;
    v[i] = k < 0 ? 0 : (k >= n ? n - 1 : k);
  }
  const int r2 = a.vox[vox_index(sc, v)];
  if (entry < 0) {
    set_region(sc, pk, r2);
    return true;
  }
  const double n1 = sc->reg[nr].n, n2 = sc->reg[r2].n;
  if (n1 == n2) {
    set_region(sc, pk, r2);
    return true;
  }
  if (voxel_interface<T, TRACE>(a, pk, ln, L, entry, r2, n1, n2)) return true;
  // reflected off the grid: it leaves through the face it came to
  escape_face<T, TRACE>(a, pk, ln, L, 2 * entry + (comp(pk.u, entry) > T(0) ? 1 : 0), true);
  return false;
}

// One move of the voxel walk: to the exit face of voxel v or to the
// interaction point, whichever is nearer, tallying the piece.  Sets
// pk.state = kInteract when the optical depth runs out.  Returns false when
// the packet has ended (escape or step cap).
template <typename T, bool TRACE>
__device__ bool voxel_step(JobRef a, Packet<T>& pk, int v[3], Lane& ln, LdsTallies& L, int max_steps,
                           uint32_t max_events) {
  ScP sc = kptr(a.sc);
  if (++pk.steps > max_steps || pk.k > max_events) {
    atomicAdd(&L.stalled, pk.w);
    atomicAdd(&L.cnt[kCStalls], 1ull);
    record<T, TRACE>(a, pk, ln, SMCRT_EV_STALL);
    return false;
  }
  ++ln.n_steps;
  T texit = tinf<T>();
  int ax = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T ui = comp(pk.u, i);
    if (ui == T(0)) continue;
    const T face = Tab<T>::g_lo(sc, i) + T(v[i] + (ui > T(0) ? 1 : 0)) * Tab<T>::g_d(sc, i);
    // from the compensated position (FP32: p + pe)
    const T t = tmax(((face - comp(pk.p, i)) - comp(pk.pe, i)) / ui, T(0));
    if (t < texit) {
      texit = t;
      ax = i;
    }
  }
  const int idx = vox_index(sc, v);
  const T s = pk.mut > T(0) ? (T)(pk.tau * (double)pk.inv_mut) : tinf<T>();
  if (s <= texit) {  // interaction inside this voxel
    if (a.fluence != nullptr && s > T(0)) run_add(a.fluence, ln, idx, pk.w * (double)s);
    shift(pk, s);
    pk.tau = 0.0;
    pk.state = kInteract;
    return true;
  }
  if (a.fluence != nullptr && texit > T(0)) run_add(a.fluence, ln, idx, pk.w * (double)texit);
  shift(pk, texit);
  pk.tau -= (double)pk.mut * (double)texit;
  const T ua = comp(pk.u, ax);
  int w2[3] = {v[0], v[1], v[2]};
  w2[ax] += ua > T(0) ? 1 : -1;
  const int face = 2 * ax + (ua > T(0) ? 1 : 0);
  const bool off = w2[ax] < 0 || w2[ax] >= sc->g_dims[ax];
  const int r2 = off ? sc->n_regions : (int)a.vox[vox_index(sc, w2)];
  const double n1 = sc->reg[pk.region].n, n2 = sc->reg[r2].n;
  if (n1 == n2) {
    if (off) {
      escape_face<T, TRACE>(a, pk, ln, L, face, true);
      return false;
    }
    v[0] = w2[0]; v[1] = w2[1]; v[2] = w2[2];
    if (r2 != pk.region) set_region(sc, pk, r2);
    return true;
  }
  if (!voxel_interface<T, TRACE>(a, pk, ln, L, ax, r2, n1, n2)) return true;  // reflected: same voxel
  if (off) {  // transmitted out of the grid
    atomicAdd(&L.escaped[face], pk.w);
    atomicAdd(&L.cnt[kCEscapes], 1ull);
    detect<T>(a, pk, face, (face & 1) ? Tab<T>::g_hi(sc, face >> 1) : Tab<T>::g_lo(sc, face >> 1));
    record<T, TRACE>(a, pk, ln, SMCRT_EV_ESCAPE);
    return false;
  }
  v[0] = w2[0]; v[1] = w2[1]; v[2] = w2[2];
  return true;
}

}  // namespace smcrt
