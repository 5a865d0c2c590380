// walk.hip -- the persistent photon-packet walk through an SDF scene on
// gfx950 (McMillan, Bruce & Dholakia 2021, Sec. 2.3), one packet per lane.
//
// Each lane owns a packet: emission (Sec. 3.1 sources, Eq. 1 free path),
// sphere-tracing steps over every region SDF (Sec. 2.3, Fig. 3), the
// interface step in FP64 (Fresnel, numerical normals; Sec. 1 and Sec. 2.3),
// interactions (implicit capture, Henyey-Greenstein, roulette), and the
// path-length fluence tally (Sec. 3.1, rectangular bins).  When its packet
// ends the lane takes the next packet id from a global counter, so the grid
// is sized to the machine, not to the packet count.
//
// T is the transport type (float or double): positions, directions, step
// lengths, the SDFs of the stepping loop and the transcendentals.  The
// interface step, remaining optical depth, weights, absorbed energy and
// tallies are FP64 in both.  Steps may be over-relaxed (a multiple of the
// surface distance, checked at the next evaluation; Sec. 5).
//
// Divergence control: lanes that reach a surface wait until surface_min
// lanes of the wave are there (or nothing else can move), so the long FP64
// interface step runs with many lanes on; dead lanes wait for refill_min
// before a wave emits.
//
// Tally: a lane keeps the straight path since its last tally pending and
// credits it through the voxel grid (a register-only DDA) before an
// interaction, an interface event or the packet's end.  Consecutive pieces
// in the same voxel (across steps, events and even packets) merge into one
// run; each run is staged in the wave's LDS stage, which is drained as
// full-wave FP64 atomics.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "voxel_model.h"
#include "walk_common.h"

namespace smcrt {

// The packet is within delta of a surface.  FP64 throughout: nearest
// surface, numerical normal, the hit where the ray meets the surface, a
// probe across it for the medium ahead, then cross, reflect or refract.
// Sets pk.state to kTransport or kInteract.
template <typename T, bool TRACE, bool XF>
__device__ void surface(JobRef a, Packet<T>& pk, Lane& ln, LdsTallies& L) {
  ScP sc = kptr(a.sc);
  V3<double> p = to_d(pk.p);
  if constexpr (sizeof(T) == 4) p = p + to_d(pk.pe);   // the position's compensated sum
  const V3<double> u = to_d(pk.u);
  const int nr = sc->n_regions;
  int j = 0;
  double dj = region_dist<double, XF>(a, 0, p);
  for (int r = 1; r < nr; ++r) {
    const double d = region_dist<double, XF>(a, r, p);
    if (__builtin_fabs(d) < __builtin_fabs(dj)) {
      dj = d;
      j = r;
    }
  }
  const double h = sc->h_normal, off = sc->offset;
  const V3<double> n0 = region_normal<XF>(a, j, p, h);
  const double c0 = dot(u, n0);
  double t_ray = 0.0;
  V3<double> ps;
  if (__builtin_fabs(c0) >= sc->snap_cos) {
    t_ray = -dj / c0;
    ps = p + t_ray * u;
  } else {
    ps = p - dj * n0;
  }
  const V3<double> nrm = region_normal<XF>(a, j, ps, h);
  const double c = dot(u, nrm);
  const double sg = c > 0.0 ? 1.0 : -1.0;
  const V3<double> q = ps + (sg * off) * nrm;
  const int r2 = (c == 0.0) ? pk.region : region_of<double, XF>(a, q);
  RegRef R1 = sc->reg[pk.region];
  double tau = pk.tau;
  const double s_rem = R1.mut > 0.0 ? tau / R1.mut : __builtin_inf();
  if (r2 == pk.region) {
    // no change of medium ahead: advance 2*delta along the ray
    atomicAdd(&L.cnt[kCAdvances], 1ull);
    if (s_rem <= off) {
      advance(pk, (T)s_rem);
      pk.tau = 0.0;
      pk.state = kInteract;
      return;
    }
    advance(pk, (T)off);
    pk.tau = tau - R1.mut * off;
    pk.state = kTransport;
    return;
  }
  if (t_ray > 0.0) {
    if (s_rem <= t_ray) {
      advance(pk, (T)s_rem);
      pk.tau = 0.0;
      pk.state = kInteract;
      return;
    }
    advance(pk, (T)t_ray);
    tau -= R1.mut * t_ray;
  }
  // the position jumps or the direction changes below: credit the straight
  // path up to the surface first
  flush_tally<T>(a, pk, ln);
  pk.k += 1;
  pk.steps = 0;
  pk.pd = T(-1);
  atomicAdd(&L.cnt[kCInterfaces], 1ull);
  pk.tau = tau;
  pk.state = kTransport;
  const double n1 = R1.n, n2 = sc->reg[r2].n;
  if (n1 == n2) {  // index matched: cross undeflected
    set_position(pk, q);
    set_region(sc, pk, r2);
    atomicAdd(&L.cnt[kCCrossings], 1ull);
    record<T, TRACE>(a, pk, ln, SMCRT_EV_CROSS);
    return;
  }
  const U4 rr = philox10(pk.k, (uint32_t)pk.pid, (uint32_t)(pk.pid >> 32), 0u, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
  const double x0 = xi_of<double>(rr.w0);
  const double ci = __builtin_fabs(c), eta = n1 / n2;
  double ctr;
  const double R = fresnel(n1, n2, ci, &ctr);
  V3<double> v;
  if (x0 < R) {  // specular reflection, back on the incident side
    v = u - (2.0 * c) * nrm;
    set_position(pk, ps - (sg * off) * nrm);
    v = (1.0 / __builtin_sqrt(dot(v, v))) * v;
    pk.u = from_d<T>(v);
    atomicAdd(&L.cnt[kCReflections], 1ull);
    record<T, TRACE>(a, pk, ln, SMCRT_EV_REFLECT);
  } else {  // refraction (vector Snell's law) into the far medium
    v = eta * u + ((ctr - eta * ci) * sg) * nrm;
    v = (1.0 / __builtin_sqrt(dot(v, v))) * v;
    pk.u = from_d<T>(v);
    set_position(pk, q);
    set_region(sc, pk, r2);
    atomicAdd(&L.cnt[kCRefractions], 1ull);
    record<T, TRACE>(a, pk, ln, SMCRT_EV_REFRACT);
  }
}

// The persistent walk over a table of jobs (scene tables, seed, packet
// range, outputs).  Each wave works on one job at a time, so the job's
// tables are wave uniform and come through the scalar cache; waves start
// spread over the jobs in proportion to their count and, when their job's
// packets are all handed out and their lanes have drained, flush their sums
// into that job's outputs and move on to the next job with packets left.
// GEOM selects the geometry model: sphere tracing through the SDFs, or the
// voxel walk of the voxelised comparison model.  XF adds the path of placed,
// modified and further-shape primitives.  The launch takes only the jobs of
// its (GEOM, XF) class.  4 waves per SIMD in FP32 (3 in FP64) keep the
// walk's state in registers.
//
// STAGE (FP32, scenes whose accelerated region is plain capsules): the
// workgroup is 16 waves, one per SIMD slot of a CU, that work on one job
// together.  It copies the job's capsule records into an LDS table once per
// job, so the grid queries of the step loop -- a gather of a few capsules
// per lane per step -- read LDS instead of global memory; the waves meet at
// a barrier when the job is drained, and the workgroup takes the next job
// and its table together.
//
// EPOCH (resident serving): the launch stops at B.deadline, saving the
// packets in flight, and resumes the jobs' saved packets before taking new
// ids.  A separate instantiation: the save and resume paths cost registers
// the plain walk does not spend.
//
// SEG (kLaunchSegment jobs): every evaluation also bounds the way along the
// ray to each region's surface (segment tracing), and a step runs to the
// nearest such bound less delta when that is longer than the distance.
template <typename T, bool TRACE, int GEOM, bool XF, bool STAGE, bool EPOCH, bool SEG>
__global__ void __launch_bounds__(STAGE ? 1024 : 256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 3)))
walk_kernel(const WalkArgs* __restrict__ job_table, BatchArgs B) {
  static_assert(!STAGE || (sizeof(T) == 4 && GEOM == kGeomSdf && !XF && !TRACE), "staged capsules: FP32 SDF walks");
  static_assert(!EPOCH || !TRACE, "epochs are for runs, not traces");
  static_assert(!SEG || (GEOM == kGeomSdf && !XF && !STAGE), "segment tracing: plain SDF walks");
  constexpr int kWaves = STAGE ? 16 : 4;
  const SMCRT_K WalkArgs* jobs = kptr(job_table);
  __shared__ LdsTallies Lw[kWaves];
  __shared__ WaveStage Sw[kWaves];
  LdsCaps caps_lds = nullptr;
  F4* caps_fill = nullptr;
  int* wg_job = nullptr;
  uint64_t* wg_t0 = nullptr;
  if constexpr (STAGE) {
    __shared__ F4 s_caps[2 * kStageCaps];
    __shared__ int s_job;
    __shared__ uint64_t s_t0;
    caps_lds = (LdsCaps)s_caps;
    caps_fill = s_caps;
    wg_job = &s_job;
    wg_t0 = &s_t0;
  }
  const int lane = lane_id();
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index in the block (wave uniform)
  LdsTallies& L = Lw[wib];
  if (lane == 0) {
    Sw[wib].n = 0;
    for (int r = 0; r < kMaxRegions; ++r) L.absorbed[r] = 0.0;
    for (int f = 0; f < 6; ++f) L.escaped[f] = 0.0;
    for (int c = 0; c < 16; ++c) L.cnt[c] = 0ull;
    L.gain = L.loss = L.stalled = 0.0;
  }
  __threadfence_block();

  Lane ln;
  ln.stage = &Sw[wib];
  ln.run.v = -1;
  ln.run.sum = 0.0;
  ln.abs_sum = 0.0;
  ln.abs_region = -1;
  ln.n_steps = ln.n_inter = ln.n_pieces = ln.n_atomics = 0;
  ln.rec = nullptr;
  ln.n_rec = 0;

  // resident serving: a launch with a deadline stops when the device wall
  // clock has run deadline ticks past its start (the workgroup's start in
  // the staged kernel, so that its waves agree), saving the packets still
  // in flight for the next epoch
  uint64_t t0 = 0;
  bool stop = false;
  int iter = 0;
  if constexpr (EPOCH && !STAGE) t0 = __builtin_amdgcn_s_memrealtime();

  // First jobs, XCD-aware: workgroups go to the 8 XCDs in turn (block b to
  // XCD b mod 8), and each XCD has its own L2.  The jobs are split into 8
  // runs of consecutive jobs, one per XCD, and every workgroup of an XCD
  // starts at the first job of its run; a job that runs out sends its
  // workgroups on to the next one (pick_job scans forward).  So an XCD's L2
  // holds the grid lists and tables of about one job at a time instead of
  // a slice of every job's.
  const int first_job = (int)(((long)(blockIdx.x & 7) * B.n_jobs) / 8);
  int cur = 0;
  if constexpr (STAGE) {
    // the workgroup's first job, then its table
    if (wib == 0) {
      const int j = pick_job(jobs, B, first_job);
      if (lane == 0) {
        *wg_job = j;
        *wg_t0 = __builtin_amdgcn_s_memrealtime();
      }
    }
    __syncthreads();
    t0 = *wg_t0;
    cur = *wg_job;
    if (cur < 0) return;  // every wave of the workgroup leaves together
    if (!stage_caps(jobs[cur], caps_fill)) caps_lds = nullptr;
    __syncthreads();
  } else if constexpr (!TRACE) {
    cur = pick_job(jobs, B, first_job);
    if (cur < 0) return;
  }
  Packet<T> pk;
  pk.pend = T(0);  // lanes that never get a packet have nothing to credit
  int vx[3] = {0, 0, 0};  // voxel model: the packet's voxel
  bool live = false;

  // outer loop over jobs, inner loop over that job's packets: within the
  // inner loop the job is fixed, so its fields (a noalias read-only kernel
  // argument) and the scene scalars below stay in registers
  for (;;) {
    JobRef a = jobs[cur];
    ScP sc = kptr(a.sc);
    const int nr = sc->n_regions;
    const T delta = Tab<T>::delta(sc);
    const int max_steps = sc->max_steps;
    const uint32_t max_events = (uint32_t)sc->max_events;
    bool exhausted = false;     // wave uniform: no packet of this job left to take
    bool resumed_all = false;   // wave uniform: no saved packet of this job left to resume

    if constexpr (TRACE) {
      const int id = blockIdx.x * blockDim.x + threadIdx.x;
      exhausted = true;
      if (id < a.n_trace) {
        ln.rec = reinterpret_cast<smcrt_event*>(a.trace_out) + (size_t)id * a.max_records;
        pk.pid = a.trace_ids[id];
        live = true;
        emit<T, TRACE, XF>(a, pk, ln, L);
        if constexpr (GEOM == kGeomVoxel) live = enter_grid<T, TRACE>(a, pk, vx, ln, L);
      }
    }

    for (;;) {
      // ---- end of a resident-serving epoch: save the packets in flight
      if constexpr (EPOCH) {
        if (!stop && (++iter & 15) == 0 && __builtin_amdgcn_s_memrealtime() - t0 > B.deadline) stop = true;
        if (stop) {
          save_live<T>(B, a, live, pk, vx, lane);
          live = false;
          exhausted = true;
          break;
        }
      }

      // ---- refill dead lanes: packets saved by the previous epoch first,
      // then new ids from the job's packet counter
      if constexpr (!TRACE) {
        const uint64_t dmask = __ballot(!live);
        const int ndead = __popcll(dmask);
        if (!exhausted && ndead > 0 && (ndead >= B.refill_min || ndead == __popcll(__ballot(1)))) {
          const int leader = __ffsll((unsigned long long)dmask) - 1;
          const int rank = __popcll(dmask & ((1ull << lane) - 1ull));
          int rtake = 0;
          if (EPOCH && a.resume_n > 0 && !resumed_all) {
            unsigned int rb = 0;
            if (lane == leader) rb = atomicAdd(a.resume_next, (unsigned int)ndead);
            rb = __shfl(rb, leader);
            rtake = rb < a.resume_n ? (int)min((unsigned int)ndead, a.resume_n - rb) : 0;
            if (rtake < ndead) resumed_all = true;
            if (!live && rank < rtake) {
              load_saved<T>(a, rb + (unsigned int)rank, pk, vx);
              live = true;
            }
          }
          const int rest = ndead - rtake;
          if (rest > 0) {
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(a.counter, (unsigned long long)rest);
            base = __shfl(base, leader);
            if (base + (uint64_t)rest >= a.n) exhausted = true;
            if (!live && rank >= rtake) {
              const uint64_t id = base + (uint64_t)(rank - rtake);
              if (id < a.n) {
                pk.pid = a.first + id;
                live = true;
                emit<T, TRACE, XF>(a, pk, ln, L);
                if constexpr (GEOM == kGeomVoxel) live = enter_grid<T, TRACE>(a, pk, vx, ln, L);
              }
            }
          }
        }
      }
      const uint64_t lmask = __ballot(live);
      if (lmask == 0ull) {
        if (exhausted) break;
        continue;
      }

      // ---- one voxel move (voxelised model)
      if constexpr (GEOM == kGeomVoxel) {
        if (live && pk.state == kTransport && !voxel_step<T, TRACE>(a, pk, vx, ln, L, max_steps, max_events)) live = false;
      }

      // ---- free-flight reuse: the distance evaluated at the last step's
      // start, less the path since, bounds the distance to every surface;
      // an interaction inside that ball (inside a region, so inside the
      // volume) is the one an evaluation would give, so none is made.
      // Margin: delta, plus per reuse 4 units in the last place of the
      // position for the rounding of the moves
      bool reused = false;
      if (GEOM == kGeomSdf && live && pk.state == kTransport && pk.safe > T(0) && pk.region < nr &&
          pk.links < kReuseLinks) {
        const T s = pk.mut > T(0) ? (T)(pk.tau * (double)pk.inv_mut) : tinf<T>();
        const T pmax = tmax(tabs(pk.p.x), tmax(tabs(pk.p.y), tabs(pk.p.z)));
        const T ulp4 = sizeof(T) == 4 ? T(0x1p-21) : T(0x1p-50);
        if (s <= pk.safe - delta - T(pk.links + 1) * pmax * ulp4) {
          advance(pk, s);
          pk.tau = 0.0;
          pk.state = kInteract;
          pk.safe -= s;
          ++pk.links;
          reused = true;
        }
      }

      // ---- one sphere-tracing step (Sec. 2.3)
      if (GEOM == kGeomSdf && live && pk.state == kTransport && !reused) {
        pk.safe = T(-1);
        if (++pk.steps > max_steps || pk.k > max_events) {
          atomicAdd(&L.stalled, pk.w);
          atomicAdd(&L.cnt[kCStalls], 1ull);
          record<T, TRACE>(a, pk, ln, SMCRT_EV_STALL);
          live = false;
        } else {
          ++ln.n_steps;
          T dmin = tinf<T>(), tseg = tinf<T>();
          if constexpr (SEG) {
            const T err = Tab<T>::seg_err(sc);
            for (int r = 0; r < nr; ++r) {
              T tb;
              dmin = tmin(dmin, tabs(region_seg<T, XF>(a, r, pk.p, pk.u, err, &tb)));
              tseg = tmin(tseg, tb);
            }
          } else {
            for (int r = 0; r < nr; ++r) dmin = tmin(dmin, tabs(region_dist<T, XF>(a, r, pk.p, caps_lds)));
          }
          int face;
          const bool outside = outside_volume<T>(sc, pk.p, &face);
          bool rejected = false;
          if (pk.pl < T(0)) {
            // check of an over-relaxed step (Sec. 5): the open balls of
            // radius pd at its start and dmin at its end hold no surface;
            // unless they cover the step with a margin of delta it goes back
            // to the plain step of pd, and this evaluation is spent
            const T len = -pk.pl;
            if (pk.pd + dmin >= len + delta) {
              pk.pl = len;
            } else {
              rejected = true;
              step_along(pk, pk.pd - len);
              pk.pl = pk.pd;
            }
          }
          if (rejected) {
            // the next evaluation starts from the plain step's end
          } else if (outside) {  // outside the simulation volume
            atomicAdd(&L.escaped[face], pk.w);
            atomicAdd(&L.cnt[kCEscapes], 1ull);
            detect<T>(a, pk, face, Tab<T>::bb_c(sc, face >> 1) + ((face & 1) ? Tab<T>::bb_h(sc, face >> 1) : -Tab<T>::bb_h(sc, face >> 1)));
            record<T, TRACE>(a, pk, ln, SMCRT_EV_ESCAPE);
            live = false;
          } else {
            const T s = pk.mut > T(0) ? (T)(pk.tau * (double)pk.inv_mut) : tinf<T>();
            // segment tracing: a step may run to the nearest bound along the
            // ray less delta, or delta past the volume's boundary when that
            // comes first
            T seg = dmin;
            if constexpr (SEG) {
              if (tseg - delta > dmin) seg = tmax(dmin, tmin(tseg - delta, volume_exit<T>(sc, pk.p, pk.u) + delta));
            }
            if (s <= dmin) {  // the optical depth runs out before any surface
              advance(pk, s);
              pk.tau = 0.0;
              pk.state = kInteract;
              if (pk.region < nr) {  // the ball of radius dmin about the step's start holds no surface
                pk.safe = dmin - s;
                pk.links = 0;
              }
            } else if (dmin < delta) {
              pk.state = kSurface;
            } else if (SEG && seg > dmin && s <= seg) {
              // segment tracing: the interaction point lies on the free
              // segment ahead, where plain steps would reach it; no free
              // ball about it is known
              advance(pk, s);
              pk.tau = 0.0;
              pk.state = kInteract;
            } else {
              // a step of dmin, or an over-relaxed one of omega * dmin when it
              // would pass its check were the surface a plane met at the
              // angle the previous step saw (its distance falls by
              // (pd - dmin)/pl per unit length): dmin + dmin - omega (pd -
              // dmin) dmin / pl >= omega dmin + delta, times pl > 0
              const T om = Tab<T>::relax(sc);
              const bool rel = om > T(1) && pk.pd >= T(0) &&
                               dmin * (Tab<T>::relax_k(sc) * pk.pl - om * (pk.pd - dmin)) >= delta * pk.pl &&
                               om * dmin < s;
              T len = rel ? om * dmin : dmin;
              bool skip = false;
              if (pk.region == nr) {
                // ambient skip, when the boxes' margin of delta/2 covers
                // the rounding of the box test and of the move: 4 units in
                // the last place of the largest coordinate plus the skip
                const T tf = ambient_free<T>(sc, nr, pk.p, pk.u, delta);
                const T pmax = tmax(tabs(pk.p.x), tmax(tabs(pk.p.y), tabs(pk.p.z)));
                const T ulp4 = sizeof(T) == 4 ? T(0x1p-21) : T(0x1p-50);
                if (tf > len && tf >= seg && T(0.5) * delta >= ulp4 * (pmax + tf)) {
                  len = tf;
                  skip = true;
                }
              }
              const bool segment = !skip && seg > len;
              if (segment) len = seg;
              const T moved = step_along(pk, len);
              pk.pd = skip || segment ? T(-1) : dmin;
              pk.pl = rel && !skip ? -moved : moved;
            }
          }
        }
      }

      // ---- interface steps, gathered
      if constexpr (GEOM == kGeomSdf) {
        const uint64_t smask = __ballot(live && pk.state == kSurface);
        const int nsurf = __popcll(smask);
        if (nsurf > 0 && (nsurf >= B.surface_min || nsurf == __popcll(__ballot(live)))) {
          if (live && pk.state == kSurface) surface<T, TRACE, XF>(a, pk, ln, L);
        }
      }

      // ---- tally: lanes whose packet ended or is about to scatter credit
      // their straight path since the last event to the grid, together
      if constexpr (GEOM == kGeomSdf) {
        if (pk.pend > T(0) && (!live || pk.state == kInteract)) flush_tally<T>(a, pk, ln);
      }

      // ---- interactions
      if (live && pk.state == kInteract) {
        pk.state = kTransport;
        if (!interact<T, TRACE>(a, pk, ln, L)) live = false;
      }

      // ---- grid additions staged this iteration, as full-wave atomics.
      // Last in the iteration: one counter tracks a wave's vector loads and
      // its atomics in issue order, so the first per-lane table load after
      // a drain (the region's coefficients in the interaction) waits until
      // every drained atomic has completed at the L2.  Issued here, they
      // complete while the next iteration's step runs.
      if (a.fluence != nullptr) stage_drain(a.fluence, *ln.stage, kDrain, lane);
    }

    if constexpr (TRACE) {
      const int id = blockIdx.x * blockDim.x + threadIdx.x;
      if (id < a.n_trace) a.trace_count[id] = ln.n_rec < a.max_records ? ln.n_rec : a.max_records;
      flush_wave(a, ln, L, lane);
      break;
    } else if constexpr (STAGE) {
      // job drained by this wave: hand in its sums; once every wave is done
      // with the job (and its table), the workgroup takes the next one
      flush_wave(a, ln, L, lane);
      __syncthreads();
      if (wib == 0) {
        const bool late = EPOCH && __builtin_amdgcn_s_memrealtime() - t0 > B.deadline;
        const int j = late ? -1 : pick_job(jobs, B, cur + 1);
        if (lane == 0) *wg_job = j;
      }
      __syncthreads();
      cur = *wg_job;
      if (cur < 0) break;
      caps_lds = (LdsCaps)caps_fill;
      if (!stage_caps(jobs[cur], caps_fill)) caps_lds = nullptr;
      __syncthreads();
    } else {
      // job drained by this wave (or the epoch ended): hand in its sums,
      // take the next job
      flush_wave(a, ln, L, lane);
      if (stop) break;
      cur = pick_job(jobs, B, cur + 1);
      if (cur < 0) break;
    }
  }
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

__global__ void scale_kernel(const double* __restrict__ in, double* __restrict__ out, size_t n, double s) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = in[i] * s;
}

template <int GEOM, bool XF, bool SEG = false>
static void launch_geom(int precision, bool trace, dim3 grid, dim3 block, const BatchArgs& args, hipStream_t stream) {
  const bool epoch = args.deadline != 0;
  if (precision == 1) {
    if (trace) hipLaunchKernelGGL((walk_kernel<double, true, GEOM, XF, false, false, SEG>), grid, block, 0, stream, args.jobs, args);
    else if (epoch) hipLaunchKernelGGL((walk_kernel<double, false, GEOM, XF, false, true, SEG>), grid, block, 0, stream, args.jobs, args);
    else hipLaunchKernelGGL((walk_kernel<double, false, GEOM, XF, false, false, SEG>), grid, block, 0, stream, args.jobs, args);
  } else {
    if (trace) hipLaunchKernelGGL((walk_kernel<float, true, GEOM, XF, false, false, SEG>), grid, block, 0, stream, args.jobs, args);
    else if (epoch) hipLaunchKernelGGL((walk_kernel<float, false, GEOM, XF, false, true, SEG>), grid, block, 0, stream, args.jobs, args);
    else hipLaunchKernelGGL((walk_kernel<float, false, GEOM, XF, false, false, SEG>), grid, block, 0, stream, args.jobs, args);
  }
}

// args.geometry is the launch class: the geometry model plus kLaunchXf when
// the jobs' scenes have placed or modified primitives
hipError_t launch_walk(int precision, bool trace, const LaunchCfg& cfg, const BatchArgs& args, hipStream_t stream) {
  if (!args.jobs || args.n_jobs < 1 || (trace && args.n_jobs != 1)) return hipErrorInvalidValue;
  if (args.refill_min < 1 || args.refill_min > 64 || args.surface_min < 1 || args.surface_min > 64) return hipErrorInvalidValue;
  if (args.geometry < 0 || args.geometry >= kLaunchClasses) return hipErrorInvalidValue;
  if (args.geometry == kLaunchStaged) {
    // FP32 staged-capsule walk: workgroups of 16 waves, no trace variant
    if (precision != 0 || trace || cfg.block != 1024 || cfg.grid < 1) return hipErrorInvalidConfiguration;
    if (args.deadline)
      hipLaunchKernelGGL((walk_kernel<float, false, kGeomSdf, false, true, true, false>), dim3(cfg.grid), dim3(1024), 0, stream,
                         args.jobs, args);
    else
      hipLaunchKernelGGL((walk_kernel<float, false, kGeomSdf, false, true, false, false>), dim3(cfg.grid), dim3(1024), 0, stream,
                         args.jobs, args);
    return hipGetLastError();
  }
  if (cfg.block < 64 || cfg.block > 256 || cfg.block % 64 || cfg.grid < 1) return hipErrorInvalidConfiguration;
  dim3 grid(cfg.grid), block(cfg.block);
  switch (args.geometry) {
    case kGeomSdf: launch_geom<kGeomSdf, false>(precision, trace, grid, block, args, stream); break;
    case kGeomVoxel: launch_geom<kGeomVoxel, false>(precision, trace, grid, block, args, stream); break;
    case kGeomSdf + kLaunchXf: launch_geom<kGeomSdf, true>(precision, trace, grid, block, args, stream); break;
    case kLaunchSegment: launch_geom<kGeomSdf, false, true>(precision, trace, grid, block, args, stream); break;
    default: launch_geom<kGeomVoxel, true>(precision, trace, grid, block, args, stream); break;
  }
  return hipGetLastError();
}

__global__ void zero_u64_n_kernel(unsigned long long* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

hipError_t launch_zero_u64_n(unsigned long long* p, int n, hipStream_t stream) {
  if (!p || n < 1) return hipErrorInvalidValue;
  const int blocks = (n + 255) / 256;
  hipLaunchKernelGGL(zero_u64_n_kernel, dim3(blocks < 1024 ? blocks : 1024), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

__global__ void zero_f64_kernel(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

// F (x fastest, nx*ny*nz) += S (2x2x2 bricks)
__global__ void brick_add_kernel(const double* __restrict__ S, double* __restrict__ F, int nx, int ny, int nz) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % (size_t)nx), y = (int)((i / (size_t)nx) % (size_t)ny), z = (int)(i / ((size_t)nx * ny));
    F[i] += S[brick_index(x, y, z, nx, ny)];
  }
}

hipError_t launch_zero_f64(double* p, size_t n, hipStream_t stream) {
  if (!p || n == 0) return hipErrorInvalidValue;
  const size_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(zero_f64_kernel, dim3(blocks < 4096 ? (unsigned)blocks : 4096u), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_brick_add(const double* S, double* F, int nx, int ny, int nz, hipStream_t stream) {
  if (!S || !F || nx < 1 || ny < 1 || nz < 1) return hipErrorInvalidValue;
  const size_t n = (size_t)nx * ny * nz, blocks = (n + 255) / 256;
  hipLaunchKernelGGL(brick_add_kernel, dim3(blocks < 4096 ? (unsigned)blocks : 4096u), dim3(256), 0, stream, S, F, nx, ny, nz);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t stream) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_scale(const double* in, double* out, size_t n, double scale, hipStream_t stream) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, in, out, n, scale);
  return hipGetLastError();
}

template <int GEOM, bool XF, bool SEG = false>
static hipError_t occupancy(int* n, int precision, int block) {
  return precision == 1
             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(n, walk_kernel<double, false, GEOM, XF, false, false, SEG>, block, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(n, walk_kernel<float, false, GEOM, XF, false, false, SEG>, block, 0);
}

int walk_max_blocks_per_cu(int precision, int block, int launch_class) {
  int n = 0;
  hipError_t e;
  if (launch_class == kLaunchStaged) {
    if (precision != 0 || block != 1024) return 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, walk_kernel<float, false, kGeomSdf, false, true, false, false>, 1024, 0);
    return e == hipSuccess ? n : 0;
  }
  switch (launch_class) {
    case kGeomSdf: e = occupancy<kGeomSdf, false>(&n, precision, block); break;
    case kGeomVoxel: e = occupancy<kGeomVoxel, false>(&n, precision, block); break;
    case kGeomSdf + kLaunchXf: e = occupancy<kGeomSdf, true>(&n, precision, block); break;
    case kLaunchSegment: e = occupancy<kGeomSdf, false, true>(&n, precision, block); break;
    default: e = occupancy<kGeomVoxel, true>(&n, precision, block); break;
  }
  return e == hipSuccess ? n : 0;
}

}  // namespace smcrt