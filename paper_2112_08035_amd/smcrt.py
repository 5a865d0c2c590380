"""ctypes binding of libsmcrt (include/smcrt.h).

The ``smcrt_*`` functions mirror the C entry points one to one and only
marshal arguments; every step of the walk runs in the HIP kernels of
``libsmcrt.so``.  If the library is missing this module raises: there is no
CPU fallback.  Device buffers are torch CUDA tensors (ROCm); streams are
torch streams.

Convenience layer: :class:`Scene` builds a library scene from a scene
dictionary of :mod:`paper_2112_08035_amd.workloads`, :class:`Engine` owns a
device engine, and :func:`run` / :func:`trace` allocate outputs and return
them.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# another build of the same library (a sanitizer build, say) when SMCRT_LIB names one
LIB_PATH = os.environ.get("SMCRT_LIB") or os.path.join(HERE, "libsmcrt.so")

OK, E_INVALID, E_NOMEM, E_HIP, E_BUDGET, E_CANCELLED, E_STATE = 0, -1, -2, -3, -4, -5, -6
PRIM = {"sphere": 0, "box": 1, "capsule": 2, "cylinder": 3, "torus": 4,
        "cone": 5, "octahedron": 6, "hexprism": 7, "ellipsoid": 8}
OP = {"union": 0, "smooth_union": 1, "intersect": 2, "subtract": 3}
SRC = {"point": 0, "pencil": 1, "disc": 2, "rect": 3}
PREC = {"f32": 0, "f64": 1}
EVENT_TYPES = ["EMIT", "SCATTER", "ABSORB", "KILL", "REFLECT", "REFRACT", "CROSS", "ESCAPE", "STALL"]


class SmcrtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"smcrt status {status}: {msg}")
        self.status = status


class Tallies(C.Structure):
    _fields_ = [("launched", C.c_double), ("escaped_face", C.c_double * 6), ("roulette_gain", C.c_double),
                ("roulette_loss", C.c_double), ("stalled", C.c_double)] + [
        (n, C.c_uint64) for n in ("events", "steps", "interactions", "interfaces", "reflections", "refractions",
                                  "crossings", "advances", "voxel_pieces", "kills", "stalls", "escapes",
                                  "grid_atomics")]


class Event(C.Structure):
    _fields_ = [("event", C.c_uint32), ("type", C.c_uint32), ("region", C.c_int32), ("pad", C.c_int32),
                ("p", C.c_double * 3), ("u", C.c_double * 3), ("w", C.c_double), ("tau", C.c_double)]


class ServerInfo(C.Structure):
    _fields_ = [("epochs", C.c_uint64), ("packets_done", C.c_uint64), ("queued", C.c_uint64), ("active", C.c_uint64),
                ("bytes_in_use", C.c_uint64), ("busy_s", C.c_double), ("uptime_s", C.c_double),
                ("in_flight", C.c_uint64), ("saved_total", C.c_uint64)]


REQ_STATES = ["QUEUED", "RUNNING", "DONE", "FAILED", "CANCELLED"]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("refill_min", C.c_int32), ("surface_min", C.c_int32), ("use_graph", C.c_int32),
                ("tally_layout", C.c_int32), ("no_stage", C.c_int32)]


class OutputsStruct(C.Structure):
    """smcrt_outputs"""
    _fields_ = [("fluence_raw", C.c_void_p), ("absorbed", C.c_void_p), ("tallies", C.c_void_p),
                ("detector", C.c_void_p)]


_lib = None
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_SIGS = {
    "smcrt_last_error": ([], C.c_char_p),
    "smcrt_abi_version": ([], C.c_int),
    "smcrt_scene_create": ([C.POINTER(_vp), C.c_double, C.c_double, C.c_double], C.c_int),
    "smcrt_scene_destroy": ([_vp], C.c_int),
    "smcrt_scene_add_primitive": ([_vp, C.c_int, _dp, C.c_int, C.POINTER(C.c_int32)], C.c_int),
    "smcrt_scene_add_region": ([_vp, C.POINTER(C.c_int32), C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.POINTER(C.c_int32)], C.c_int),
    "smcrt_scene_set_source": ([_vp, C.c_int, _dp, C.c_int], C.c_int),
    "smcrt_scene_set_grid": ([_vp, _dp, _dp, C.POINTER(C.c_int32)], C.c_int),
    "smcrt_scene_set_roulette": ([_vp, C.c_double, C.c_int32], C.c_int),
    "smcrt_scene_set_limits": ([_vp, C.c_int32, C.c_int64], C.c_int),
    "smcrt_scene_set_relaxation": ([_vp, C.c_double], C.c_int),
    "smcrt_scene_set_segment_tracing": ([_vp, C.c_int32], C.c_int),
    "smcrt_scene_set_primitive_placement": ([_vp, C.c_int32, _dp, C.c_double, _dp], C.c_int),
    "smcrt_scene_set_primitive_modifiers": ([_vp, C.c_int32, C.c_double, C.c_double, C.c_double], C.c_int),
    "smcrt_scene_set_primitive_elongation": ([_vp, C.c_int32, _dp], C.c_int),
    "smcrt_scene_set_primitive_bend": ([_vp, C.c_int32, C.c_double], C.c_int),
    "smcrt_scene_set_primitive_displacement": ([_vp, C.c_int32, C.c_double, C.c_double], C.c_int),
    "smcrt_scene_set_primitive_repetition": ([_vp, C.c_int32, _dp, C.POINTER(C.c_int32)], C.c_int),
    "smcrt_scene_set_accel": ([_vp, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "smcrt_scene_set_geometry": ([_vp, C.c_int], C.c_int),
    "smcrt_scene_set_detector": ([_vp, C.c_int, _dp, _dp, C.POINTER(C.c_int32)], C.c_int),
    "smcrt_run_ex": ([_vp, _vp, C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(OutputsStruct), _vp], C.c_int),
    "smcrt_run_ex_static": ([_vp, _vp, C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(OutputsStruct), _vp], C.c_int),
    "smcrt_run_batch_ex": ([_vp, C.c_int, C.POINTER(_vp), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                            C.POINTER(C.c_uint64), C.POINTER(OutputsStruct), _vp], C.c_int),
    "smcrt_scene_info": ([_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _dp, _dp], C.c_int),
    "smcrt_engine_create": ([C.POINTER(_vp), C.c_int], C.c_int),
    "smcrt_engine_destroy": ([_vp], C.c_int),
    "smcrt_engine_get_opts": ([_vp, C.POINTER(Opts)], C.c_int),
    "smcrt_engine_set_opts": ([_vp, C.POINTER(Opts)], C.c_int),
    "smcrt_engine_autotune": ([_vp, _vp, C.c_uint64, C.POINTER(Opts), C.POINTER(C.c_double)], C.c_int),
    "smcrt_engine_autotune_batch": ([_vp, C.c_int, C.POINTER(_vp), C.c_uint64, C.POINTER(Opts), C.POINTER(C.c_double)],
                                    C.c_int),
    "smcrt_run": ([_vp, _vp, C.c_uint64, C.c_uint64, C.c_uint64, _vp, _vp, _vp, _vp], C.c_int),
    "smcrt_run_batch": ([_vp, C.c_int, C.POINTER(_vp), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                         C.POINTER(C.c_uint64), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), _vp], C.c_int),
    "smcrt_normalize_fluence": ([_vp, _vp, C.c_double, _vp, _vp], C.c_int),
    "smcrt_trace": ([_vp, _vp, C.c_uint64, _vp, C.c_int, C.c_int, _vp, _vp, _vp], C.c_int),
    "smcrt_voxelize": ([_vp, _vp, _vp, _vp], C.c_int),
    "smcrt_scene_distance": ([_vp, _vp, _vp, C.c_uint64, C.c_int32, _vp, _vp, _vp, _vp], C.c_int),
    "smcrt_server_create": ([C.POINTER(_vp), C.c_int, C.c_uint64, C.c_uint64, C.POINTER(Opts)], C.c_int),
    "smcrt_server_destroy": ([_vp], C.c_int),
    "smcrt_submit": ([_vp, _vp, C.c_uint64, C.c_uint64, _vp, _vp, _vp, C.POINTER(C.c_uint64)], C.c_int),
    "smcrt_poll": ([_vp, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double),
                    C.POINTER(C.c_double)], C.c_int),
    "smcrt_wait": ([_vp, C.c_uint64, C.c_double], C.c_int),
    "smcrt_cancel": ([_vp, C.c_uint64], C.c_int),
    "smcrt_server_stats": ([_vp, C.POINTER(ServerInfo)], C.c_int),
    "smcrt_server_set_epoch_us": ([_vp, C.c_uint64], C.c_int),
}


def lib():
    """Loads libsmcrt.so (built in-tree by build_lib.py); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2112_08035_amd.build_lib)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(st):
    if st != OK:
        raise SmcrtError(st, lib().smcrt_last_error().decode())


def _darr(vals):
    return (C.c_double * len(vals))(*[float(v) for v in vals])


# ---------------------------------------------------------------- 1:1 ABI

def smcrt_abi_version():
    return lib().smcrt_abi_version()


def smcrt_last_error():
    return lib().smcrt_last_error().decode()


def smcrt_scene_create(n_ambient, delta, pad):
    h = _vp()
    _check(lib().smcrt_scene_create(C.byref(h), n_ambient, delta, pad))
    return h


def smcrt_scene_destroy(scene):
    _check(lib().smcrt_scene_destroy(scene))


def smcrt_scene_add_primitive(scene, kind, params):
    out = C.c_int32()
    _check(lib().smcrt_scene_add_primitive(scene, kind, _darr(params), len(params), C.byref(out)))
    return out.value


def smcrt_scene_set_primitive_placement(scene, prim, rot, scale, trans):
    _check(lib().smcrt_scene_set_primitive_placement(scene, prim, _darr(rot), scale, _darr(trans)))


def smcrt_scene_set_primitive_modifiers(scene, prim, round_r, onion_t, twist_k):
    _check(lib().smcrt_scene_set_primitive_modifiers(scene, prim, round_r, onion_t, twist_k))


def smcrt_scene_set_primitive_bend(scene, prim, bend_k):
    _check(lib().smcrt_scene_set_primitive_bend(scene, prim, bend_k))


def smcrt_scene_set_primitive_elongation(scene, prim, h):
    _check(lib().smcrt_scene_set_primitive_elongation(scene, prim, _darr(h)))


def smcrt_scene_set_primitive_displacement(scene, prim, amplitude, frequency):
    _check(lib().smcrt_scene_set_primitive_displacement(scene, prim, amplitude, frequency))


def smcrt_scene_set_primitive_repetition(scene, prim, spacing, counts):
    _check(lib().smcrt_scene_set_primitive_repetition(scene, prim, _darr(spacing),
                                                      (C.c_int32 * 3)(*[int(c) for c in counts])))


def smcrt_scene_add_region(scene, prims, op, k_cm, mu_a, mu_s, g, n):
    arr = (C.c_int32 * len(prims))(*[int(p) for p in prims])
    out = C.c_int32()
    _check(lib().smcrt_scene_add_region(scene, arr, len(prims), op, k_cm, mu_a, mu_s, g, n, C.byref(out)))
    return out.value


def smcrt_scene_set_source(scene, kind, params):
    _check(lib().smcrt_scene_set_source(scene, kind, _darr(params), len(params)))


def smcrt_scene_set_grid(scene, lo, hi, dims):
    _check(lib().smcrt_scene_set_grid(scene, _darr(lo), _darr(hi), (C.c_int32 * 3)(*[int(d) for d in dims])))


def smcrt_scene_set_roulette(scene, w_threshold, m_survive):
    _check(lib().smcrt_scene_set_roulette(scene, w_threshold, m_survive))


def smcrt_scene_set_limits(scene, max_steps, max_events):
    _check(lib().smcrt_scene_set_limits(scene, max_steps, max_events))


def smcrt_scene_set_relaxation(scene, omega):
    _check(lib().smcrt_scene_set_relaxation(scene, omega))


def smcrt_scene_set_segment_tracing(scene, on):
    _check(lib().smcrt_scene_set_segment_tracing(scene, int(on)))


def smcrt_scene_set_accel(scene, region, cells):
    _check(lib().smcrt_scene_set_accel(scene, region, (C.c_int32 * 3)(*[int(c) for c in cells]) if cells else None))


GEOM = {"sdf": 0, "voxel": 1}


def smcrt_scene_set_geometry(scene, mode):
    _check(lib().smcrt_scene_set_geometry(scene, GEOM[mode] if isinstance(mode, str) else int(mode)))


def smcrt_scene_set_detector(scene, face, lo, hi, dims):
    _check(lib().smcrt_scene_set_detector(scene, int(face), (C.c_double * 2)(*lo), (C.c_double * 2)(*hi),
                                          (C.c_int32 * 2)(*[int(d) for d in dims])))


def smcrt_run_ex(engine, scene, seed, first_packet, n_packets, outputs, stream):
    _check(lib().smcrt_run_ex(engine, scene, seed, first_packet, n_packets, C.byref(outputs), stream))


def smcrt_run_ex_static(engine, scene, seed, first_packet, n_packets, outputs, stream):
    _check(lib().smcrt_run_ex_static(engine, scene, seed, first_packet, n_packets, C.byref(outputs), stream))


def smcrt_run_batch_ex(engine, scenes, seeds, first_packets, n_packets, outputs, stream):
    n = len(scenes)
    arr = (OutputsStruct * n)(*outputs)
    _check(lib().smcrt_run_batch_ex(engine, n, (_vp * n)(*scenes), (C.c_uint64 * n)(*seeds),
                                    (C.c_uint64 * n)(*first_packets) if first_packets is not None else None,
                                    (C.c_uint64 * n)(*n_packets), arr, stream))


def smcrt_scene_info(scene):
    nr, npr = C.c_int32(), C.c_int32()
    lo, hi = (C.c_double * 3)(), (C.c_double * 3)()
    _check(lib().smcrt_scene_info(scene, C.byref(nr), C.byref(npr), lo, hi))
    return nr.value, npr.value, np.array(lo[:]), np.array(hi[:])


def smcrt_engine_create(device):
    h = _vp()
    _check(lib().smcrt_engine_create(C.byref(h), device))
    return h


def smcrt_engine_destroy(engine):
    _check(lib().smcrt_engine_destroy(engine))


def smcrt_engine_get_opts(engine):
    o = Opts()
    _check(lib().smcrt_engine_get_opts(engine, C.byref(o)))
    return o


def smcrt_engine_set_opts(engine, opts):
    _check(lib().smcrt_engine_set_opts(engine, C.byref(opts)))


def smcrt_engine_autotune(engine, scene, n_trial):
    o = Opts()
    rate = C.c_double()
    _check(lib().smcrt_engine_autotune(engine, scene, n_trial, C.byref(o), C.byref(rate)))
    return o, rate.value


def smcrt_engine_autotune_batch(engine, scenes, n_trial):
    o = Opts()
    rate = C.c_double()
    arr = (_vp * len(scenes))(*scenes)
    _check(lib().smcrt_engine_autotune_batch(engine, len(scenes), arr, n_trial, C.byref(o), C.byref(rate)))
    return o, rate.value


def smcrt_run(engine, scene, seed, first_packet, n_packets, d_fluence_raw, d_absorbed, d_tallies, stream):
    _check(lib().smcrt_run(engine, scene, seed, first_packet, n_packets, d_fluence_raw, d_absorbed, d_tallies, stream))


def smcrt_run_batch(engine, scenes, seeds, first_packets, n_packets, d_fluence_raw, d_absorbed, d_tallies, stream):
    n = len(scenes)
    arr = lambda T, v: (T * n)(*v)
    _check(lib().smcrt_run_batch(engine, n, arr(_vp, scenes), arr(C.c_uint64, seeds),
                                 arr(C.c_uint64, first_packets) if first_packets is not None else None,
                                 arr(C.c_uint64, n_packets), arr(_vp, d_fluence_raw), arr(_vp, d_absorbed),
                                 arr(_vp, d_tallies), stream))


def smcrt_normalize_fluence(scene, d_raw, launched, d_phi, stream):
    _check(lib().smcrt_normalize_fluence(scene, d_raw, launched, d_phi, stream))


def smcrt_trace(engine, scene, seed, d_packet_ids, n_ids, max_events, d_out, d_count, stream):
    _check(lib().smcrt_trace(engine, scene, seed, d_packet_ids, n_ids, max_events, d_out, d_count, stream))


def smcrt_voxelize(engine, scene, d_out, stream):
    _check(lib().smcrt_voxelize(engine, scene, d_out, stream))


def smcrt_scene_distance(engine, scene, d_points, n, accelerated, d_dist, d_owner, d_normals, stream):
    _check(lib().smcrt_scene_distance(engine, scene, d_points, n, accelerated, d_dist, d_owner, d_normals, stream))


def smcrt_server_create(device, hbm_budget_bytes, epoch_packets=0, opts=None):
    h = _vp()
    _check(lib().smcrt_server_create(C.byref(h), device, hbm_budget_bytes, epoch_packets,
                                     C.byref(opts) if opts is not None else None))
    return h


def smcrt_server_destroy(server):
    _check(lib().smcrt_server_destroy(server))


def smcrt_submit(server, scene, seed, n_packets, d_fluence_raw, d_absorbed, d_tallies):
    rid = C.c_uint64()
    _check(lib().smcrt_submit(server, scene, seed, n_packets, d_fluence_raw, d_absorbed, d_tallies, C.byref(rid)))
    return rid.value


def smcrt_poll(server, request):
    st, ts, ta, td = C.c_int(), C.c_double(), C.c_double(), C.c_double()
    _check(lib().smcrt_poll(server, request, C.byref(st), C.byref(ts), C.byref(ta), C.byref(td)))
    return REQ_STATES[st.value], ts.value, ta.value, td.value


def smcrt_wait(server, request, timeout_s=-1.0):
    _check(lib().smcrt_wait(server, request, timeout_s))


def smcrt_cancel(server, request):
    _check(lib().smcrt_cancel(server, request))


def smcrt_server_set_epoch_us(server, epoch_us):
    _check(lib().smcrt_server_set_epoch_us(server, int(epoch_us)))


def smcrt_server_stats(server):
    info = ServerInfo()
    _check(lib().smcrt_server_stats(server, C.byref(info)))
    return {k: getattr(info, k) for k, _ in ServerInfo._fields_}


# ---------------------------------------------------------------- helpers

class Scene:
    """A library scene built from a workloads scene dictionary."""

    def __init__(self, desc):
        self.desc = desc
        self.h = smcrt_scene_create(desc["n_ambient"], desc["delta"], desc["pad"])
        ids = []
        for p in desc["prims"]:
            if p["kind"] == "sphere":
                vals = list(p["c"]) + [p["r"]]
            elif p["kind"] == "box":
                vals = list(p["c"]) + list(p["half"])
            elif p["kind"] == "torus":
                vals = list(p["c"]) + list(p["axis"]) + [p["R"], p["r"]]
            elif p["kind"] == "cone":
                vals = list(p["a"]) + list(p["b"]) + [p["ra"], p["rb"]]
            elif p["kind"] == "octahedron":
                vals = list(p["c"]) + [p["s"]]
            elif p["kind"] == "hexprism":
                vals = list(p["c"]) + [p["h"], p["hz"]]
            elif p["kind"] == "ellipsoid":
                vals = list(p["c"]) + list(p["radii"])
            else:
                vals = list(p["a"]) + list(p["b"]) + [p["r"]]
            pid = smcrt_scene_add_primitive(self.h, PRIM[p["kind"]], vals)
            ids.append(pid)
            xf = p.get("transform")
            if xf:
                R = [float(x) for row in xf["R"] for x in row]
                smcrt_scene_set_primitive_placement(self.h, pid, R, float(xf["s"]), [float(x) for x in xf["t"]])
            if p.get("round", 0.0) or p.get("onion", 0.0) or p.get("twist", 0.0):
                smcrt_scene_set_primitive_modifiers(self.h, pid, float(p.get("round", 0.0)),
                                                    float(p.get("onion", 0.0)), float(p.get("twist", 0.0)))
            if p.get("bend", 0.0):
                smcrt_scene_set_primitive_bend(self.h, pid, float(p["bend"]))
            if p.get("elongate"):
                smcrt_scene_set_primitive_elongation(self.h, pid, [float(x) for x in p["elongate"]])
            if p.get("displace"):
                smcrt_scene_set_primitive_displacement(self.h, pid, float(p["displace"]["a"]), float(p["displace"]["f"]))
            if p.get("repeat"):
                smcrt_scene_set_primitive_repetition(self.h, pid, [float(x) for x in p["repeat"]["c"]],
                                                     [int(x) for x in p["repeat"]["n"]])
        for rg in desc["regions"]:
            smcrt_scene_add_region(self.h, [ids[i] for i in rg["prims"]], OP[rg["op"]], rg.get("k", 0.0),
                                   rg["mua"], rg["mus"], rg["g"], rg["n"])
        s = desc["source"]
        if s["kind"] == "point":
            vals = list(s["p"])
        elif s["kind"] == "pencil":
            vals = list(s["p"]) + list(s["u"])
        elif s["kind"] == "disc":
            vals = list(s["c"]) + [s["r"]] + list(s["u"])
        else:
            vals = list(s["c"]) + list(s["half"]) + list(s["u"])
        smcrt_scene_set_source(self.h, SRC[s["kind"]], vals)
        g = desc.get("grid")
        if g:
            smcrt_scene_set_grid(self.h, g["lo"], g["hi"], g["dims"])
            self.dims = tuple(int(d) for d in g["dims"])
        else:
            smcrt_scene_set_grid(self.h, [0, 0, 0], [1, 1, 1], [0, 0, 0])
            self.dims = (0, 0, 0)
        ro = desc["roulette"]
        smcrt_scene_set_roulette(self.h, ro["w_threshold"], ro["m"])
        smcrt_scene_set_limits(self.h, desc["max_steps"], desc["max_events"])
        smcrt_scene_set_segment_tracing(self.h, 0)
        smcrt_scene_set_relaxation(self.h, float(desc.get("relax", 1.0)))
        smcrt_scene_set_segment_tracing(self.h, bool(desc.get("segment", False)))
        if desc.get("accel_cells"):
            # accelerate the union region with the most primitives
            counts = [len(rg["prims"]) if rg["op"] == "union" else 0 for rg in desc["regions"]]
            r = max(range(len(counts)), key=lambda i: counts[i])
            if counts[r] > 1:
                smcrt_scene_set_accel(self.h, r, desc["accel_cells"])
        if desc.get("geometry", "sdf") != "sdf":
            smcrt_scene_set_geometry(self.h, desc["geometry"])
        det = desc.get("detector")
        self.det_dims = (int(det["dims"][0]), int(det["dims"][1])) if det else None
        if det:
            smcrt_scene_set_detector(self.h, det["face"], det["lo"], det["hi"], det["dims"])
        self.n_regions = len(desc["regions"])

    @property
    def n_voxels(self):
        return self.dims[0] * self.dims[1] * self.dims[2]

    def close(self):
        if self.h:
            smcrt_scene_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _torch_device_init():
    """Device memory and streams of this binding come from torch: its HIP
    context must exist before the library first touches the device, or
    torch's own lazy initialisation fails afterwards."""
    import torch
    torch.cuda.init()


class Engine:
    def __init__(self, device=0, **opts):
        self.device = device
        _torch_device_init()
        self.h = smcrt_engine_create(device)
        if opts:
            self.set_opts(**opts)

    def set_opts(self, precision=None, block=None, blocks_per_cu=None, refill_min=None, surface_min=None,
                 use_graph=None, tally_layout=None, no_stage=None):
        o = smcrt_engine_get_opts(self.h)
        if precision is not None:
            o.precision = PREC[precision] if isinstance(precision, str) else int(precision)
        for k, v in (("block", block), ("blocks_per_cu", blocks_per_cu), ("refill_min", refill_min),
                     ("surface_min", surface_min), ("use_graph", use_graph), ("tally_layout", tally_layout),
                     ("no_stage", no_stage)):
            if v is not None:
                setattr(o, k, int(v))
        smcrt_engine_set_opts(self.h, o)

    def autotune(self, scene, n_trial=500_000):
        """Times launch options on the scene -- or, given a list of scenes, on
        one batched launch of them, n_trial packets each -- and keeps the
        fastest; returns (options dict, packets/s of the winner)."""
        if isinstance(scene, (list, tuple)):
            scs = [s if isinstance(s, Scene) else Scene(s) for s in scene]
            _, rate = smcrt_engine_autotune_batch(self.h, [s.h for s in scs], n_trial)
        else:
            sc = scene if isinstance(scene, Scene) else Scene(scene)
            _, rate = smcrt_engine_autotune(self.h, sc.h, n_trial)
        return self.opts(), rate

    def opts(self):
        o = smcrt_engine_get_opts(self.h)
        return {k: getattr(o, k) for k in ("precision", "block", "blocks_per_cu", "refill_min", "surface_min",
                                           "use_graph", "tally_layout", "no_stage")}

    def close(self):
        if self.h:
            smcrt_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Outputs:
    """Device outputs of a run (caller-owned, zeroed, accumulated into)."""

    def __init__(self, scene, device=0, tally=True):
        import torch
        dev = torch.device("cuda", device)
        self.tally = bool(tally) and scene.n_voxels > 0
        self.fluence = torch.zeros(scene.n_voxels if self.tally else 1, dtype=torch.float64, device=dev)
        self.absorbed = torch.zeros(scene.n_regions, dtype=torch.float64, device=dev)
        self.tallies = torch.zeros(C.sizeof(Tallies), dtype=torch.uint8, device=dev)
        self.dims = scene.dims
        self.det_dims = scene.det_dims
        self.detector = (torch.zeros(self.det_dims[0] * self.det_dims[1], dtype=torch.float64, device=dev)
                         if self.det_dims else None)

    def zero_(self):
        self.fluence.zero_()
        self.absorbed.zero_()
        self.tallies.zero_()
        if self.detector is not None:
            self.detector.zero_()
        return self

    def struct(self):
        """The buffers as an smcrt_outputs."""
        f, a, t = self.ptrs()
        d = C.c_void_p(self.detector.data_ptr()) if self.detector is not None else None
        return OutputsStruct(f, a, t, d)

    def ptrs(self):
        f = C.c_void_p(self.fluence.data_ptr()) if self.tally else None
        return f, C.c_void_p(self.absorbed.data_ptr()), C.c_void_p(self.tallies.data_ptr())

    def host(self):
        """Copies to host: dict of numpy arrays and tally values."""
        t = Tallies.from_buffer_copy(bytes(self.tallies.cpu().numpy().tobytes()))
        out = {"launched": t.launched, "escaped_face": np.array(t.escaped_face[:]),
               "roulette_gain": t.roulette_gain, "roulette_loss": t.roulette_loss, "stalled": t.stalled}
        for name, _ in Tallies._fields_[5:]:
            out[name] = int(getattr(t, name))
        out["absorbed"] = self.absorbed.cpu().numpy()
        nx, ny, nz = self.dims
        out["fluence_raw"] = self.fluence.cpu().numpy().reshape(nz, ny, nx) if self.tally else None
        if self.detector is not None:
            out["image"] = self.detector.cpu().numpy().reshape(self.det_dims[1], self.det_dims[0])
        return out


def launch(engine, scene, seed, n, first=0, outputs=None, stream=None):
    """Queues one run on the stream; returns the Outputs (not synchronised)."""
    out = outputs if outputs is not None else Outputs(scene, engine.device)
    smcrt_run_ex(engine.h, scene.h, seed, first, n, out.struct(), _stream_ptr(stream))
    return out


def launch_batch(engine, scenes, seeds, n_packets, firsts=None, outputs=None, stream=None):
    """Queues one batched run (one persistent launch for all jobs); returns
    the list of Outputs (not synchronised)."""
    outs = outputs if outputs is not None else [Outputs(sc, engine.device) for sc in scenes]
    smcrt_run_batch_ex(engine.h, [sc.h for sc in scenes], list(seeds), list(firsts) if firsts is not None else None,
                       list(n_packets), [o.struct() for o in outs], _stream_ptr(stream))
    return outs


def run_batch(descs, seeds, n_packets, engine=None, precision="f32", firsts=None):
    """Runs several scenes in one launch; returns host copies per job."""
    import torch
    eng = engine if engine is not None else Engine(0)
    eng.set_opts(precision=precision)
    scenes = [d if isinstance(d, Scene) else Scene(d) for d in descs]
    outs = launch_batch(eng, scenes, seeds, n_packets, firsts)
    torch.cuda.synchronize()
    return [o.host() for o in outs]


def run(desc, seed, n, first=0, engine=None, precision="f32", tally=True, **opts):
    """Runs packets [first, first + n) of a scene dictionary on the GPU and
    returns host copies of the tallies; tally=False runs without the
    fluence tally (fluence_raw is None)."""
    import torch
    eng = engine if engine is not None else Engine(0)
    eng.set_opts(precision=precision, **opts)
    sc = desc if isinstance(desc, Scene) else Scene(desc)
    out = launch(eng, sc, seed, n, first, outputs=Outputs(sc, eng.device, tally=tally))
    torch.cuda.synchronize()
    return out.host()


def trace(desc, seed, pids, max_events=50, engine=None, precision="f32"):
    """Event records of the given packets: list (per packet) of dicts."""
    import torch
    eng = engine if engine is not None else Engine(0)
    eng.set_opts(precision=precision)
    sc = desc if isinstance(desc, Scene) else Scene(desc)
    dev = torch.device("cuda", eng.device)
    ids = torch.tensor(np.asarray(pids, dtype=np.uint64).view(np.int64), device=dev)
    n = len(pids)
    out = torch.zeros(n * max_events * C.sizeof(Event), dtype=torch.uint8, device=dev)
    cnt = torch.zeros(n, dtype=torch.int32, device=dev)
    smcrt_trace(eng.h, sc.h, seed, C.c_void_p(ids.data_ptr()), n, max_events, C.c_void_p(out.data_ptr()),
                C.c_void_p(cnt.data_ptr()), _stream_ptr(None))
    torch.cuda.synchronize()
    raw = out.cpu().numpy().tobytes()
    counts = cnt.cpu().numpy()
    res = []
    sz = C.sizeof(Event)
    for i in range(n):
        evs = []
        for j in range(int(counts[i])):
            e = Event.from_buffer_copy(raw[(i * max_events + j) * sz:(i * max_events + j + 1) * sz])
            evs.append({"event": e.event, "type": EVENT_TYPES[e.type], "region": e.region, "p": np.array(e.p[:]),
                        "u": np.array(e.u[:]), "w": e.w, "tau": e.tau})
        res.append(evs)
    return res


def voxelize(desc, engine=None):
    """Region of every voxel centre of the scene's grid from the device
    (-1 = ambient), shape (nz, ny, nx)."""
    import torch
    eng = engine if engine is not None else Engine(0)
    sc = desc if isinstance(desc, Scene) else Scene(desc)
    out = torch.empty(sc.n_voxels, dtype=torch.uint8, device=torch.device("cuda", eng.device))
    smcrt_voxelize(eng.h, sc.h, C.c_void_p(out.data_ptr()), _stream_ptr(None))
    torch.cuda.synchronize()
    v = out.cpu().numpy().astype(np.int8)
    v[v == sc.n_regions] = -1
    return v.reshape(sc.dims[2], sc.dims[1], sc.dims[0])


def distance(desc, points, engine=None, precision="f64", accelerated=False, normals=False):
    """Every region's SDF at the points (array-like, shape (n, 3)) from the
    device, and each point's owning region (-1 = ambient): returns
    (distances (n, n_regions), owners (n,)) as host arrays, and with
    normals=True also every region's FP64 numerical normal (n, n_regions, 3)."""
    import torch
    eng = engine if engine is not None else Engine(0)
    eng.set_opts(precision=precision)
    sc = desc if isinstance(desc, Scene) else Scene(desc)
    dev = torch.device("cuda", eng.device)
    pts = torch.as_tensor(np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)).to(dev)
    n = pts.shape[0]
    dist = torch.empty((n, sc.n_regions), dtype=torch.float64, device=dev)
    own = torch.empty(n, dtype=torch.int32, device=dev)
    nrm = torch.empty((n, sc.n_regions, 3), dtype=torch.float64, device=dev) if normals else None
    smcrt_scene_distance(eng.h, sc.h, C.c_void_p(pts.data_ptr()), n, 1 if accelerated else 0,
                         C.c_void_p(dist.data_ptr()), C.c_void_p(own.data_ptr()),
                         C.c_void_p(nrm.data_ptr()) if normals else None, _stream_ptr(None))
    torch.cuda.synchronize()
    o = own.cpu().numpy().astype(np.int64)
    o[o == sc.n_regions] = -1
    if normals:
        return dist.cpu().numpy(), o, nrm.cpu().numpy()
    return dist.cpu().numpy(), o


class Server:
    """Continuous-batching request server (smcrt_server_*).  device=-1 runs
    the scheduler alone (no device work)."""

    def __init__(self, device=0, hbm_budget_bytes=32 << 30, epoch_packets=0, epoch_us=0, **opts):
        o = None
        if opts:
            o = Opts()
            o.precision, o.block, o.blocks_per_cu, o.refill_min, o.surface_min = 0, 256, 0, 4, 8
            for k, v in opts.items():
                setattr(o, k, PREC[v] if k == "precision" and isinstance(v, str) else int(v))
        self.device = device
        if device >= 0:
            _torch_device_init()
        self.h = smcrt_server_create(device, hbm_budget_bytes, epoch_packets, o)
        if epoch_us:
            smcrt_server_set_epoch_us(self.h, epoch_us)
        self._keep = {}

    def submit(self, scene, seed, n_packets, outputs=None):
        """Queues a request; returns (request id, Outputs or None)."""
        sc = scene if isinstance(scene, Scene) else Scene(scene)
        if self.device >= 0:
            out = outputs if outputs is not None else Outputs(sc, self.device)
            f, a, t = out.ptrs()
        else:
            out, f, a, t = None, None, None, None
        rid = smcrt_submit(self.h, sc.h, seed, n_packets, f, a, t)
        self._keep[rid] = (sc, out)
        return rid, out

    def poll(self, rid):
        return smcrt_poll(self.h, rid)

    def wait(self, rid, timeout_s=-1.0):
        smcrt_wait(self.h, rid, timeout_s)

    def cancel(self, rid):
        smcrt_cancel(self.h, rid)

    def stats(self):
        return smcrt_server_stats(self.h)

    def close(self):
        if self.h:
            smcrt_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
