"""ctypes wrapper of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
import this module.  It reads the scene dictionaries of
``paper_2112_08035_amd.workloads`` (pure input data) and marshals them into
the oracle's own C structs; it shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import build as _build

PRIM_KINDS = {"sphere": 0, "box": 1, "capsule": 2, "cylinder": 3, "torus": 4,
              "cone": 5, "octahedron": 6, "hexprism": 7, "ellipsoid": 8}
OPS = {"union": 0, "smooth_union": 1, "intersect": 2, "subtract": 3}
SRC_KINDS = {"point": 0, "pencil": 1, "disc": 2, "rect": 3}
EVENT_TYPES = ["EMIT", "SCATTER", "ABSORB", "KILL", "REFLECT", "REFRACT", "CROSS", "ESCAPE", "STALL"]


class Prim(C.Structure):
    _fields_ = [("kind", C.c_int32), ("flags", C.c_int32), ("p", C.c_double * 8),
                ("rot", C.c_double * 9), ("t", C.c_double * 3), ("s", C.c_double),
                ("round_r", C.c_double), ("onion_t", C.c_double),
                ("twist_k", C.c_double), ("twist_rho", C.c_double), ("twist_zlo", C.c_double),
                ("twist_zhi", C.c_double), ("elong", C.c_double * 3), ("disp_a", C.c_double),
                ("disp_f", C.c_double), ("rep_c", C.c_double * 3), ("rep_n", C.c_int32 * 3), ("pad", C.c_int32),
                ("rep_gap", C.c_double)]


class Region(C.Structure):
    _fields_ = [("first_prim", C.c_int32), ("n_prims", C.c_int32), ("op", C.c_int32), ("pad", C.c_int32),
                ("k", C.c_double), ("mua", C.c_double), ("mus", C.c_double), ("g", C.c_double),
                ("n", C.c_double), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3)]


class Scene(C.Structure):
    _fields_ = [("n_prims", C.c_int32), ("n_regions", C.c_int32),
                ("prims", C.POINTER(Prim)), ("regions", C.POINTER(Region)),
                ("n_ambient", C.c_double), ("delta", C.c_double),
                ("bb_lo", C.c_double * 3), ("bb_hi", C.c_double * 3),
                ("g_lo", C.c_double * 3), ("g_hi", C.c_double * 3), ("g_dims", C.c_int32 * 3),
                ("src_kind", C.c_int32), ("src", C.c_double * 8),
                ("w_threshold", C.c_double), ("m_survive", C.c_int32), ("max_steps", C.c_int32),
                ("max_events", C.c_int64),
                ("det_face", C.c_int32), ("det_dims", C.c_int32 * 2),
                ("det_lo", C.c_double * 2), ("det_hi", C.c_double * 2),
                ("relax", C.c_double), ("reuse", C.c_int32), ("skip", C.c_int32),
                ("segment", C.c_int32), ("pad_segment", C.c_int32)]


class Tallies(C.Structure):
    _fields_ = [("launched", C.c_double), ("escaped_face", C.c_double * 6), ("roulette_gain", C.c_double),
                ("roulette_loss", C.c_double), ("stalled", C.c_double)] + [
        (n, C.c_uint64) for n in ("events", "steps", "interactions", "interfaces", "reflections",
                                  "refractions", "crossings", "advances", "voxel_segments", "kills",
                                  "stalls", "escapes")]


class Event(C.Structure):
    _fields_ = [("event", C.c_uint32), ("type", C.c_uint32), ("region", C.c_int32), ("pad", C.c_int32),
                ("p", C.c_double * 3), ("u", C.c_double * 3), ("w", C.c_double), ("tau", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _build.is_stale():
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_xi.argtypes = [C.c_uint32]
        L.orc_xi.restype = C.c_double
        L.orc_prim_sdf.argtypes = [C.POINTER(Prim), dp]
        L.orc_prim_sdf.restype = C.c_double
        L.orc_smooth_union.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_smooth_union.restype = C.c_double
        L.orc_region_sdf.argtypes = [C.POINTER(Scene), C.c_int, dp]
        L.orc_region_sdf.restype = C.c_double
        L.orc_region_of.argtypes = [C.POINTER(Scene), dp]
        L.orc_region_of.restype = C.c_int
        L.orc_region_normal.argtypes = [C.POINTER(Scene), C.c_int, dp, C.c_double, dp]
        L.orc_box_sdf.argtypes = [dp, dp, dp]
        L.orc_box_sdf.restype = C.c_double
        L.orc_fresnel.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_fresnel.restype = C.c_double
        L.orc_hg_cos.argtypes = [C.c_double, C.c_double]
        L.orc_hg_cos.restype = C.c_double
        L.orc_rotate.argtypes = [dp, C.c_double, C.c_double]
        L.orc_tally_segment.argtypes = [C.POINTER(Scene), dp, dp, C.c_double, dp]
        L.orc_tally_segment.restype = C.c_int64
        L.orc_run.argtypes = [C.POINTER(Scene), C.c_uint64, C.c_uint64, C.c_uint64, C.c_int, dp, dp,
                              C.POINTER(Tallies)]
        L.orc_run.restype = C.c_int
        L.orc_trace.argtypes = [C.POINTER(Scene), C.c_uint64, C.c_uint64, C.c_int, C.POINTER(Event)]
        L.orc_trace.restype = C.c_int
        L.orc_voxelize.argtypes = [C.POINTER(Scene), C.POINTER(C.c_int8)]
        L.orc_run_voxel.argtypes = L.orc_run.argtypes
        L.orc_run_voxel.restype = C.c_int
        L.orc_run_ex.argtypes = [C.POINTER(Scene), C.c_uint64, C.c_uint64, C.c_uint64, C.c_int, C.c_int,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(Tallies)]
        L.orc_run_ex.restype = C.c_int
        L.orc_trace_voxel.argtypes = L.orc_trace.argtypes
        L.orc_trace_voxel.restype = C.c_int
        L.orc_segment_bound.argtypes = [C.POINTER(Scene), C.c_int, dp, dp]
        L.orc_segment_bound.restype = C.c_double
        _lib = L
    return _lib


def _d3(v):
    return (C.c_double * 3)(*[float(x) for x in v])


def modified_box(p):
    """Box of one copy of the modified shape in the primitive's frame: its
    local box grown by the elongation per axis and by rounding, shell and
    displacement amplitude on every side"""
    lo, hi = local_aabb(p)
    h = np.asarray(p.get("elongate", [0.0, 0.0, 0.0]), float)
    g = float(p.get("round", 0.0)) + float(p.get("onion", 0.0)) + float(p.get("displace", {}).get("a", 0.0))
    return lo - h - g, hi + h + g


def turn_k(p):
    """Turn rate of a twisted (about z, by k z) or bent (about z, by k x)
    primitive, 0 for neither"""
    return float(p.get("twist", 0.0)) or float(p.get("bend", 0.0))


def twist_cylinder(p):
    """Bounding cylinder about the local z axis of a twisted or bent
    primitive (its modified box; a turn about z keeps the distance from the
    axis): radius 1.001 x the largest distance of that box from the axis,
    z range the box's grown by 0.1 % of its length at each end."""
    lo, hi = modified_box(p)
    rho = max(math.hypot(x, y) for x in (lo[0], hi[0]) for y in (lo[1], hi[1]))
    m = 1e-3 * (hi[2] - lo[2])
    return 1.001 * rho, lo[2] - m, hi[2] + m


def copy_box(p):
    """Box of one copy in the primitive's frame: the modified box, or the
    twist's or bend's bounding cylinder's box"""
    if turn_k(p) != 0.0:
        rho, zlo, zhi = twist_cylinder(p)
        return np.array([-rho, -rho, zlo]), np.array([rho, rho, zhi])
    return modified_box(p)


def repetition_gap(p):
    """Smallest distance from a copy's box to a face of its cell that another
    copy lies behind; raises if a copy does not fit its cell"""
    rep = p["repeat"]
    lo, hi = copy_box(p)
    gap = math.inf
    for a in range(3):
        if int(rep["n"][a]) > 1:
            gap = min(gap, 0.5 * float(rep["c"][a]) - max(abs(lo[a]), abs(hi[a])))
    if not gap > 0:
        raise ValueError("repeated copies must fit their cells")
    return gap


def prim_struct(p):
    s = Prim()
    s.kind = PRIM_KINDS[p["kind"]]
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
    for i, v in enumerate(vals):
        s.p[i] = float(v)
    flags = 0
    xf = p.get("transform")
    R, t, sc = np.eye(3), np.zeros(3), 1.0
    if xf:
        flags |= 1
        R, t, sc = np.asarray(xf["R"], float).reshape(3, 3), np.asarray(xf["t"], float), float(xf["s"])
    s.rot = (C.c_double * 9)(*R.ravel())
    s.t = (C.c_double * 3)(*t)
    s.s = sc
    s.round_r = float(p.get("round", 0.0))
    s.onion_t = float(p.get("onion", 0.0))
    if p.get("twist", 0.0) != 0.0 and p.get("bend", 0.0) != 0.0:
        raise ValueError("a primitive is either twisted or bent")
    if turn_k(p) != 0.0:
        flags |= 2 | (8 if p.get("bend", 0.0) != 0.0 else 0)
        s.twist_k = turn_k(p)
        s.twist_rho, s.twist_zlo, s.twist_zhi = twist_cylinder(p)
    s.elong = (C.c_double * 3)(*[float(x) for x in p.get("elongate", [0.0, 0.0, 0.0])])
    disp = p.get("displace")
    if disp:
        s.disp_a, s.disp_f = float(disp["a"]), float(disp["f"])
    rep = p.get("repeat")
    if rep and any(int(n) > 1 for n in rep["n"]):
        flags |= 4
        s.rep_c = (C.c_double * 3)(*[float(x) for x in rep["c"]])
        s.rep_n = (C.c_int32 * 3)(*[int(x) for x in rep["n"]])
        s.rep_gap = repetition_gap(p)
    else:
        s.rep_c = (C.c_double * 3)(1.0, 1.0, 1.0)
        s.rep_n = (C.c_int32 * 3)(1, 1, 1)
    s.flags = flags
    return s


def prim_aabb(p):
    """Conservative world box of a primitive: the box of one copy (grown by
    elongation, rounding, shell and displacement, or the twist's bounding
    cylinder's box), over the repeated array, with the 8 corners placed in
    the world."""
    lo, hi = copy_box(p)
    rep = p.get("repeat")
    if rep:
        ext = np.array([0.5 * (int(n) - 1) * float(c) for n, c in zip(rep["n"], rep["c"])])
        lo, hi = lo - ext, hi + ext
    xf = p.get("transform")
    if not xf:
        return lo, hi
    R, t, sc = np.asarray(xf["R"], float).reshape(3, 3), np.asarray(xf["t"], float), float(xf["s"])
    corners = np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])])
    w = sc * corners @ R.T + t
    return w.min(axis=0), w.max(axis=0)


def local_aabb(p):
    """Conservative box of a primitive in its own frame: sphere c -/+ r, box
    c -/+ half, capsule and cylinder the end points' box grown by r, torus
    with unit axis e: c -/+ (R sqrt(1 - e_i^2) + r) per axis (the ring's
    box grown by the tube radius)."""
    if p["kind"] == "sphere":
        c, r = np.array(p["c"], float), float(p["r"])
        return c - r, c + r
    if p["kind"] == "box":
        c, h = np.array(p["c"], float), np.array(p["half"], float)
        return c - h, c + h
    if p["kind"] == "torus":
        c, e = np.array(p["c"], float), np.array(p["axis"], float)
        e = e / np.linalg.norm(e)
        ext = float(p["R"]) * np.sqrt(np.maximum(1.0 - e * e, 0.0)) + float(p["r"])
        return c - ext, c + ext
    if p["kind"] == "cone":   # the end points' box grown by the larger radius
        a, b = np.array(p["a"], float), np.array(p["b"], float)
        r = max(float(p["ra"]), float(p["rb"]))
        return np.minimum(a, b) - r, np.maximum(a, b) + r
    if p["kind"] == "octahedron":
        c, sz = np.array(p["c"], float), float(p["s"])
        return c - sz, c + sz
    if p["kind"] == "hexprism":   # circumradius 2h/sqrt(3) in x and y
        c = np.array(p["c"], float)
        e = np.array([2.0 * float(p["h"]) / math.sqrt(3.0), float(p["h"]), float(p["hz"])])
        return c - e, c + e
    if p["kind"] == "ellipsoid":
        c, r = np.array(p["c"], float), np.array(p["radii"], float)
        return c - r, c + r
    a, b, r = np.array(p["a"], float), np.array(p["b"], float), float(p["r"])
    return np.minimum(a, b) - r, np.maximum(a, b) + r


def source_points(src):
    if src["kind"] in ("point", "pencil"):
        return [np.array(src["p"], float)]
    if src["kind"] == "disc":
        c, r = np.array(src["c"], float), float(src["r"])
        return [c + np.array([-r, -r, 0.0]), c + np.array([r, r, 0.0])]
    c, h = np.array(src["c"], float), src["half"]
    return [c + np.array([-h[0], -h[1], 0.0]), c + np.array([h[0], h[1], 0.0])]


def bounding_box(scene):
    """Simulation volume (Sec. 2.3): box around every SDF and the source's
    emission points, padded by scene["pad"] on every side."""
    los, his = zip(*[prim_aabb(p) for p in scene["prims"]])
    pts = source_points(scene["source"])
    lo = np.minimum(np.min(los, axis=0), np.min(pts, axis=0)) - scene["pad"]
    hi = np.maximum(np.max(his, axis=0), np.max(pts, axis=0)) + scene["pad"]
    return lo, hi


class CScene:
    """Keeps the C arrays alive beside the struct."""

    def __init__(self, scene):
        prims = [prim_struct(p) for p in scene["prims"]]
        self.prims = (Prim * len(prims))(*prims)
        regs = []
        order = []
        for rg in scene["regions"]:
            r = Region()
            r.first_prim = len(order)
            r.n_prims = len(rg["prims"])
            order.extend(rg["prims"])
            r.op = OPS[rg["op"]]
            r.k = float(rg.get("k", 0.0))
            r.mua, r.mus, r.g, r.n = (float(rg[x]) for x in ("mua", "mus", "g", "n"))
            # ambient skip: the region's surface lies in its primitives'
            # boxes; a smooth union reaches at most k/4 beyond them
            los, his = zip(*[prim_aabb(scene["prims"][i]) for i in rg["prims"]])
            grow = (r.k if rg["op"] == "smooth_union" else 0.0) + 0.5 * float(scene["delta"])
            r.box_lo = _d3(np.min(los, axis=0) - grow)
            r.box_hi = _d3(np.max(his, axis=0) + grow)
            regs.append(r)
        # region primitive lists are stored contiguously in region order
        self.prims = (Prim * len(order))(*[prims[i] for i in order])
        self.regions = (Region * len(regs))(*regs)
        s = Scene()
        s.n_prims = len(order)
        s.n_regions = len(regs)
        s.prims = C.cast(self.prims, C.POINTER(Prim))
        s.regions = C.cast(self.regions, C.POINTER(Region))
        s.n_ambient = float(scene["n_ambient"])
        s.delta = float(scene["delta"])
        lo, hi = bounding_box(scene)
        s.bb_lo, s.bb_hi = _d3(lo), _d3(hi)
        g = scene.get("grid")
        if g:
            s.g_lo, s.g_hi = _d3(g["lo"]), _d3(g["hi"])
            s.g_dims = (C.c_int32 * 3)(*[int(x) for x in g["dims"]])
        else:
            s.g_dims = (C.c_int32 * 3)(0, 0, 0)
        src = scene["source"]
        s.src_kind = SRC_KINDS[src["kind"]]
        if src["kind"] == "point":
            vals = list(src["p"])
        elif src["kind"] == "pencil":
            vals = list(src["p"]) + list(src["u"])
        elif src["kind"] == "disc":
            vals = list(src["c"]) + [src["r"]] + list(src["u"])
        else:
            vals = list(src["c"]) + list(src["half"]) + list(src["u"])
        for i, v in enumerate(vals):
            s.src[i] = float(v)
        ro = scene["roulette"]
        s.w_threshold = float(ro["w_threshold"])
        s.m_survive = int(ro["m"])
        s.max_steps = int(scene["max_steps"])
        s.max_events = int(scene["max_events"])
        s.relax = float(scene.get("relax", 1.0))
        # the plain Sec. 2.3 march unless the scene asks for the kernels'
        # shortcuts (used by tests that compare SDF evaluation counts)
        s.reuse = 1 if scene.get("reuse", False) else 0
        s.skip = 1 if scene.get("ambient_skip", False) else 0
        s.segment = 1 if scene.get("segment", False) else 0
        det = scene.get("detector")
        if det:
            s.det_face = int(det["face"])
            s.det_dims = (C.c_int32 * 2)(*[int(x) for x in det["dims"]])
            s.det_lo, s.det_hi = (C.c_double * 2)(*det["lo"]), (C.c_double * 2)(*det["hi"])
        self.s = s
        self.bbox = (lo, hi)

    @property
    def ref(self):
        return C.byref(self.s)


def grid_dims(scene):
    g = scene.get("grid")
    return tuple(int(x) for x in g["dims"]) if g else (0, 0, 0)


def tallies_dict(t):
    d = {"launched": t.launched, "escaped_face": np.array(t.escaped_face[:]),
         "roulette_gain": t.roulette_gain, "roulette_loss": t.roulette_loss, "stalled": t.stalled}
    for name, _ in Tallies._fields_[5:]:
        d[name] = int(getattr(t, name))
    return d


def run(scene, seed, n, first=0, threads=0, with_grid=True, voxel=False):
    """Runs packets [first, first + n).  Returns a dict with the raw
    fluence F (nz, ny, nx), absorbed weight per region, the tallies and,
    when the scene has a detector, its escape image (dims[1], dims[0]).
    voxel=True runs the voxel-geometry model on the fluence grid instead of
    the SDF walk; with_grid=False skips the fluence tally."""
    cs = CScene(scene)
    dims = grid_dims(scene)
    nvox = dims[0] * dims[1] * dims[2]
    tally = bool(nvox and with_grid)
    f = np.zeros(nvox, dtype=np.float64) if tally else None
    absorbed = np.zeros(len(scene["regions"]), dtype=np.float64)
    det = scene.get("detector")
    img = np.zeros(int(det["dims"][0]) * int(det["dims"][1]), dtype=np.float64) if det else None
    t = Tallies()
    if not with_grid and not voxel:
        cs.s.g_dims = (C.c_int32 * 3)(0, 0, 0)
    dp = C.POINTER(C.c_double)
    rc = lib().orc_run_ex(cs.ref, C.c_uint64(seed), C.c_uint64(first), C.c_uint64(n), threads, 1 if voxel else 0,
                          f.ctypes.data_as(dp) if tally else None, absorbed.ctypes.data_as(dp),
                          img.ctypes.data_as(dp) if det else None, C.byref(t))
    if rc != 0:
        raise RuntimeError(f"oracle run failed ({rc})")
    out = tallies_dict(t)
    out["absorbed"] = absorbed
    out["fluence_raw"] = f.reshape(dims[2], dims[1], dims[0]) if tally else None
    if det:
        out["image"] = img.reshape(int(det["dims"][1]), int(det["dims"][0]))
    return out


def trace(scene, seed, pid, cap=50, voxel=False):
    """Event records of packet pid: list of dicts (event, type, region, p, u, w, tau)."""
    cs = CScene(scene)
    buf = (Event * cap)()
    fn = lib().orc_trace_voxel if voxel else lib().orc_trace
    n = fn(cs.ref, C.c_uint64(seed), C.c_uint64(pid), cap, buf)
    if n < 0:
        raise RuntimeError("oracle trace failed")
    return [{"event": e.event, "type": EVENT_TYPES[e.type], "region": e.region, "p": np.array(e.p[:]),
             "u": np.array(e.u[:]), "w": e.w, "tau": e.tau} for e in buf[:n]]


# ---- unit functions (for the pins) ----

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def xi(word):
    return lib().orc_xi(C.c_uint32(word))


def prim_sdf(prim, p):
    s = prim_struct(prim)
    return lib().orc_prim_sdf(C.byref(s), _d3(p))


def smooth_union(a, b, k):
    return lib().orc_smooth_union(a, b, k)


def region_sdf(scene, r, p, _cache={}):
    cs = CScene(scene)
    return lib().orc_region_sdf(cs.ref, r, _d3(p))


def segment_bound(scene, r, p, u):
    """no surface of region r lies on the ray p + t u closer than this"""
    cs = CScene(scene)
    return lib().orc_segment_bound(cs.ref, r, _d3(p), _d3(u))


def region_of(scene, p):
    cs = CScene(scene)
    return lib().orc_region_of(cs.ref, _d3(p))


def region_normal(scene, r, p, h):
    cs = CScene(scene)
    n = (C.c_double * 3)()
    lib().orc_region_normal(cs.ref, r, _d3(p), h, n)
    return np.array(n[:])


def fresnel(n1, n2, cos_i):
    ct = C.c_double()
    R = lib().orc_fresnel(n1, n2, cos_i, C.byref(ct))
    return R, ct.value


def hg_cos(g, x):
    return lib().orc_hg_cos(g, x)


def rotate(u, cos_t, phi):
    v = _d3(u)
    lib().orc_rotate(v, cos_t, phi)
    return np.array(v[:])


def tally_segment(scene, a, b, w):
    cs = CScene(scene)
    dims = grid_dims(scene)
    f = np.zeros(dims[0] * dims[1] * dims[2])
    n = lib().orc_tally_segment(cs.ref, _d3(a), _d3(b), w, f.ctypes.data_as(C.POINTER(C.c_double)))
    return f.reshape(dims[2], dims[1], dims[0]), n


def voxelize(scene):
    """Region index (-1 ambient) of every voxel centre, shape (nz, ny, nx)."""
    cs = CScene(scene)
    dims = grid_dims(scene)
    vox = np.zeros(dims[0] * dims[1] * dims[2], dtype=np.int8)
    lib().orc_voxelize(cs.ref, vox.ctypes.data_as(C.POINTER(C.c_int8)))
    return vox.reshape(dims[2], dims[1], dims[0])


def lib_path():
    return os.path.abspath(_build.LIB)
