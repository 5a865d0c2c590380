"""Seeded synthetic scenes and request streams (input data only).

This module is shared by the GPU path, its tests, the benchmark and the CPU
oracle's tests.  It only describes inputs -- geometry, optical properties,
sources, grids, seeds -- and holds none of the transport arithmetic.

Scene dictionaries (lengths in cm, coefficients in 1/cm):

  {"name": str,
   "n_ambient": float,            refractive index outside every region
   "delta": float,                sphere-tracing surface threshold (Sec. 2.3)
   "pad": float,                  padding of the simulation volume
   "prims": [prim, ...],          see below
   "regions": [{"prims": [i, ...], "op": "union" | "smooth_union" | "intersect" | "subtract", "k": float,
                "mua": float, "mus": float, "g": float, "n": float}, ...],
   "source": source,
   "grid": {"lo": [3], "hi": [3], "dims": [nx, ny, nz]}   (optional),
   "roulette": {"w_threshold": float, "m": int},
   "max_steps": int, "max_events": int}

  prim:   {"kind": "sphere",   "c": [3], "r": float}
          {"kind": "box",      "c": [3], "half": [3]}
          {"kind": "capsule",  "a": [3], "b": [3], "r": float}
          {"kind": "cylinder", "a": [3], "b": [3], "r": float}   (flat caps)
          {"kind": "torus",    "c": [3], "axis": [3], "R": float, "r": float}
  "subtract" is the first listed primitive minus all the others.
  source: {"kind": "point",  "p": [3]}                             isotropic
          {"kind": "pencil", "p": [3], "u": [3]}
          {"kind": "disc",   "c": [3], "r": float, "u": [3]}       top hat, z-plane
          {"kind": "rect",   "c": [3], "half": [hx, hy], "u": [3]} uniform, z-plane

Later regions take priority where regions overlap; outside every region the
medium is ambient (no absorption or scattering, index n_ambient).
"""
from __future__ import annotations

import copy
import math

import numpy as np

AIR = 1.0
ROULETTE = {"w_threshold": 1e-4, "m": 10}
MAX_STEPS = 100_000
MAX_EVENTS = 1_000_000


def _scene(name, prims, regions, source, grid=None, delta=1e-5, pad=None, n_ambient=AIR):
    return {
        "name": name,
        "n_ambient": n_ambient,
        "delta": delta,
        "pad": 10.0 * delta if pad is None else pad,
        "prims": prims,
        "regions": regions,
        "source": source,
        "grid": grid,
        "roulette": dict(ROULETTE),
        "max_steps": MAX_STEPS,
        "max_events": MAX_EVENTS,
    }


def _region(prims, mua, mus, g, n, op="union", k=0.0):
    return {"prims": list(prims), "op": op, "k": k, "mua": mua, "mus": mus, "g": g, "n": n}


# --------------------------------------------------------------------------
# the five workload families
# --------------------------------------------------------------------------

def sphere_scene(n_grid=50):
    """Homogeneous sphere, r = 1 cm (mu_a 0.1, mu_s 10, g 0.9, n 1.38) in
    air, isotropic point source at the centre, fluence on n_grid^3 voxels over
    the sphere's bounding box."""
    prims = [{"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": 1.0}]
    regions = [_region([0], 0.1, 10.0, 0.9, 1.38)]
    grid = {"lo": [-1.0] * 3, "hi": [1.0] * 3, "dims": [n_grid] * 3}
    return _scene("sphere", prims, regions, {"kind": "point", "p": [0.0, 0.0, 0.0]}, grid)


SLAB_LAYERS = (  # (top z, bottom z, mu_a, mu_s, g, n)
    (0.0, -0.01, 1.0, 100.0, 0.8, 1.5),
    (-0.01, -0.21, 0.2, 200.0, 0.9, 1.4),
    (-0.21, -1.21, 0.1, 100.0, 0.9, 1.4),
)


def slab_scene(n_grid=200, layers=SLAB_LAYERS, half_xy=1.0):
    """Three stacked boxes, 2 x 2 cm laterally, 0.01 / 0.2 / 1 cm thick, top
    face at z = 0; normally incident pencil beam along -z starting half a pad
    above the top face; fluence on n_grid^3 voxels over the tissue."""
    prims, regions = [], []
    for i, (top, bot, mua, mus, g, n) in enumerate(layers):
        prims.append({"kind": "box", "c": [0.0, 0.0, 0.5 * (top + bot)],
                      "half": [half_xy, half_xy, 0.5 * (top - bot)]})
        regions.append(_region([i], mua, mus, g, n))
    z_top, z_bot = layers[0][0], layers[-1][1]
    grid = {"lo": [-half_xy, -half_xy, z_bot], "hi": [half_xy, half_xy, z_top], "dims": [n_grid] * 3}
    sc = _scene("slab", prims, regions, None, grid)
    sc["source"] = {"kind": "pencil", "p": [0.0, 0.0, z_top + 0.5 * sc["pad"]], "u": [0.0, 0.0, -1.0]}
    return sc


def cylinder_scene(n_grid=256):
    """1 cm tissue cube (mu_a 0.2, mu_s 100, g 0.9, n 1.38) holding a capped
    cylinder vessel of radius 0.05 cm and length 0.8 cm (mu_a 20, mu_s 400,
    g 0.98, n 1.4) 0.2 cm below the top face, perpendicular to the beam;
    tissue = smooth union (k = 0.01 cm) of the cube and the vessel; top-hat
    beam of radius 0.1 cm along -z."""
    prims = [
        {"kind": "box", "c": [0.0, 0.0, 0.0], "half": [0.5, 0.5, 0.5]},
        {"kind": "cylinder", "a": [-0.4, 0.0, 0.3], "b": [0.4, 0.0, 0.3], "r": 0.05},
    ]
    regions = [
        _region([0, 1], 0.2, 100.0, 0.9, 1.38, op="smooth_union", k=0.01),
        _region([1], 20.0, 400.0, 0.98, 1.4),
    ]
    grid = {"lo": [-0.5] * 3, "hi": [0.5] * 3, "dims": [n_grid] * 3}
    sc = _scene("cylinder", prims, regions, None, grid)
    sc["source"] = {"kind": "disc", "c": [0.0, 0.0, 0.5 + 0.5 * sc["pad"]], "r": 0.1,
                    "u": [0.0, 0.0, -1.0]}
    return sc


_TREES = {}


def vessel_tree(seed, n_caps=2000, side=0.2, r_min=5e-4, r_max=5e-3,
                angle_deg=(20.0, 60.0), length_per_radius=8.0):
    key = (int(seed), n_caps, side, r_min, r_max, tuple(angle_deg), length_per_radius)
    if key not in _TREES:
        _TREES[key] = _vessel_tree(*key[:5], key[5], key[6])
    return [tuple(c) for c in _TREES[key]]


def _vessel_tree(seed, n_caps, side, r_min, r_max, angle_deg, length_per_radius):
    """Seeded random branching tree of capsules inside the cube [0, side]^3.

    Roots start at the centre of the top face pointing -z (later roots at
    random points of the top face if a tree dies out).  Breadth first, every
    capsule end spawns two children at branch angles uniform in angle_deg
    and opposite random azimuths.  Radii are log-uniform in [r_min, r_max],
    lengths length_per_radius * radius; a child is shortened to stay inside
    the cube (one radius from every face) and dropped if that leaves less
    than one radius.  Returns a list of (a, b, r)."""
    rng = np.random.default_rng(seed)
    lo, hi = 0.0, side
    caps = []

    def inside(x, r):
        return np.all(x >= lo + r) and np.all(x <= hi - r)

    def clip_length(a, d, length, r):
        # largest t <= length with a + t d inside [lo + r, hi - r]^3
        t = length
        for i in range(3):
            if d[i] > 0:
                t = min(t, (hi - r - a[i]) / d[i])
            elif d[i] < 0:
                t = min(t, (lo + r - a[i]) / d[i])
        return t

    def new_root(first):
        r = float(math.exp(rng.uniform(math.log(r_min), math.log(r_max))))
        if first:
            a = np.array([0.5 * side, 0.5 * side, hi - r])
        else:
            a = np.array([rng.uniform(lo + r, hi - r), rng.uniform(lo + r, hi - r), hi - r])
        return [(a, np.array([0.0, 0.0, -1.0]))]

    queue = new_root(True)
    while len(caps) < n_caps:
        if not queue:
            queue = new_root(False)
        a, d = queue.pop(0)
        r = float(math.exp(rng.uniform(math.log(r_min), math.log(r_max))))
        if not inside(a, r):
            continue
        length = clip_length(a, d, length_per_radius * r, r)
        if length < r:
            continue
        b = a + length * d
        caps.append((a.tolist(), b.tolist(), r))
        # two children
        d = d / np.linalg.norm(d)
        helper = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(d, helper)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(d, e1)
        az = rng.uniform(0.0, 2.0 * math.pi)
        for k in range(2):
            th = math.radians(rng.uniform(*angle_deg))
            phi = az + k * math.pi
            nd = math.cos(th) * d + math.sin(th) * (math.cos(phi) * e1 + math.sin(phi) * e2)
            queue.append((b.copy(), nd / np.linalg.norm(nd)))
    return caps[:n_caps]


TISSUE = (0.2, 100.0, 0.9, 1.38)
BLOOD = (20.0, 400.0, 0.98, 1.4)


def vessel_scene(seed, mus_scale=1.0, n_caps=2000, n_grid=128, side=0.2):
    """Tissue cube [0, 0.2]^3 cm holding a union of n_caps capsules (the
    seeded vessel tree), tissue and blood properties of the cylinder scene
    with mu_s scaled by mus_scale, uniform illumination of the top face."""
    caps = vessel_tree(seed, n_caps=n_caps, side=side)
    prims = [{"kind": "box", "c": [0.5 * side] * 3, "half": [0.5 * side] * 3}]
    prims += [{"kind": "capsule", "a": a, "b": b, "r": r} for a, b, r in caps]
    t, bl = TISSUE, BLOOD
    regions = [
        _region([0], t[0], t[1] * mus_scale, t[2], t[3]),
        _region(range(1, 1 + len(caps)), bl[0], bl[1] * mus_scale, bl[2], bl[3]),
    ]
    grid = {"lo": [0.0] * 3, "hi": [side] * 3, "dims": [n_grid] * 3}
    sc = _scene("vessels", prims, regions, None, grid, delta=1e-6)
    sc["source"] = {"kind": "rect", "c": [0.5 * side, 0.5 * side, side + 0.5 * sc["pad"]],
                    "half": [0.5 * side, 0.5 * side], "u": [0.0, 0.0, -1.0]}
    sc["seed_tree"] = int(seed)
    # uniform grid of 64^3 cells (31 um): measured on 16 scenes of 2000
    # capsules (FP32, staged capsules) 6.1e6 packets/s at 32^3, 8.7e6 at
    # 48^3, 9.8e6 at 64^3, 9.7e6 at 96^3 -- shorter cell lists outweigh the
    # extra steps the smaller margin costs
    sc["accel_cells"] = [64, 64, 64]
    return sc


def vessel_batch(n_scenes=64, base_seed=1000, n_caps=2000, n_grid=128):
    """n_scenes vessel scenes with seeds base_seed + i and mu_s scaled
    log-uniformly in [0.5, 2]."""
    rng = np.random.default_rng(base_seed)
    scales = np.exp(rng.uniform(math.log(0.5), math.log(2.0), size=n_scenes))
    return [vessel_scene(base_seed + i, float(scales[i]), n_caps=n_caps, n_grid=n_grid)
            for i in range(n_scenes)]


def request_stream(seed, n_requests=1000, rate_hz=10.0, families=("sphere", "slab", "cylinder", "vessels"),
                   packets=(1e4, 1e7), grid_sides=(32, 64, 128, 256), vessel_caps=2000):
    """Poisson stream of requests: (arrival time s, scene, seed, n_packets).
    Family uniform over the given ones; every region's mu_a log-uniform in
    [0.01, 5], mu_s log-uniform in [10, 500], g uniform in [0.7, 0.99], n
    uniform in [1.33, 1.5]; packets log-uniform; grid side uniform over
    grid_sides."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        fam = families[int(rng.integers(len(families)))]
        side = int(grid_sides[int(rng.integers(len(grid_sides)))])
        if fam == "sphere":
            sc = sphere_scene(side)
        elif fam == "slab":
            sc = slab_scene(side)
        elif fam == "cylinder":
            sc = cylinder_scene(side)
        else:  # one of eight trees; the optical properties below make each request distinct
            sc = vessel_scene(int(rng.integers(8)), 1.0, n_caps=vessel_caps, n_grid=side)
        for rg in sc["regions"]:
            rg["mua"] = float(math.exp(rng.uniform(math.log(0.01), math.log(5.0))))
            rg["mus"] = float(math.exp(rng.uniform(math.log(10.0), math.log(500.0))))
            rg["g"] = float(rng.uniform(0.7, 0.99))
            rg["n"] = float(rng.uniform(1.33, 1.5))
        n_pk = int(round(math.exp(rng.uniform(math.log(packets[0]), math.log(packets[1])))))
        out.append({"id": i, "arrival": t, "scene": sc,
                    "seed": int(rng.integers(1 << 62)), "n_packets": n_pk})
    return out


# --------------------------------------------------------------------------
# validation scenes (closed-form special cases)
# --------------------------------------------------------------------------

def beer_lambert_slab(mua=2.0, thickness=0.5, n=1.5, half_xy=50.0):
    """Non-scattering slab at normal incidence: a box of the given thickness
    (top face z = 0) under a pencil beam along -z."""
    prims = [{"kind": "box", "c": [0.0, 0.0, -0.5 * thickness], "half": [half_xy, half_xy, 0.5 * thickness]}]
    regions = [_region([0], mua, 0.0, 0.0, n)]
    grid = {"lo": [-half_xy, -half_xy, -thickness], "hi": [half_xy, half_xy, 0.0], "dims": [1, 1, 50]}
    sc = _scene("beer_lambert", prims, regions, None, grid)
    sc["source"] = {"kind": "pencil", "p": [0.0, 0.0, 0.5 * sc["pad"]], "u": [0.0, 0.0, -1.0]}
    return sc


def stack_scene(layers, half_xy=50.0, nz=0):
    """Non-scattering stack of boxes; layers = [(thickness, mua, n), ...] from
    the top face z = 0 down; pencil beam along -z.  nz > 0 adds a 1 x 1 x nz
    depth grid over the whole stack."""
    prims, regions, z = [], [], 0.0
    for i, (th, mua, n) in enumerate(layers):
        prims.append({"kind": "box", "c": [0.0, 0.0, z - 0.5 * th], "half": [half_xy, half_xy, 0.5 * th]})
        regions.append(_region([i], mua, 0.0, 0.0, n))
        z -= th
    grid = {"lo": [-half_xy, -half_xy, z], "hi": [half_xy, half_xy, 0.0], "dims": [1, 1, nz]} if nz else None
    sc = _scene("stack", prims, regions, None, grid)
    sc["source"] = {"kind": "pencil", "p": [0.0, 0.0, 0.5 * sc["pad"]], "u": [0.0, 0.0, -1.0]}
    return sc


def absorbing_sphere(mua=1.0, r=1.0, n=1.0, n_grid=0):
    """Non-scattering sphere with an isotropic point source at its centre."""
    prims = [{"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": r}]
    regions = [_region([0], mua, 0.0, 0.0, n)]
    grid = {"lo": [-r] * 3, "hi": [r] * 3, "dims": [n_grid] * 3} if n_grid else None
    return _scene("absorbing_sphere", prims, regions, {"kind": "point", "p": [0.0, 0.0, 0.0]}, grid)


def scattering_sphere(tau, r=0.5, n=1.0):
    """Eq. 4 test: purely scattering (mu_a = 0), isotropic (g = 0),
    index-matched sphere of radius r and radial optical depth tau, point
    source at the centre."""
    prims = [{"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": r}]
    regions = [_region([0], 0.0, tau / r, 0.0, n)]
    return _scene("scattering_sphere", prims, regions, {"kind": "point", "p": [0.0, 0.0, 0.0]}, None)


def semi_infinite_slab(mua, mus_reduced, g=0.9, n=1.38, thickness=4.0, half_xy=50.0, nz=400):
    """Sec. 3.1 validation medium: a slab much wider and deeper than the
    penetration depth, light incident along -z.  A pencil beam with one
    lateral bin gives the laterally integrated depth profile, which equals
    the profile under uniform incidence on an infinite slab."""
    mus = mus_reduced / (1.0 - g)
    prims = [{"kind": "box", "c": [0.0, 0.0, -0.5 * thickness], "half": [half_xy, half_xy, 0.5 * thickness]}]
    regions = [_region([0], mua, mus, g, n)]
    grid = {"lo": [-half_xy, -half_xy, -thickness], "hi": [half_xy, half_xy, 0.0], "dims": [1, 1, nz]}
    sc = _scene("semi_infinite", prims, regions, None, grid)
    sc["source"] = {"kind": "pencil", "p": [0.0, 0.0, 0.5 * sc["pad"]], "u": [0.0, 0.0, -1.0]}
    return sc


def absorbing_shell(mua=2.0, r_in=0.7, r_out=1.0, n=1.5):
    """Non-scattering spherical shell (a sphere minus a concentric sphere)
    around an isotropic point source in its hollow centre: every path is
    radial, so escape follows the normal-incidence slab formulas."""
    prims = [{"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": r_out}, {"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": r_in}]
    regions = [_region([0, 1], mua, 0.0, 0.0, n, op="subtract")]
    return _scene("shell", prims, regions, {"kind": "point", "p": [0.0, 0.0, 0.0]}, None)


def absorbing_lens(mua=1.5, r=1.0, sep=1.2):
    """Non-scattering, index-matched lens: the intersection of two unit
    spheres whose centres lie sep apart on x, point source at its centre."""
    prims = [{"kind": "sphere", "c": [-0.5 * sep, 0.0, 0.0], "r": r}, {"kind": "sphere", "c": [0.5 * sep, 0.0, 0.0], "r": r}]
    regions = [_region([0, 1], mua, 0.0, 0.0, 1.0, op="intersect")]
    return _scene("lens", prims, regions, {"kind": "point", "p": [0.0, 0.0, 0.0]}, None)


def torus_beam(mua=2.0, R=1.0, r=0.3, x=1.0):
    """Non-scattering, index-matched torus (axis z, ring radius R, tube
    radius r) under a pencil beam along -z at lateral position x."""
    prims = [{"kind": "torus", "c": [0.0, 0.0, 0.0], "axis": [0.0, 0.0, 1.0], "R": R, "r": r}]
    regions = [_region([0], mua, 0.0, 0.0, 1.0)]
    sc = _scene("torus_beam", prims, regions, None, None)
    sc["source"] = {"kind": "pencil", "p": [x, 0.0, r + 0.5 * sc["pad"]], "u": [0.0, 0.0, -1.0]}
    return sc


def glass_sphere_scene(n_grid=64):
    """Shaped like the paper's curved-surface test (Sec. 3.2): a glass
    sphere (n 1.46, radius 1 cm) at (0.5, 0, -1) cm inside a weakly
    scattering water-like medium (mu_a 0.05, mu_s 2, g 0.9, n 1.33) that
    fills z in [-3, 0.5] over 4 x 4 cm, lit from above by a 0.3 cm top-hat
    beam centred over the sphere's top.  The medium around the sphere is not
    given in the paper; this one is synthetic."""
    prims = [{"kind": "box", "c": [0.0, 0.0, -1.25], "half": [2.0, 2.0, 1.75]},
             {"kind": "sphere", "c": [0.5, 0.0, -1.0], "r": 1.0}]
    regions = [_region([0], 0.05, 2.0, 0.9, 1.33), _region([1], 0.01, 0.0, 0.0, 1.46)]
    grid = {"lo": [-2.0, -2.0, -3.0], "hi": [2.0, 2.0, 0.5], "dims": [n_grid, n_grid, n_grid]}
    sc = _scene("glass_sphere", prims, regions, None, grid)
    sc["source"] = {"kind": "disc", "c": [0.5, 0.0, 0.5 + 0.5 * sc["pad"]], "r": 0.3, "u": [0.0, 0.0, -1.0]}
    return sc


def bottle_scene(n_grid=64):
    """Shaped like the paper's bottle example (Sec. 4 gallery): a glass
    bottle (n 1.5) whose body and neck are each a capped cylinder minus a
    thinner one, partly filled with a milky liquid (the inner cylinder
    intersected with a box below the fill line), lit from above through the
    neck by a 0.3 cm top-hat beam.  Regions: liquid, body, neck (later ones
    own the overlaps).  Synthetic dimensions (cm)."""
    prims = [
        {"kind": "cylinder", "a": [0.0, 0.0, 0.1], "b": [0.0, 0.0, 2.4], "r": 0.9},    # 0 body inside
        {"kind": "box", "c": [0.0, 0.0, 0.8], "half": [1.0, 1.0, 0.8]},                  # 1 below the fill line
        {"kind": "cylinder", "a": [0.0, 0.0, 0.0], "b": [0.0, 0.0, 2.5], "r": 1.0},    # 2 body outside
        {"kind": "cylinder", "a": [0.0, 0.0, 2.3], "b": [0.0, 0.0, 3.5], "r": 0.35},   # 3 neck outside
        {"kind": "cylinder", "a": [0.0, 0.0, 2.2], "b": [0.0, 0.0, 3.6], "r": 0.25},   # 4 neck inside
    ]
    regions = [
        _region([0, 1], 0.05, 20.0, 0.8, 1.33, op="intersect"),   # liquid
        _region([2, 0, 4], 0.02, 0.0, 0.0, 1.5, op="subtract"),   # body glass
        _region([3, 4], 0.02, 0.0, 0.0, 1.5, op="subtract"),      # neck glass
    ]
    grid = {"lo": [-1.0, -1.0, 0.0], "hi": [1.0, 1.0, 3.5], "dims": [n_grid, n_grid, n_grid]}
    sc = _scene("bottle", prims, regions, None, grid)
    sc["source"] = {"kind": "disc", "c": [0.0, 0.0, 3.5 + 0.5 * sc["pad"]], "r": 0.3, "u": [0.0, 0.0, -1.0]}
    return sc


def with_grid(scene, dims, lo=None, hi=None):
    sc = copy.deepcopy(scene)
    g = sc.get("grid") or {}
    sc["grid"] = {"lo": list(lo if lo is not None else g["lo"]), "hi": list(hi if hi is not None else g["hi"]),
                  "dims": list(dims)}
    return sc


def rotation(axis, angle):
    """3 x 3 rotation matrix (nested lists) by angle radians about axis"""
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return (np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * K @ K).tolist()


def gallery_scene(n_grid=64):
    """Shaped like the paper's SDF gallery (Sec. 2.2): placed and modified
    primitives in a 2 x 2 x 2 cm scattering medium (mu_a 0.1, mu_s 20,
    g 0.9, n 1.33) lit from above by a 0.5 cm top-hat beam:
    - a glass box (n 1.5, weakly absorbing) turned 30 deg about (1, 1, 0);
    - a twisted bar (1 rad/cm) of absorbing tissue;
    - a rounded capsule and a scaled torus of blood (one union region);
    - an onion shell of a displaced (bumpy) sphere of dense scatterer;
    - a 3 x 2 array of elongated spheres (capsule-like rods) of glass."""
    prims = [
        {"kind": "box", "c": [0.0, 0.0, 0.0], "half": [1.0, 1.0, 1.0]},
        {"kind": "box", "c": [0.0, 0.0, 0.0], "half": [0.3, 0.2, 0.15],
         "transform": {"R": rotation([1, 1, 0], math.pi / 6), "t": [0.35, 0.35, 0.45], "s": 1.0}},
        {"kind": "box", "c": [0.0, 0.0, 0.0], "half": [0.25, 0.08, 0.5], "twist": 1.0,
         "transform": {"R": rotation([1, 0, 0], math.pi / 2), "t": [-0.4, 0.0, 0.3], "s": 1.0}},
        {"kind": "capsule", "a": [-0.6, -0.5, -0.3], "b": [0.5, -0.6, -0.2], "r": 0.04, "round": 0.03},
        {"kind": "torus", "c": [0.0, 0.0, 0.0], "axis": [0.0, 0.0, 1.0], "R": 1.0, "r": 0.2,
         "transform": {"R": rotation([0, 1, 0], 0.4), "t": [0.3, 0.3, -0.5], "s": 0.35}},
        {"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": 0.25, "onion": 0.06, "displace": {"a": 0.01, "f": 25.0},
         "transform": {"R": rotation([0, 0, 1], 0.0), "t": [-0.45, 0.5, -0.45], "s": 1.0}},
        {"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": 0.05, "elongate": [0.1, 0.0, 0.0],
         "repeat": {"c": [0.35, 0.2, 1.0], "n": [3, 2, 1]},
         "transform": {"R": rotation([0, 0, 1], 0.3), "t": [0.45, -0.45, 0.0], "s": 1.0}},
    ]
    regions = [
        _region([0], 0.1, 20.0, 0.9, 1.33),
        _region([1], 0.05, 0.5, 0.0, 1.5),
        _region([2], 2.0, 80.0, 0.9, 1.4),
        _region([3, 4], 20.0, 400.0, 0.98, 1.4),
        _region([5], 0.5, 300.0, 0.8, 1.45),
        _region([6], 0.02, 0.0, 0.0, 1.5),
    ]
    grid = {"lo": [-1.0] * 3, "hi": [1.0] * 3, "dims": [n_grid] * 3}
    sc = _scene("gallery", prims, regions, None, grid)
    sc["source"] = {"kind": "disc", "c": [0.0, 0.0, 1.0 + 0.5 * sc["pad"]], "r": 0.5, "u": [0.0, 0.0, -1.0]}
    return sc


def shapes_scene(n_grid=48):
    """The further basic shapes of the paper's SDF gallery (Sec. 2.2) in a
    2 x 2 x 2 cm scattering medium (mu_a 0.1, mu_s 20, g 0.9, n 1.33) lit
    from above by a 0.6 cm top-hat beam: a glass frustum, a tilted
    octahedron of absorbing tissue, a hexagonal glass prism, an ellipsoid
    of dense scatterer and a bent rod (a capsule curved by 1.5 rad/cm) of
    blood, each its own region."""
    prims = [
        {"kind": "box", "c": [0.0, 0.0, 0.0], "half": [1.0, 1.0, 1.0]},
        {"kind": "cone", "a": [-0.5, -0.4, 0.5], "b": [-0.3, -0.3, -0.1], "ra": 0.3, "rb": 0.1},
        {"kind": "octahedron", "c": [0.0, 0.0, 0.0], "s": 0.3,
         "transform": {"R": rotation([1, 2, 0], 0.5), "t": [0.45, 0.4, 0.3], "s": 1.0}},
        {"kind": "hexprism", "c": [0.4, -0.45, -0.4], "h": 0.25, "hz": 0.2},
        {"kind": "ellipsoid", "c": [-0.4, 0.45, -0.45], "radii": [0.35, 0.2, 0.15]},
        {"kind": "capsule", "a": [-0.35, 0.0, 0.0], "b": [0.35, 0.0, 0.0], "r": 0.05, "bend": 1.5,
         "transform": {"R": rotation([1, 0, 0], math.pi / 2), "t": [0.1, 0.0, -0.1], "s": 1.0}},
    ]
    regions = [
        _region([0], 0.1, 20.0, 0.9, 1.33),
        _region([1], 0.05, 0.0, 0.0, 1.5),
        _region([2], 3.0, 60.0, 0.9, 1.4),
        _region([3], 0.02, 0.0, 0.0, 1.46),
        _region([4], 0.5, 300.0, 0.8, 1.38),
        _region([5], 20.0, 400.0, 0.98, 1.4),
    ]
    grid = {"lo": [-1.0] * 3, "hi": [1.0] * 3, "dims": [n_grid] * 3}
    sc = _scene("shapes", prims, regions, None, grid)
    sc["source"] = {"kind": "disc", "c": [0.0, 0.0, 1.0 + 0.5 * sc["pad"]], "r": 0.6, "u": [0.0, 0.0, -1.0]}
    return sc


def random_scene(seed, n_grid=16):
    """A seeded random scene for property tests: a scattering medium box
    (2 cm) holding 2-4 further regions of 1-3 primitives each, of every
    kind, placed (rotation, uniform scale, translation) or not, with random
    modifiers (rounding, onion shell, twist or bend, elongation,
    displacement, finite repetition of small spheres), region operations
    (union, smooth union, intersection, difference), optical properties
    (index-matched, glass, scattering) and source (point inside, pencil or
    disc from above)."""
    rng = np.random.default_rng(seed)
    u = lambda a, b: float(rng.uniform(a, b))
    prims = [{"kind": "box", "c": [0.0, 0.0, 0.0], "half": [1.0, 1.0, 1.0]}]
    regions = [_region([0], u(0.05, 1.0), u(5.0, 40.0), u(0.0, 0.95), u(1.0, 1.45))]

    def shape():
        kind = str(rng.choice(["sphere", "box", "capsule", "cylinder", "torus", "cone", "octahedron",
                               "hexprism", "ellipsoid"]))
        c = [0.0, 0.0, 0.0]
        if kind == "sphere":
            return {"kind": kind, "c": c, "r": u(0.08, 0.25)}
        if kind == "box":
            return {"kind": kind, "c": c, "half": [u(0.05, 0.25) for _ in range(3)]}
        if kind in ("capsule", "cylinder"):
            h = u(0.05, 0.25)
            return {"kind": kind, "a": [-h, 0.0, 0.0], "b": [h, 0.0, 0.0], "r": u(0.03, 0.12)}
        if kind == "torus":
            R = u(0.1, 0.25)
            return {"kind": kind, "c": c, "axis": rng.normal(size=3).tolist(), "R": R, "r": u(0.02, 0.5 * R)}
        if kind == "cone":
            h = u(0.05, 0.25)
            return {"kind": kind, "a": [0.0, 0.0, -h], "b": [0.0, 0.0, h], "ra": u(0.03, 0.2), "rb": u(0.0, 0.15)}
        if kind == "octahedron":
            return {"kind": kind, "c": c, "s": u(0.1, 0.3)}
        if kind == "hexprism":
            return {"kind": kind, "c": c, "h": u(0.05, 0.2), "hz": u(0.05, 0.2)}
        return {"kind": kind, "c": c, "radii": [u(0.05, 0.25) for _ in range(3)]}

    def prim(centre):
        p = shape()
        r = rng.uniform()
        if r < 0.12:  # a small repeated sphere
            p = {"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": u(0.03, 0.06),
                 "repeat": {"c": [0.2, 0.2, 0.2], "n": [int(rng.integers(1, 4)) for _ in range(3)]}}
        else:
            if rng.uniform() < 0.3:
                p["round"] = u(0.005, 0.03)
            if rng.uniform() < 0.2:
                p["onion"] = u(0.01, 0.03)
            t = rng.uniform()
            if t < 0.12:
                p["twist"] = u(-3.0, 3.0)
            elif t < 0.24:
                p["bend"] = u(-2.0, 2.0)
            if rng.uniform() < 0.15:
                p["elongate"] = [u(0.0, 0.1) for _ in range(3)]
            if rng.uniform() < 0.12:
                p["displace"] = {"a": u(0.002, 0.01), "f": u(5.0, 30.0)}
        p["transform"] = {"R": rotation(rng.normal(size=3), u(0.0, math.pi)) if rng.uniform() < 0.6 else np.eye(3).tolist(),
                          "t": list(centre), "s": u(0.6, 1.4)}
        return p

    for _ in range(int(rng.integers(2, 5))):
        centre = rng.uniform(-0.55, 0.55, 3)
        ids = []
        for _ in range(int(rng.integers(1, 4))):
            ids.append(len(prims))
            prims.append(prim(centre + rng.uniform(-0.12, 0.12, 3)))
        op = "union"
        if len(ids) > 1:
            op = str(rng.choice(["union", "smooth_union", "intersect", "subtract"]))
        k = u(0.01, 0.08) if op == "smooth_union" else 0.0
        kind = rng.uniform()
        if kind < 0.25:    # index-matched
            mua, mus, g, n = u(0.1, 5.0), u(1.0, 50.0), u(0.0, 0.9), regions[0]["n"]
        elif kind < 0.5:   # glass
            mua, mus, g, n = u(0.01, 0.5), 0.0, 0.0, u(1.3, 1.6)
        else:
            mua, mus, g, n = u(0.1, 10.0), u(5.0, 200.0), u(0.0, 0.98), u(1.3, 1.6)
        regions.append(_region(ids, mua, mus, g, n, op=op, k=k))
    grid = {"lo": [-1.0] * 3, "hi": [1.0] * 3, "dims": [n_grid] * 3}
    sc = _scene(f"random{seed}", prims, regions, None, grid)
    src = rng.uniform()
    if src < 0.3:
        sc["source"] = {"kind": "point", "p": rng.uniform(-0.9, 0.9, 3).tolist()}
    elif src < 0.65:
        sc["source"] = {"kind": "pencil", "p": [u(-0.5, 0.5), u(-0.5, 0.5), 1.0 + 0.5 * sc["pad"]], "u": [0.0, 0.0, -1.0]}
    else:
        sc["source"] = {"kind": "disc", "c": [0.0, 0.0, 1.0 + 0.5 * sc["pad"]], "r": u(0.2, 0.8), "u": [0.0, 0.0, -1.0]}
    return sc


WORKLOADS = {
    "sphere": sphere_scene,
    "slab": slab_scene,
    "cylinder": cylinder_scene,
    "glass_sphere": glass_sphere_scene,
    "bottle": bottle_scene,
    "gallery": gallery_scene,
    "shapes": shapes_scene,
}


# ------------------------------------------------------------ scene files

def _plain(x):
    """numpy scalars and arrays as plain JSON values"""
    if isinstance(x, dict):
        return {k: _plain(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_plain(v) for v in x]
    if isinstance(x, np.ndarray):
        return _plain(x.tolist())
    if isinstance(x, np.integer):
        return int(x)
    if isinstance(x, np.floating):
        return float(x)
    return x


def save_scene(scene, path):
    """Writes a scene dictionary as JSON (the same keys the binding and the
    oracle read)."""
    import json
    with open(path, "w") as f:
        json.dump(_plain(scene), f, indent=1)


def load_scene(path):
    """Reads a scene dictionary written by save_scene (or by hand)."""
    import json
    with open(path) as f:
        return json.load(f)
