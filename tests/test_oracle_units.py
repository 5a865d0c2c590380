"""Pins of the oracle's building blocks against definitions it does not use:
published known answers, brute force on tiny inputs, other closed forms of
the same quantity, and invariants."""
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- RNG ----

def test_philox_known_answers(orc):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        words = [int(x, 16) for x in r]
        assert orc.philox(words[0:4], words[4:6]) == words[6:10]


def test_xi_open_interval_and_exact_in_fp32(orc):
    assert orc.xi(0) == 0.5 / 2 ** 23
    assert orc.xi(0xFFFFFFFF) == 1.0 - 0.5 / 2 ** 23
    rng = np.random.default_rng(0)
    for w in rng.integers(0, 2 ** 32, size=2000):
        x = orc.xi(int(w))
        assert 0.0 < x < 1.0
        assert float(np.float32(x)) == x  # same variate in FP32 and FP64
        assert x == ((int(w) >> 9) * 2 + 1) / 2 ** 24


def test_philox_variates_are_uniform(orc):
    xs = np.array([orc.xi(w) for c in range(5000) for w in orc.philox([c, 7, 0, 0], [12345, 678])])
    n = len(xs)
    assert abs(xs.mean() - 0.5) < 4 * math.sqrt(1 / 12 / n)
    hist = np.histogram(xs, bins=20, range=(0, 1))[0]
    chi2 = ((hist - n / 20) ** 2 / (n / 20)).sum()
    assert chi2 < 45  # 19 dof, p ~ 1e-3


# --------------------------------------------------------------- SDFs ----

def _frame(axis):
    axis = axis / np.linalg.norm(axis)
    helper = np.array([1.0, 0, 0]) if abs(axis[0]) < 0.9 else np.array([0, 1.0, 0])
    e1 = np.cross(axis, helper)
    e1 /= np.linalg.norm(e1)
    return axis, e1, np.cross(axis, e1)


def _sphere_surface(c, r, n):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = math.pi * (1 + 5 ** 0.5) * i
    return np.array(c) + r * np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


def _box_surface(c, h, step):
    pts = []
    for ax in range(3):
        o = [a for a in range(3) if a != ax]
        u = np.arange(-h[o[0]], h[o[0]] + 1e-12, step)
        v = np.arange(-h[o[1]], h[o[1]] + 1e-12, step)
        U, V = np.meshgrid(u, v)
        for s in (-1, 1):
            P = np.zeros((U.size, 3))
            P[:, o[0]], P[:, o[1]], P[:, ax] = U.ravel(), V.ravel(), s * h[ax]
            pts.append(P)
    return np.concatenate(pts) + np.array(c)


def _capsule_surface(a, b, r, step):
    a, b = np.array(a), np.array(b)
    L = np.linalg.norm(b - a)
    ax, e1, e2 = _frame(b - a)
    nt = int(2 * math.pi * r / step) + 1
    th = np.linspace(0, 2 * math.pi, nt, endpoint=False)
    xs = np.arange(0, L + 1e-12, step)
    X, T = np.meshgrid(xs, th)
    side = a + X.ravel()[:, None] * ax + r * (np.cos(T.ravel())[:, None] * e1 + np.sin(T.ravel())[:, None] * e2)
    sph = _sphere_surface([0, 0, 0], r, int(4 * math.pi * r * r / step ** 2) + 10)
    caps = np.concatenate([a + sph[sph @ ax <= 0], b + sph[sph @ ax >= 0]])
    return np.concatenate([side, caps])


def _cylinder_surface(a, b, r, step):
    a, b = np.array(a), np.array(b)
    L = np.linalg.norm(b - a)
    ax, e1, e2 = _frame(b - a)
    nt = int(2 * math.pi * r / step) + 1
    th = np.linspace(0, 2 * math.pi, nt, endpoint=False)
    xs = np.arange(0, L + 1e-12, step)
    X, T = np.meshgrid(xs, th)
    side = a + X.ravel()[:, None] * ax + r * (np.cos(T.ravel())[:, None] * e1 + np.sin(T.ravel())[:, None] * e2)
    g = np.arange(-r, r + 1e-12, step)
    G1, G2 = np.meshgrid(g, g)
    keep = G1 ** 2 + G2 ** 2 <= r * r
    disc = G1[keep][:, None] * e1 + G2[keep][:, None] * e2
    return np.concatenate([side, a + disc, b + disc])


def _torus_surface(c, axis, R, r, step):
    ax, e1, e2 = _frame(np.array(axis, float))
    nt = int(2 * math.pi * (R + r) / step) + 1
    npf = int(2 * math.pi * r / step) + 1
    th = np.linspace(0, 2 * math.pi, nt, endpoint=False)
    ph = np.linspace(0, 2 * math.pi, npf, endpoint=False)
    T, F = np.meshgrid(th, ph)
    T, F = T.ravel()[:, None], F.ravel()[:, None]
    ring = np.cos(T) * e1 + np.sin(T) * e2
    return np.array(c) + (R + r * np.cos(F)) * ring + r * np.sin(F) * ax


def _inside_torus(P, pr):
    # inside iff some point of a dense sampling of the ring circle is closer than r
    ax, e1, e2 = _frame(np.array(pr["axis"], float))
    th = np.linspace(0, 2 * math.pi, 20000, endpoint=False)[:, None]
    ring = np.array(pr["c"]) + pr["R"] * (np.cos(th) * e1 + np.sin(th) * e2)
    return cKDTree(ring).query(P)[0] < pr["r"]


def _inside_sphere(P, pr):
    return np.linalg.norm(P - np.array(pr["c"]), axis=1) < pr["r"]


def _inside_box(P, pr):
    return np.all(np.abs(P - np.array(pr["c"])) < np.array(pr["half"]), axis=1)


def _inside_capsule(P, pr):
    # inside iff some point of a dense sampling of the axis is closer than r
    a, b = np.array(pr["a"]), np.array(pr["b"])
    ts = np.linspace(0, 1, 4001)
    axis_pts = a + ts[:, None] * (b - a)
    d = cKDTree(axis_pts).query(P)[0]
    return d < pr["r"]


def _inside_cylinder(P, pr):
    a, b = np.array(pr["a"]), np.array(pr["b"])
    L = np.linalg.norm(b - a)
    ax = (b - a) / L
    x = (P - a) @ ax
    rho = np.linalg.norm((P - a) - x[:, None] * ax, axis=1)
    return (x > 0) & (x < L) & (rho < pr["r"])


PRIMS = [
    ({"kind": "sphere", "c": [0.1, -0.2, 0.3], "r": 0.7}, _sphere_surface, _inside_sphere),
    ({"kind": "box", "c": [0.0, 0.1, -0.1], "half": [0.5, 0.3, 0.8]}, _box_surface, _inside_box),
    ({"kind": "capsule", "a": [-0.4, 0.1, 0.0], "b": [0.3, -0.2, 0.5], "r": 0.25}, _capsule_surface, _inside_capsule),
    ({"kind": "cylinder", "a": [-0.4, 0.1, 0.0], "b": [0.3, -0.2, 0.5], "r": 0.25}, _cylinder_surface, _inside_cylinder),
    ({"kind": "torus", "c": [0.05, 0.0, 0.1], "axis": [0.3, -0.5, 0.8], "R": 0.6, "r": 0.2}, _torus_surface, _inside_torus),
]


@pytest.mark.parametrize("prim,surface,inside", PRIMS, ids=[p[0]["kind"] for p in PRIMS])
def test_sdf_against_brute_force_surface_distance(orc, prim, surface, inside):
    step = 0.004
    if prim["kind"] == "sphere":
        S = surface(prim["c"], prim["r"], 400000)
    elif prim["kind"] == "box":
        S = surface(prim["c"], prim["half"], step)
    elif prim["kind"] == "torus":
        S = surface(prim["c"], prim["axis"], prim["R"], prim["r"], step)
    else:
        S = surface(prim["a"], prim["b"], prim["r"], step)
    tree = cKDTree(S)
    rng = np.random.default_rng(1)
    P = rng.uniform(-1.2, 1.2, size=(600, 3))
    brute = tree.query(P)[0]
    ins = inside(P, prim)
    d = np.array([orc.prim_sdf(prim, p) for p in P])
    # sign from an independent inside test, magnitude from the nearest sample
    assert np.all((d < 0) == ins)
    assert np.all(np.abs(d) <= brute + 1e-12)
    assert np.all(np.abs(d) >= brute - 1.5 * step)


def test_sdf_special_values(orc):
    cap = {"kind": "capsule", "a": [0, 0, 0], "b": [0, 0, 1], "r": 0.2}
    assert orc.prim_sdf(cap, [0, 0, 1.5]) == pytest.approx(0.3, abs=1e-15)
    assert orc.prim_sdf(cap, [0.5, 0, 0.5]) == pytest.approx(0.3, abs=1e-15)
    assert orc.prim_sdf(cap, [0, 0, 0.5]) == pytest.approx(-0.2, abs=1e-15)
    cyl = {"kind": "cylinder", "a": [0, 0, 0], "b": [0, 0, 1], "r": 0.2}
    assert orc.prim_sdf(cyl, [0, 0, 1.5]) == pytest.approx(0.5, abs=1e-15)     # above the cap
    assert orc.prim_sdf(cyl, [0.5, 0, 0.5]) == pytest.approx(0.3, abs=1e-15)   # beside the side
    assert orc.prim_sdf(cyl, [0.5, 0, 1.4]) == pytest.approx(0.5, abs=1e-15)   # beyond the rim: 0.3-0.4-0.5
    assert orc.prim_sdf(cyl, [0, 0, 0.9]) == pytest.approx(-0.1, abs=1e-15)    # nearest is the cap
    box = {"kind": "box", "c": [0, 0, 0], "half": [1, 2, 3]}
    assert orc.prim_sdf(box, [4, 6, 3]) == pytest.approx(5.0, abs=1e-15)       # beyond a corner edge: 3-4-5
    assert orc.prim_sdf(box, [0, 0, 0]) == pytest.approx(-1.0, abs=1e-15)
    sph = {"kind": "sphere", "c": [1, 1, 1], "r": 2}
    assert orc.prim_sdf(sph, [1, 1, 1]) == -2.0
    assert orc.prim_sdf(sph, [4, 5, 1]) == pytest.approx(3.0, abs=1e-15)


def _csg_scene(W, op, prims):
    regions = [W._region(list(range(len(prims))), 0.1, 1.0, 0.0, 1.4, op=op)]
    sc = W._scene("csg", prims, regions, {"kind": "point", "p": [0.0, 0.0, 0.0]})
    return sc


@pytest.mark.parametrize("op", ["intersect", "subtract"])
def test_csg_region_sign_bound_and_lipschitz(orc, W, op):
    A = {"kind": "box", "c": [0.0, 0.0, 0.0], "half": [0.6, 0.5, 0.4]}
    B = {"kind": "sphere", "c": [0.3, 0.2, 0.1], "r": 0.55}
    sc = _csg_scene(W, op, [A, B])
    rng = np.random.default_rng(7)
    P = rng.uniform(-1.0, 1.0, size=(1500, 3))
    inA, inB = _inside_box(P, A), _inside_sphere(P, B)
    inside = (inA & inB) if op == "intersect" else (inA & ~inB)
    d = np.array([orc.region_sdf(sc, 0, p) for p in P])
    assert np.all((d < 0) == inside)
    # the boundary of the combination, sampled: pieces of each surface
    SA, SB = _box_surface(A["c"], A["half"], 0.004), _sphere_surface(B["c"], B["r"], 400000)
    if op == "intersect":
        bnd = np.concatenate([SA[_inside_sphere(SA, B)], SB[_inside_box(SB, A)]])
    else:
        bnd = np.concatenate([SA[~_inside_sphere(SA, B)], SB[_inside_box(SB, A)]])
    true = cKDTree(bnd).query(P)[0]
    assert np.all(np.abs(d) <= true + 1e-12)  # a lower bound of the distance
    # exact where the nearest boundary point is on the face of one primitive
    # away from the other: check a point straight above the box top face
    # outside the sphere
    if op == "subtract":
        assert orc.region_sdf(sc, 0, [-0.5, -0.4, 0.7]) == pytest.approx(0.3, abs=1e-12)
    Q = P + rng.normal(scale=0.05, size=P.shape)
    dq = np.array([orc.region_sdf(sc, 0, q) for q in Q])
    assert np.all(np.abs(dq - d) <= np.linalg.norm(Q - P, axis=1) + 1e-12)


def test_smooth_union_properties(orc):
    rng = np.random.default_rng(2)
    for _ in range(2000):
        a, b = rng.uniform(-1, 1, 2)
        k = rng.uniform(0.01, 0.5)
        s = orc.smooth_union(a, b, k)
        assert s <= min(a, b) + 1e-15
        assert s >= min(a, b) - k / 4 - 1e-15          # deepest blend is k/4 at a == b
        assert s == pytest.approx(orc.smooth_union(b, a, k), abs=1e-14)
        if abs(a - b) >= k:
            assert s == min(a, b)
    assert orc.smooth_union(0.3, 0.3, 0.2) == pytest.approx(0.3 - 0.05, abs=1e-15)
    # Lipschitz 1 along a line through the blend zone
    xs = np.linspace(-1, 1, 4001)
    vals = np.array([orc.smooth_union(x, -x * 0.5 + 0.1, 0.3) for x in xs])
    assert np.max(np.abs(np.diff(vals)) / np.diff(xs)) <= 1.0 + 1e-9


def test_region_priority_and_ambient(orc, W):
    sc = W.sphere_scene()
    sc["prims"] = [{"kind": "sphere", "c": [0, 0, 0], "r": 1.0}, {"kind": "sphere", "c": [0, 0, 0], "r": 0.5},
                   {"kind": "box", "c": [0.9, 0, 0], "half": [0.2, 0.2, 0.2]}]
    sc["regions"] = [dict(sc["regions"][0], prims=[0]), dict(sc["regions"][0], prims=[1]),
                     dict(sc["regions"][0], prims=[2])]
    assert orc.region_of(sc, [0, 0, 0]) == 1          # nested: the later region
    assert orc.region_of(sc, [0, 0.75, 0]) == 0
    assert orc.region_of(sc, [0.95, 0, 0]) == 2       # overlapping: the later region
    assert orc.region_of(sc, [1.05, 0, 0]) == 2       # outside region 0, inside region 2
    assert orc.region_of(sc, [0, 2, 0]) == -1         # ambient


def _analytic_normal(prim, p):
    if prim["kind"] == "sphere":
        v = p - np.array(prim["c"])
        return v / np.linalg.norm(v)
    a, b = np.array(prim["a"]), np.array(prim["b"])
    ax = (b - a) / np.linalg.norm(b - a)
    t = np.clip((p - a) @ (b - a) / ((b - a) @ (b - a)), 0, 1)
    v = p - (a + t * (b - a))
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("kind", ["sphere", "capsule", "box", "cylinder"])
def test_numerical_normals_match_analytic(orc, W, kind):
    sc = W.sphere_scene()
    rng = np.random.default_rng(3)
    h = 1e-7
    for _ in range(50):
        if kind == "sphere":
            prim = {"kind": "sphere", "c": [0.2, 0.1, -0.3], "r": 0.6}
            v = rng.normal(size=3)
            p = np.array(prim["c"]) + 0.6 * v / np.linalg.norm(v)
            want = _analytic_normal(prim, p)
        elif kind == "capsule":
            prim = {"kind": "capsule", "a": [-0.3, 0, 0], "b": [0.3, 0.2, 0.1], "r": 0.2}
            a, b = np.array(prim["a"]), np.array(prim["b"])
            t = rng.uniform(-0.3, 1.3)
            axis = (b - a) / np.linalg.norm(b - a)
            v = rng.normal(size=3)
            if 0 <= t <= 1:
                v -= (v @ axis) * axis
            base = a + np.clip(t, 0, 1) * (b - a)
            p = base + 0.2 * v / np.linalg.norm(v)
            want = _analytic_normal(prim, p)
        elif kind == "box":
            prim = {"kind": "box", "c": [0.1, 0, 0], "half": [0.4, 0.5, 0.6]}
            ax = rng.integers(3)
            s = rng.choice([-1, 1])
            p = np.array(prim["c"]) + rng.uniform(-0.8, 0.8, 3) * np.array(prim["half"])
            p[ax] = prim["c"][ax] + s * prim["half"][ax]
            want = np.zeros(3)
            want[ax] = s
        else:
            prim = {"kind": "cylinder", "a": [0, 0, -0.5], "b": [0, 0, 0.5], "r": 0.3}
            if rng.uniform() < 0.5:  # side
                th = rng.uniform(0, 2 * math.pi)
                p = np.array([0.3 * math.cos(th), 0.3 * math.sin(th), rng.uniform(-0.4, 0.4)])
                want = np.array([math.cos(th), math.sin(th), 0.0])
            else:  # cap
                s = rng.choice([-1, 1])
                rr, th = 0.25 * math.sqrt(rng.uniform()), rng.uniform(0, 2 * math.pi)
                p = np.array([rr * math.cos(th), rr * math.sin(th), 0.5 * s])
                want = np.array([0, 0, float(s)])
        sc["prims"] = [prim]
        sc["regions"] = [dict(sc["regions"][0], prims=[0])]
        n = orc.region_normal(sc, 0, p, h)
        assert np.linalg.norm(n - want) < 1e-7


def test_box_sdf_of_volume(orc):
    lo, hi = [-1, -2, -3], [1, 2, 3]
    lib = orc.lib()
    d3 = orc._d3
    assert lib.orc_box_sdf(d3(lo), d3(hi), d3([0, 0, 0])) == -1.0
    assert lib.orc_box_sdf(d3(lo), d3(hi), d3([0, 0, 3.5])) == pytest.approx(0.5)


# ------------------------------------------------------------ Fresnel ----

def test_fresnel_normal_incidence(orc):
    for n1, n2, want in [(1.0, 1.38, 0.025493), (1.0, 1.5, 0.04), (1.5, 1.0, 0.04), (1.4, 1.4, 0.0)]:
        R, ct = orc.fresnel(n1, n2, 1.0)
        assert R == pytest.approx(((n1 - n2) / (n1 + n2)) ** 2, abs=1e-15)
        assert R == pytest.approx(want, abs=1e-6)
        assert ct == pytest.approx(1.0, abs=1e-15)


def test_fresnel_matches_sine_and_tangent_laws(orc):
    # Fresnel's laws in trigonometric form: r_s = -sin(i - t)/sin(i + t),
    # r_p = tan(i - t)/tan(i + t), with Snell's law n1 sin i = n2 sin t
    for n1, n2 in [(1.0, 1.38), (1.0, 1.5), (1.38, 1.0), (1.5, 1.4), (1.4, 1.5)]:
        crit = math.asin(n2 / n1) if n1 > n2 else math.pi / 2
        for ti in np.linspace(0.01, min(crit, math.pi / 2) - 1e-3, 40):
            tt = math.asin(n1 * math.sin(ti) / n2)
            rs = -math.sin(ti - tt) / math.sin(ti + tt)
            rp = math.tan(ti - tt) / math.tan(ti + tt)
            R, ct = orc.fresnel(n1, n2, math.cos(ti))
            assert R == pytest.approx(0.5 * (rs * rs + rp * rp), abs=1e-12)
            assert ct == pytest.approx(math.cos(tt), abs=1e-12)


def test_fresnel_total_internal_reflection_and_reciprocity(orc):
    crit = math.degrees(math.asin(1.0 / 1.38))
    assert crit == pytest.approx(46.44, abs=0.01)
    assert orc.fresnel(1.38, 1.0, math.cos(math.radians(crit + 0.1)))[0] == 1.0
    assert orc.fresnel(1.38, 1.0, math.cos(math.radians(crit - 0.1)))[0] < 1.0
    # reciprocity: the same reflectance from either side along the same ray pair
    for ci in np.linspace(0.05, 1.0, 30):
        R12, ct = orc.fresnel(1.0, 1.5, ci)
        R21, ci_back = orc.fresnel(1.5, 1.0, ct)
        assert R21 == pytest.approx(R12, abs=1e-12)
        assert ci_back == pytest.approx(ci, abs=1e-12)
    # Brewster: the p wave vanishes, R = R_s / 2
    tb = math.atan(1.5)
    tt = math.pi / 2 - tb
    R, _ = orc.fresnel(1.0, 1.5, math.cos(tb))
    assert R == pytest.approx(0.5 * (math.sin(tb - tt) / math.sin(tb + tt)) ** 2, abs=1e-12)


# ------------------------------------------------------------ scattering --

@pytest.mark.parametrize("g", [0.0, 0.5, 0.8, 0.9, 0.98, -0.3])
def test_hg_moments_by_quadrature(orc, g):
    n = 200000
    xs = (np.arange(n) + 0.5) / n
    c = np.array([orc.hg_cos(g, x) for x in xs])
    assert np.all(np.abs(c) <= 1.0)
    assert c.mean() == pytest.approx(g, abs=2e-4)                 # first moment of HG is g
    assert (c ** 2).mean() == pytest.approx((1 + 2 * g * g) / 3, abs=2e-4)  # second is (1 + 2 g^2)/3


def test_hg_cdf_matches_phase_function(orc):
    # P(cos <= x) from the sampled variates equals the integral of the HG density
    g = 0.9
    n = 100000
    c = np.sort([orc.hg_cos(g, x) for x in (np.arange(n) + 0.5) / n])
    for x in (-0.5, 0.0, 0.5, 0.9, 0.99):
        cdf = (1 - g * g) / (2 * g) * (1 / math.sqrt(1 + g * g - 2 * g * x) - 1 / (1 + g))
        assert np.searchsorted(c, x) / n == pytest.approx(cdf, abs=1e-4)


def test_rotation_keeps_norm_and_angle(orc):
    rng = np.random.default_rng(4)
    for i in range(3000):
        u = rng.normal(size=3)
        if i % 10 == 0:
            u = np.array([1e-4, -2e-4, rng.choice([-1, 1])])
        u /= np.linalg.norm(u)
        ct = rng.uniform(-1, 1)
        phi = rng.uniform(0, 2 * math.pi)
        v = orc.rotate(u, ct, phi)
        assert np.linalg.norm(v) == pytest.approx(1.0, abs=1e-14)
        # near the poles u is taken as exactly +-z: error bounded by |u_perp|
        tol = 2 * math.sqrt(1 - u[2] ** 2) + 1e-12 if abs(u[2]) > 1 - 1e-5 else 1e-12
        assert v @ u == pytest.approx(ct, abs=tol)
        w = orc.rotate(u, ct, phi + math.pi)
        # opposite azimuths: the components normal to u cancel
        perp = (v - (v @ u) * u) + (w - (w @ u) * u)
        assert np.linalg.norm(perp) < 2 * tol


# ------------------------------------------------------------ tally ------

def test_tally_against_dense_sampling(orc, W):
    sc = W.sphere_scene()
    sc["grid"] = {"lo": [-1.0, -0.5, 0.0], "hi": [1.0, 0.5, 2.0], "dims": [7, 5, 9]}
    lo, hi, nd = (np.array(sc["grid"][k], float) for k in ("lo", "hi", "dims"))
    D = (hi - lo) / nd
    rng = np.random.default_rng(5)
    for _ in range(40):
        a = rng.uniform(-1.5, 2.5, 3)
        b = rng.uniform(-1.5, 2.5, 3)
        if rng.uniform() < 0.3:
            b[1] = a[1]  # some segments parallel to a coordinate plane
        f, npieces = orc.tally_segment(sc, a, b, 0.7)
        m = 400000
        t = (np.arange(m) + 0.5) / m
        P = a + t[:, None] * (b - a)
        inside = np.all((P >= lo) & (P <= hi), axis=1)
        idx = np.clip(np.floor((P[inside] - lo) / D).astype(int), 0, nd.astype(int) - 1)
        ref = np.zeros(tuple(nd.astype(int)[::-1]))
        np.add.at(ref, (idx[:, 2], idx[:, 1], idx[:, 0]), 0.7 * np.linalg.norm(b - a) / m)
        assert np.abs(f - ref).max() < 4 * 0.7 * np.linalg.norm(b - a) / m + 1e-12
        assert npieces == np.count_nonzero(f) or npieces >= np.count_nonzero(f)


def test_tally_single_voxel_and_outside(orc, W):
    sc = W.sphere_scene()
    sc["grid"] = {"lo": [0, 0, 0], "hi": [1, 1, 1], "dims": [4, 4, 4]}
    f, n = orc.tally_segment(sc, [0.30, 0.30, 0.30], [0.45, 0.35, 0.40], 2.0)
    assert n == 1
    assert f[1, 1, 1] == pytest.approx(2.0 * math.sqrt(0.15 ** 2 + 0.05 ** 2 + 0.1 ** 2), abs=1e-15)
    f, n = orc.tally_segment(sc, [2, 2, 2], [3, 3, 2], 1.0)
    assert n == 0 and f.sum() == 0
