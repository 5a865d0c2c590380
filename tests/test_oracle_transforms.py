"""Pins of the oracle's placed and modified primitives (Sec. 2.2: SDFs are
translated, rotated, scaled and twisted; the gallery's rounded and hollow
shapes), against what does not use its formulas:
- brute-force nearest distance to densely sampled surfaces and inside tests
  done in the primitive's own frame;
- transport equivalences: an onion shell of a sphere is the difference of
  two spheres, a cylinder twisted about its own axis is the same cylinder,
  and a moved, turned and scaled sphere around a point source meets the
  absorbing-sphere closed form.
"""
import math

import numpy as np
import pytest


def rot(axis, ang):
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def one_prim_scene(W, prim, mua=1.0, n=1.0):
    sc = W._scene("one", [prim], [W._region([0], mua, 0.0, 0.0, n)], {"kind": "point", "p": [0.0, 0.0, 0.0]}, None)
    return sc


def box_surface(half, m=40):
    """points on the faces of the axis-aligned box [-half, half]"""
    h = np.asarray(half, float)
    pts = []
    g = np.linspace(-1, 1, m)
    U, V = np.meshgrid(g, g)
    for ax in range(3):
        o = [i for i in range(3) if i != ax]
        for sgn in (-1, 1):
            P = np.zeros((m * m, 3))
            P[:, ax] = sgn * h[ax]
            P[:, o[0]] = U.ravel() * h[o[0]]
            P[:, o[1]] = V.ravel() * h[o[1]]
            pts.append(P)
    return np.concatenate(pts)


def test_turned_scaled_box_distance_and_sign(orc, W):
    half = np.array([0.3, 0.2, 0.5])
    R, t, s = rot([1, 2, 3], 0.7), np.array([0.1, -0.2, 0.3]), 1.7
    prim = {"kind": "box", "c": [0, 0, 0], "half": half.tolist(),
            "transform": {"R": R.tolist(), "t": t.tolist(), "s": s}}
    sc = one_prim_scene(W, prim)
    surf = s * box_surface(half, 60) @ R.T + t
    rng = np.random.default_rng(1)
    pts = t + rng.uniform(-1.5, 1.5, (300, 3))
    for p in pts:
        d = orc.region_sdf(sc, 0, p)
        local = R.T @ (p - t) / s
        inside = np.all(np.abs(local) < half)
        assert (d < 0) == inside
        near = np.min(np.linalg.norm(surf - p, axis=1))
        # sampled surface: spacing s * 2 * 0.5 / 59 at most
        assert abs(abs(d) - near) < s * 0.5 / 59 * 1.5 + 1e-12, (p, d, near)


def test_scaled_sphere_is_a_sphere(orc, W):
    R, t, s = rot([0, 1, 1], 1.1), np.array([0.4, 0.0, -0.3]), 0.45
    prim = {"kind": "sphere", "c": [0.2, 0.0, 0.0], "r": 1.0,
            "transform": {"R": R.tolist(), "t": t.tolist(), "s": s}}
    sc = one_prim_scene(W, prim)
    centre = s * R @ np.array([0.2, 0.0, 0.0]) + t
    rng = np.random.default_rng(2)
    for p in rng.uniform(-1, 1, (200, 3)):
        assert orc.region_sdf(sc, 0, p) == pytest.approx(np.linalg.norm(p - centre) - s, abs=1e-12)


def test_rounded_sphere_and_onion_shell(orc, W):
    rng = np.random.default_rng(3)
    rounded = one_prim_scene(W, {"kind": "sphere", "c": [0, 0, 0], "r": 0.4, "round": 0.25})
    shell = one_prim_scene(W, {"kind": "sphere", "c": [0, 0, 0], "r": 0.6, "onion": 0.1})
    for p in rng.uniform(-1, 1, (200, 3)):
        r = np.linalg.norm(p)
        assert orc.region_sdf(rounded, 0, p) == pytest.approx(r - 0.65, abs=1e-12)
        assert orc.region_sdf(shell, 0, p) == pytest.approx(abs(r - 0.6) - 0.1, abs=1e-12)


def test_twisted_box_sign_and_lower_bound(orc, W):
    half = np.array([0.4, 0.15, 0.6])
    k = 2.0
    prim = {"kind": "box", "c": [0, 0, 0], "half": half.tolist(), "twist": k}
    sc = one_prim_scene(W, prim)
    # surface: box surface points twisted by angle k z about z
    S = box_surface(half, 80)
    a = k * S[:, 2]
    surf = np.stack([np.cos(a) * S[:, 0] - np.sin(a) * S[:, 1], np.sin(a) * S[:, 0] + np.cos(a) * S[:, 1], S[:, 2]], 1)
    rho = 1.001 * math.hypot(half[0], half[1])
    L = 0.5 * (k * rho + math.sqrt((k * rho) ** 2 + 4))
    rng = np.random.default_rng(4)
    n_in = 0
    for p in rng.uniform(-0.8, 0.8, (400, 3)):
        d = orc.region_sdf(sc, 0, p)
        b = -k * p[2]
        u = np.array([math.cos(b) * p[0] - math.sin(b) * p[1], math.sin(b) * p[0] + math.cos(b) * p[1], p[2]])
        inside = np.all(np.abs(u) < half)
        n_in += inside
        assert (d < 0) == inside, p
        near = np.min(np.linalg.norm(surf - p, axis=1))
        spacing = 2 * 0.6 / 79 * L
        assert abs(d) <= near + spacing, (p, d, near)          # never beyond the surface
        if np.linalg.norm(p[:2]) < rho and abs(p[2]) < 0.6:    # and not needlessly short
            assert abs(d) >= near / L - spacing, (p, d, near)
    assert n_in > 20


@pytest.mark.parametrize("prim", [
    {"kind": "sphere", "c": [0.25, 0.0, 0.0], "r": 0.05, "twist": 3.0},
    {"kind": "capsule", "a": [-0.3, 0.0, 0.0], "b": [0.3, 0.0, 0.0], "r": 0.1, "twist": 2.5},
    {"kind": "box", "c": [0.0, 0.0, 0.0], "half": [0.3, 0.1, 0.5], "twist": -2.5},
    {"kind": "sphere", "c": [0.0, 0.25, 0.0], "r": 0.05, "bend": 3.0},
    {"kind": "capsule", "a": [-0.3, 0.0, 0.0], "b": [0.3, 0.0, 0.0], "r": 0.1, "bend": 2.5},
    {"kind": "box", "c": [0.0, 0.0, 0.0], "half": [0.4, 0.1, 0.1], "bend": -2.0},
])
def test_turned_distance_is_1_lipschitz(orc, prim):
    # a lower bound of the distance must not grow faster than the distance:
    # the gradient of the twisted or bent SDF inside its bounding cylinder
    # has norm <= 1.  The untwist map's Jacobian reaches (k rho +
    # sqrt((k rho)^2 + 4)) / 2 where the shape's gradient mixes the turning
    # direction with the axis (a sphere off the axis, a capsule's caps);
    # dividing by sqrt(1 + (k rho)^2) instead leaves gradients up to 1.07
    # here.  The unbend map's reaches 1 + k rho on the y axis
    rho, zlo, zhi = orc.twist_cylinder(prim)
    rng = np.random.default_rng(9)
    h, worst = 1e-6, 0.0
    for _ in range(6000):
        r = (rho - 1e-4) * math.sqrt(rng.uniform()); th = rng.uniform(0, 2 * math.pi)
        p = np.array([r * math.cos(th), r * math.sin(th), rng.uniform(zlo + 1e-4, zhi - 1e-4)])
        g = [(orc.prim_sdf(prim, p + h * e) - orc.prim_sdf(prim, p - h * e)) / (2 * h) for e in np.eye(3)]
        worst = max(worst, float(np.linalg.norm(g)))
    assert worst <= 1.0 + 1e-6, worst
    assert worst > 0.6   # the bound is not needlessly loose


def bent_points(Q, k):
    """the points p of the bent shape whose unbent image is Q: p_z = q_z and
    p_xy = Rot(k p_x) q_xy, solved for p_x by bisection (unique while
    k |q_xy| < 1)"""
    out = np.empty_like(Q)
    for i, (qx, qy, qz) in enumerate(Q):
        f = lambda t: t - (math.cos(k * t) * qx - math.sin(k * t) * qy)
        a, b = -2.0, 2.0
        for _ in range(60):
            m = 0.5 * (a + b)
            a, b = (m, b) if f(m) < 0 else (a, m)
        t = 0.5 * (a + b)
        out[i] = (t, math.sin(k * t) * qx + math.cos(k * t) * qy, qz)
    return out


def test_bent_capsule_sign_and_lower_bound(orc, W):
    # a rod along x bent by k x radians about z: surface points are the
    # capsule's surface carried forward by the bend; the oracle takes the
    # inverse (unbend) map, so the two meet only through the geometry
    r, k = 0.06, 1.5
    prim = {"kind": "capsule", "a": [-0.3, 0.0, 0.0], "b": [0.3, 0.0, 0.0], "r": r, "bend": k}
    sc = one_prim_scene(W, prim)
    m = 60
    g = np.linspace(0, 1, m)
    U, V = np.meshgrid(g, g)
    ang = 2 * math.pi * U.ravel()
    side = np.column_stack([-0.3 + 0.6 * V.ravel(), r * np.cos(ang), r * np.sin(ang)])
    caps = []
    for cx, sgn in ((-0.3, -1), (0.3, 1)):
        th = 0.5 * math.pi * V.ravel()
        caps.append(np.column_stack([cx + sgn * r * np.sin(th), r * np.cos(th) * np.cos(ang), r * np.cos(th) * np.sin(ang)]))
    surf = bent_points(np.concatenate([side] + caps), k)
    rho = orc.twist_cylinder(prim)[0]
    L = 1 + k * rho
    rng = np.random.default_rng(14)
    n_in = 0
    for p in rng.uniform([-0.45, -0.25, -0.12], [0.45, 0.25, 0.12], (400, 3)):
        d = orc.region_sdf(sc, 0, p)
        b = -k * p[0]
        u = np.array([math.cos(b) * p[0] - math.sin(b) * p[1], math.sin(b) * p[0] + math.cos(b) * p[1], p[2]])
        x = min(max(u[0], -0.3), 0.3)
        inside = math.hypot(u[0] - x, math.hypot(u[1], u[2])) < r
        n_in += inside
        assert (d < 0) == inside, p
        near = np.min(np.linalg.norm(surf - p, axis=1))
        spacing = 0.03
        assert abs(d) <= near + spacing, (p, d, near)
        if np.linalg.norm(p[:2]) < rho and abs(p[2]) < r:
            assert abs(d) >= near / L - spacing, (p, d, near)
    assert n_in > 10


def test_cylinder_bent_about_its_axis_is_the_cylinder(orc, W):
    # a bend turns about the local z axis: a cylinder on that axis is
    # unchanged, and the walk meets the same events
    base = {"kind": "cylinder", "a": [0, 0, -0.5], "b": [0, 0, 0.5], "r": 0.4}
    plain = one_prim_scene(W, base, 0.5, 1.4)
    bent = one_prim_scene(W, dict(base, bend=2.0), 0.5, 1.4)
    plain["regions"][0]["mus"] = bent["regions"][0]["mus"] = 5.0
    for pid in range(40):
        a = orc.trace(plain, 8, pid, 80)
        b = orc.trace(bent, 8, pid, 80)
        assert [(e["type"], e["region"]) for e in a] == [(e["type"], e["region"]) for e in b], pid
        for ea, eb in zip(a, b):
            if ea["type"] != "ESCAPE":
                assert np.abs(ea["p"] - eb["p"]).max() < 1e-3


def test_twist_and_bend_are_exclusive(orc, W):
    prim = {"kind": "box", "c": [0, 0, 0], "half": [0.2, 0.2, 0.2], "twist": 1.0, "bend": 1.0}
    with pytest.raises(ValueError):
        orc.run(one_prim_scene(W, prim), 1, 10)


def test_onion_sphere_equals_sphere_difference(orc, W):
    mua, n = 2.0, 1.5
    onion = one_prim_scene(W, {"kind": "sphere", "c": [0, 0, 0], "r": 0.85, "onion": 0.15}, mua, n)
    diff = W.absorbing_shell(mua, 0.7, 1.0, n)
    for pid in range(40):
        a = orc.trace(onion, 7, pid, 60)
        b = orc.trace(diff, 7, pid, 60)
        assert [(e["type"], e["region"]) for e in a] == [(e["type"], e["region"]) for e in b], pid
        for ea, eb in zip(a, b):
            if ea["type"] != "ESCAPE":
                assert np.abs(ea["p"] - eb["p"]).max() < 1e-7


def test_cylinder_twisted_about_its_axis_is_the_cylinder(orc, W):
    base = {"kind": "cylinder", "a": [0, 0, -0.5], "b": [0, 0, 0.5], "r": 0.4}
    plain = one_prim_scene(W, base, 0.5, 1.4)
    twisted = one_prim_scene(W, dict(base, twist=3.0), 0.5, 1.4)
    plain["regions"][0]["mus"] = twisted["regions"][0]["mus"] = 5.0
    # the twisted distance is divided by the twist's Lipschitz bound, so the
    # one-step snap of an interface lands within delta of the surface rather
    # than on it, and a refraction there turns the path by up to delta/r more;
    # later paths carry that on: events agree exactly, positions to 1e-3 cm
    for pid in range(40):
        a = orc.trace(plain, 8, pid, 80)
        b = orc.trace(twisted, 8, pid, 80)
        assert [(e["type"], e["region"]) for e in a] == [(e["type"], e["region"]) for e in b], pid
        for ea, eb in zip(a, b):
            if ea["type"] != "ESCAPE":
                assert np.abs(ea["p"] - eb["p"]).max() < 1e-3


def test_moved_scaled_sphere_escape_closed_form(orc, W):
    mua, n, s = 1.0, 1.38, 0.6
    R, t = rot([1, 1, 0], 0.3), np.array([0.3, -0.2, 0.1])
    prim = {"kind": "sphere", "c": [0, 0, 0], "r": 1.0, "transform": {"R": R.tolist(), "t": t.tolist(), "s": s}}
    sc = one_prim_scene(W, prim, mua, n)
    sc["source"] = {"kind": "point", "p": t.tolist()}
    N = 100000
    r = orc.run(sc, seed=21, n=N)
    R0 = ((n - 1) / (n + 1)) ** 2
    e = math.exp(-mua * s)
    want = (1 - R0) * e / (1 - R0 * e * e)
    got = r["escaped_face"].sum() / N
    assert abs(got - want) < 4 * math.sqrt(want * (1 - want) / N)


def test_world_box_holds_the_shape(orc, W):
    from oracle.oracle import prim_aabb
    R, t, s = rot([3, -1, 2], 2.2), np.array([1.0, 2.0, -1.0]), 0.8
    prims = [
        {"kind": "box", "c": [0.1, 0, 0], "half": [0.3, 0.2, 0.5], "twist": 1.5, "round": 0.05,
         "transform": {"R": R.tolist(), "t": t.tolist(), "s": s}},
        {"kind": "torus", "c": [0, 0, 0], "axis": [0, 1, 1], "R": 0.5, "r": 0.1, "onion": 0.02,
         "transform": {"R": R.tolist(), "t": t.tolist(), "s": s}},
    ]
    rng = np.random.default_rng(5)
    for prim in prims:
        sc = one_prim_scene(W, prim)
        lo, hi = prim_aabb(prim)
        pts = rng.uniform(lo - 0.5, hi + 0.5, (20000, 3))
        d = np.array([orc.region_sdf(sc, 0, p) for p in pts])
        inside = pts[d < 0]
        assert len(inside) > 50
        assert np.all(inside >= lo) and np.all(inside <= hi)


# ------------------------------------------- elongation, displacement, repetition --

def test_elongated_sphere_is_a_capsule_and_box_a_box(orc, W):
    rng = np.random.default_rng(6)
    el = one_prim_scene(W, {"kind": "sphere", "c": [0, 0, 0], "r": 0.2, "elongate": [0.3, 0.0, 0.0]})
    cap = one_prim_scene(W, {"kind": "capsule", "a": [-0.3, 0, 0], "b": [0.3, 0, 0], "r": 0.2})
    eb = one_prim_scene(W, {"kind": "box", "c": [0, 0, 0], "half": [0.1, 0.2, 0.3], "elongate": [0.2, 0.0, 0.1]})
    big = one_prim_scene(W, {"kind": "box", "c": [0, 0, 0], "half": [0.3, 0.2, 0.4]})
    for p in rng.uniform(-0.8, 0.8, (300, 3)):
        assert orc.region_sdf(el, 0, p) == pytest.approx(orc.region_sdf(cap, 0, p), abs=1e-12)
        d_el, d_big = orc.region_sdf(eb, 0, p), orc.region_sdf(big, 0, p)
        if d_big >= 0:   # exact outside
            assert d_el == pytest.approx(d_big, abs=1e-12)
        else:            # inside: same sign, never beyond the surface
            assert d_el < 0 and abs(d_el) <= abs(d_big) + 1e-12


def test_displaced_sphere_sign_and_lower_bound(orc, W):
    a, f, r = 0.05, 12.0, 0.5
    sc = one_prim_scene(W, {"kind": "sphere", "c": [0, 0, 0], "r": r, "displace": {"a": a, "f": f}})
    D = lambda x: a * np.sin(f * x[..., 0]) * np.sin(f * x[..., 1]) * np.sin(f * x[..., 2])
    # surface by bisection along rays from the centre: g(t) = t - r + D(t w), increasing since a f sqrt(3) < 1
    rng = np.random.default_rng(7)
    W_ = rng.normal(size=(6000, 3))
    W_ /= np.linalg.norm(W_, axis=1, keepdims=True)
    lo, hi = np.full(len(W_), r - 2 * a), np.full(len(W_), r + 2 * a)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        g = mid - r + D(mid[:, None] * W_)
        lo, hi = np.where(g < 0, mid, lo), np.where(g < 0, hi, mid)
    surf = 0.5 * (lo + hi)[:, None] * W_
    L = 1 + a * f * math.sqrt(3)
    for p in rng.uniform(-0.9, 0.9, (300, 3)):
        d = orc.region_sdf(sc, 0, p)
        inside = np.linalg.norm(p) - r + D(p) < 0
        assert (d < 0) == inside
        near = np.min(np.linalg.norm(surf - p, axis=1))
        assert abs(d) <= near + 0.02, (p, d, near)           # 6000 surface samples: spacing ~0.02
        # the displaced surface is within a of the sphere's and |a D| <= a, so
        # |d_sphere + a D| >= near - 2a
        assert abs(d) >= (near - 2 * a) / L - 0.02


def test_repeated_sphere_sign_bound_and_walk(orc, W):
    rep = {"kind": "sphere", "c": [0, 0, 0], "r": 0.15, "repeat": {"c": [0.5, 0.4, 1.0], "n": [3, 2, 1]}}
    sc = one_prim_scene(W, rep, 0.5, 1.4)
    centres = [np.array([(i - 1) * 0.5, (j - 0.5) * 0.4, 0.0]) for i in range(3) for j in range(2)]
    rng = np.random.default_rng(8)
    for p in rng.uniform(-1.2, 1.2, (400, 3)):
        d = orc.region_sdf(sc, 0, p)
        true = min(np.linalg.norm(p - c) - 0.15 for c in centres)
        assert (d < 0) == (true < 0)
        assert abs(d) <= abs(true) + 1e-12
    # the same spheres as one union region: the same events
    prims = [{"kind": "sphere", "c": c.tolist(), "r": 0.15} for c in centres]
    union = W._scene("six", prims, [W._region(range(6), 0.5, 0.0, 0.0, 1.4)], {"kind": "point", "p": [0.0, 0.2, 0.0]}, None)
    sc["source"] = {"kind": "point", "p": [0.0, 0.2, 0.0]}
    union["regions"][0]["mus"] = sc["regions"][0]["mus"] = 3.0
    for pid in range(40):
        a = orc.trace(sc, 9, pid, 80)
        b = orc.trace(union, 9, pid, 80)
        assert [(e["type"], e["region"]) for e in a] == [(e["type"], e["region"]) for e in b], pid
        for ea, eb in zip(a, b):
            if ea["type"] != "ESCAPE":
                assert np.abs(ea["p"] - eb["p"]).max() < 1e-6


def test_repetition_must_fit_its_cells(W):
    from oracle.oracle import prim_struct
    with pytest.raises(ValueError):
        prim_struct({"kind": "sphere", "c": [0, 0, 0], "r": 0.3, "repeat": {"c": [0.5, 1, 1], "n": [2, 1, 1]}})
