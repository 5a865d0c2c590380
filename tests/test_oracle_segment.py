"""Pins of segment tracing in the oracle (Sec. 5 names it beside enhanced
sphere tracing against the many small steps along surfaces).

Outside a convex shape the exact distance along a ray is convex in the ray
parameter, so the tangent at the start bounds it from below: the ray cannot
reach the shape before f(0)/(-f'(0)).  The pins check the bound against
what it claims: the first point of random rays inside each shape (found by
plain sphere tracing on the exact distance, which closes in on it from
before) is never closer than the bound, for every convex kind and for unions; the bound is
exact for a ray aimed at a sphere's centre (so a bound twice as long would
fail); a ray moving away gets no bound from the shape; a point inside a
region gets the plain distance.  Then the walk: segment-traced steps take
the plain march's events on every scene where they apply, in fewer
steps."""
import math

import numpy as np
import pytest


def _one_region(W, prim):
    sc = W._scene("seg", [prim], [W._region([0], 1.0, 1.0, 0.0, 1.0)], None, None, pad=0.1)
    sc["source"] = {"kind": "point", "p": [0.0, 0.0, 0.0]}
    return sc


def _random_prim(rng, kind):
    c = rng.uniform(-0.3, 0.3, 3).tolist()
    if kind == "sphere":
        return {"kind": kind, "c": c, "r": float(rng.uniform(0.1, 0.4))}
    if kind == "box":
        return {"kind": kind, "c": c, "half": rng.uniform(0.05, 0.4, 3).tolist()}
    a = np.asarray(c)
    b = a + rng.normal(size=3) * 0.3
    return {"kind": kind, "a": a.tolist(), "b": b.tolist(), "r": float(rng.uniform(0.03, 0.2))}


def _first_hit(orc, sc, p, u, t_max=4.0):
    """the ray's first point in the region, by plain sphere tracing on the
    exact distance (it never passes a surface and closes in on the first one
    from before it), or inf when the ray leaves the 4 cm reach first"""
    cs = orc.CScene(sc)
    f = lambda q: orc.lib().orc_region_sdf(cs.ref, 0, orc._d3(q))
    t = 0.0
    for _ in range(200000):
        d = f(p + t * u)
        if d < 1e-12:
            return t
        t += d
        if t > t_max:
            return math.inf
    raise AssertionError("sphere tracing did not settle")


@pytest.mark.parametrize("kind", ["sphere", "box", "capsule", "cylinder"])
def test_bound_never_passes_the_first_hit(orc, W, kind):
    rng = np.random.default_rng({"sphere": 1, "box": 2, "capsule": 3, "cylinder": 4}[kind])
    hits = 0
    for _ in range(40):
        sc = _one_region(W, _random_prim(rng, kind))
        while True:
            p = rng.uniform(-1.0, 1.0, 3)
            if orc.region_sdf(sc, 0, p) > 0.02:
                break
        # most rays aim just beside a point of the shape, so that many hit
        # it and many graze it; the rest go anywhere
        prim = sc["prims"][0]
        if kind in ("capsule", "cylinder"):
            a, b = np.asarray(prim["a"]), np.asarray(prim["b"])
            target = a + rng.uniform() * (b - a) + rng.normal(size=3) * 0.7 * prim["r"]
        else:
            size = prim["r"] if kind == "sphere" else min(prim["half"])
            target = np.asarray(prim["c"]) + rng.normal(size=3) * 0.7 * size
        u = target - p if rng.uniform() < 0.8 else rng.normal(size=3)
        u /= np.linalg.norm(u)
        T = orc.segment_bound(sc, 0, p, u)
        d = orc.region_sdf(sc, 0, p)
        assert T >= d * (1 - 1e-12)                     # never shorter than the plain step
        t_hit = _first_hit(orc, sc, p, u)
        hits += math.isfinite(t_hit)
        assert T <= t_hit + 1e-9, (kind, p, u, T, t_hit)
    assert hits >= 15


def test_bound_is_exact_head_on_and_absent_moving_away(orc, W):
    sc = _one_region(W, {"kind": "sphere", "c": [0.1, -0.2, 0.05], "r": 0.3})
    c = np.array([0.1, -0.2, 0.05])
    p = np.array([0.9, 0.4, -0.3])
    u = (c - p) / np.linalg.norm(c - p)
    d = np.linalg.norm(c - p) - 0.3
    assert orc.segment_bound(sc, 0, p, u) == pytest.approx(d, rel=1e-12)   # so 2 T would pass the surface
    assert math.isinf(orc.segment_bound(sc, 0, p, -u))                       # moving away: never met
    # tangent to the sphere: the bound grows without limit as the ray turns away
    side = np.cross(u, [0.0, 0.0, 1.0])
    side /= np.linalg.norm(side)
    t_small = orc.segment_bound(sc, 0, p, (u + 0.05 * side) / np.linalg.norm(u + 0.05 * side))
    t_large = orc.segment_bound(sc, 0, p, (u + 0.4 * side) / np.linalg.norm(u + 0.4 * side))
    assert d < t_small < t_large


def test_union_bound_and_inside_points(orc, W):
    rng = np.random.default_rng(9)
    for _ in range(15):
        prims = [_random_prim(rng, k) for k in ("capsule", "sphere", "box")]
        sc = W._scene("seg", prims, [W._region([0, 1, 2], 1.0, 1.0, 0.0, 1.0)], None, None, pad=0.1)
        sc["source"] = {"kind": "point", "p": [0.0, 0.0, 0.0]}
        while True:
            p = rng.uniform(-1.0, 1.0, 3)
            if orc.region_sdf(sc, 0, p) > 0.02:
                break
        u = -p + rng.normal(size=3) * 0.3
        u /= np.linalg.norm(u)
        assert orc.segment_bound(sc, 0, p, u) <= _first_hit(orc, sc, p, u) + 1e-9
    # inside a region the bound is the plain distance (no tangent argument there)
    sc = _one_region(W, {"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": 0.5})
    p = np.array([0.1, 0.2, 0.0])
    assert orc.segment_bound(sc, 0, p, np.array([1.0, 0.0, 0.0])) == pytest.approx(0.5 - np.linalg.norm(p), rel=1e-12)
    # a smooth union is not a plain union of convex shapes: plain distance
    sm = W._scene("seg", [{"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": 0.2}, {"kind": "sphere", "c": [0.3, 0.0, 0.0], "r": 0.2}],
                  [W._region([0, 1], 1.0, 1.0, 0.0, 1.0, op="smooth_union", k=0.05)], None, None, pad=0.1)
    sm["source"] = {"kind": "point", "p": [0.0, 0.0, 0.0]}
    q = np.array([0.0, 0.8, 0.0])
    assert orc.segment_bound(sm, 0, q, np.array([0.0, 1.0, 0.0])) == pytest.approx(abs(orc.region_sdf(sm, 0, q)), rel=1e-12)


def test_intersection_and_subtraction_bounds(orc, W):
    rng = np.random.default_rng(17)
    for op in ("intersect", "subtract"):
        for _ in range(20):
            prims = [{"kind": "cylinder", "a": [0.0, 0.0, -0.4], "b": [0.0, 0.0, 0.4], "r": float(rng.uniform(0.3, 0.5))},
                     _random_prim(rng, "box" if op == "intersect" else "sphere")]
            sc = W._scene("seg", prims, [W._region([0, 1], 1.0, 1.0, 0.0, 1.0, op=op)], None, None, pad=0.1)
            sc["source"] = {"kind": "point", "p": [0.0, 0.0, 0.0]}
            while True:
                p = rng.uniform(-1.2, 1.2, 3)
                if orc.region_sdf(sc, 0, p) > 0.02:
                    break
            u = rng.normal(size=3) * 0.2 - p
            u /= np.linalg.norm(u)
            T = orc.segment_bound(sc, 0, p, u)
            assert orc.region_sdf(sc, 0, p) <= T <= _first_hit(orc, sc, p, u) + 1e-9, (op, p, u)
    # an intersection is reached only when its last member is: from outside
    # both spheres of a lens, the bound is the later of the two tangent bounds
    lens = W._scene("seg", [{"kind": "sphere", "c": [0.0, 0.0, -0.3], "r": 0.5},
                            {"kind": "sphere", "c": [0.0, 0.0, 0.3], "r": 0.5}],
                    [W._region([0, 1], 1.0, 1.0, 0.0, 1.0, op="intersect")], None, None, pad=0.1)
    lens["source"] = {"kind": "point", "p": [0.0, 0.0, 0.0]}
    p, u = np.array([0.0, 0.0, 1.5]), np.array([0.0, 0.0, -1.0])
    assert orc.segment_bound(lens, 0, p, u) == pytest.approx(1.5 - 0.2, rel=1e-12)   # exact: the far sphere's cap
    assert _first_hit(orc, lens, p, u) == pytest.approx(1.3, abs=1e-9)
    # in the hollow of a subtraction the first member gives no bound
    shell = W._scene("seg", [{"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": 0.5},
                             {"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": 0.4}],
                     [W._region([0, 1], 1.0, 1.0, 0.0, 1.0, op="subtract")], None, None, pad=0.1)
    shell["source"] = {"kind": "point", "p": [0.0, 0.0, 0.0]}
    q = np.array([0.1, 0.0, 0.0])
    assert orc.segment_bound(shell, 0, q, np.array([0.0, 1.0, 0.0])) == pytest.approx(0.3, rel=1e-12)
    assert orc.segment_bound(shell, 0, np.array([0.0, 0.0, 0.9]), np.array([0.0, 0.0, -1.0])) == pytest.approx(0.4, rel=1e-12)


SEG_SCENES = ["sphere", "slab", "glass_sphere", "vessels", "cylinder", "bottle"]


def _desc(W, name):
    if name == "vessels":
        return W.vessel_scene(3, 1.0, n_caps=150, n_grid=12)
    return W.WORKLOADS[name](n_grid=12)


@pytest.mark.parametrize("name", SEG_SCENES)
def test_segment_steps_walk_the_plain_packets(orc, W, name):
    # a segment-traced step ends where the plain march would not: the
    # march enters a surface's delta band at another point, so the surface
    # point lands O(delta^2 curvature) away (O(delta) for a grazing ray
    # that takes the normal's foot), and a ray that passes within delta of
    # a surface may or may not meet the band.  So: every event up to the
    # first surface is the plain march's to rounding (a step that jumped a
    # surface would change it), the first surface point lies within a few
    # delta, and all but a few packets take the same events throughout.
    desc = _desc(W, name)
    seg_desc = dict(desc, segment=True)
    delta = desc["delta"]
    n = 150 if name in ("vessels", "bottle", "cylinder") else 300
    same = 0
    for pid in range(n):
        a = orc.trace(desc, 43, pid, 4000)
        b = orc.trace(seg_desc, 43, pid, 4000)
        for ea, eb in zip(a, b):
            assert (ea["type"], ea["region"], ea["event"]) == (eb["type"], eb["region"], eb["event"]), (name, pid)
            d = eb["p"] - ea["p"]
            if ea["type"] == "ESCAPE":
                d = d - (d @ ea["u"]) * ea["u"]
            if ea["type"] in ("REFLECT", "REFRACT", "CROSS"):
                assert np.abs(d).max() <= 4 * delta, (name, pid, d)
                break
            assert np.abs(d).max() <= 1e-12 and eb["w"] == ea["w"], (name, pid, ea["type"], d)
        same += len(a) == len(b) and all(x["type"] == y["type"] for x, y in zip(a, b))
    assert same >= 0.98 * n, (name, same, n)
    plain = orc.run(desc, 43, 2 * n)
    seg = orc.run(seg_desc, 43, 2 * n)
    # (the sphere and the slab gain only on the way out, where a packet
    # moving away from every region crosses the pad in one step)
    assert seg["steps"] < plain["steps"], (seg["steps"], plain["steps"])


def test_segment_steps_pass_a_sphere_a_beam_grazes(orc, W):
    # a beam through a clear medium passes 1e-3 cm beside a glass sphere:
    # plain steps shrink to the 1e-3 cm gap along the sphere; segment steps
    # see that the ray never meets it
    prims = [{"kind": "box", "c": [0.0, 0.0, 0.0], "half": [2.0, 2.0, 2.0]},
             {"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": 0.5}]
    regions = [W._region([0], 1e-6, 0.0, 0.0, 1.0), W._region([1], 0.01, 0.0, 0.0, 1.5)]
    sc = W._scene("graze", prims, regions, None, None, pad=0.1)
    sc["source"] = {"kind": "pencil", "p": [-1.9, 0.501, 0.0], "u": [1.0, 0.0, 0.0]}
    plain = orc.run(sc, 1, 20)
    seg = orc.run(dict(sc, segment=True), 1, 20)
    assert seg["escaped_face"][1] == pytest.approx(plain["escaped_face"][1]) == pytest.approx(20.0)
    assert seg["interfaces"] == plain["interfaces"] == 20      # the way out of the box only
    # what is left is the march inside the box, whose own distance bounds it
    assert plain["steps"] > 20 * 100
    assert seg["steps"] * 5 < plain["steps"], (seg["steps"], plain["steps"])
