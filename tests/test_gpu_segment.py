"""GPU segment-traced steps (Sec. 5) against the oracle: traces and step
counts against the oracle's mirror of the same rule (its events are the
plain march's up to where in the delta band a surface is met, pinned in
tests/test_oracle_segment.py), tallies against the plain march on the same
packets, a grazing beam that plain steps crawl along, and the accelerated
vessel network."""
import numpy as np
import pytest

from gpu_helpers import (CHAOTIC, absorbed_agrees, check_fluence, compare_traces, extent_of,
                         identity_residual, mirror, oracle_batches)

pytestmark = pytest.mark.gpu


def _seg(desc):
    return dict(desc, segment=True)


@pytest.mark.parametrize("prec,need", [("f64", 0.99), ("f32", 0.97)])
@pytest.mark.parametrize("name", ["slab", "cylinder", "glass_sphere", "bottle"])
def test_segment_traces_match_oracle_mirror(S, eng, orc, W, name, prec, need):
    desc = _seg(W.WORKLOADS[name](n_grid=32))
    tol = 1e-6 if prec == "f64" else 1e-5
    n, seed = 256, 778
    print(f"segment traces {name} {prec}", flush=True)
    g = S.trace(desc, seed, list(range(n)), 50, engine=eng, precision=prec)
    o = [orc.trace(mirror(desc), seed, pid, 50) for pid in range(n)]
    mut = [rg["mua"] + rg["mus"] for rg in desc["regions"]]
    frac, worst, bad = compare_traces(o, g, extent_of(S, desc), tol, mut=mut)
    print(f"{name} {prec}: agree {frac:.4f} worst {worst} first disagreements {bad[:5]}")
    assert frac >= need, (frac, worst, bad[:10])


@pytest.mark.parametrize("name", ["slab", "cylinder", "glass_sphere", "bottle"])
def test_fp64_segment_steps_match_oracle_mirror(S, eng, orc, W, name):
    # the FP64 walk decides the oracle mirror's way: the same events and, to
    # a few in 1e4, the same number of SDF evaluations (its bounds carry a
    # rounding slack of 16 units in the last place that the oracle's do not)
    desc = _seg(W.WORKLOADS[name](n_grid=16))
    print(f"segment steps {name}", flush=True)
    g = S.run(desc, 21, 3000, engine=eng, precision="f64", tally=False)
    o = orc.run(mirror(desc), 21, 3000)
    p = orc.run(mirror(W.WORKLOADS[name](n_grid=16)), 21, 3000)
    print(f"{name}: steps GPU {g['steps']} mirror {o['steps']} (without segment steps {p['steps']})")
    assert g["interactions"] == o["interactions"] and g["interfaces"] == o["interfaces"]
    assert abs(g["steps"] - o["steps"]) <= 2e-4 * o["steps"], (g["steps"], o["steps"])
    # the slab's packets meet only their own layer's box and the volume (the
    # ambient skip already crosses the pad): no step changes there
    assert o["steps"] <= p["steps"] if name == "slab" else o["steps"] < p["steps"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["glass_sphere", "bottle"])
def test_segment_run_matches_plain_oracle(S, eng, orc, W, name, prec):
    # 1e4 packets: every tally of the segment-traced walk against the
    # oracle's plain march on the same packets
    plain = W.WORKLOADS[name](n_grid=48)
    n, seed = 10000, 99
    print(f"segment run {name} {prec}", flush=True)
    o, se = oracle_batches(orc, plain, seed, n, 10)
    g = S.run(_seg(plain), seed, n, engine=eng, precision=prec)
    assert g["launched"] == n
    assert abs(identity_residual(g)) <= 1e-9 * n
    diff = abs(g["absorbed"].sum() - o["absorbed"].sum())
    print(f"{name} {prec}: absorbed difference {diff:.3e} of {o['absorbed'].sum():.1f}, "
          f"steps {g['steps']} vs plain oracle {o['steps']}")
    # a packet that meets the delta band elsewhere than the plain march may
    # take other decisions later (a valid walk of the same packet): at most
    # 2 packets' weight per 1e4 on the chaotic bottle, to rounding elsewhere
    # in FP64
    if name in CHAOTIC or prec == "f32":
        assert diff <= 2.0 * n / 1e4 or diff <= 1e-4 * o["absorbed"].sum(), diff
    else:
        assert absorbed_agrees(g["absorbed"].sum(), o["absorbed"].sum(), n, "f32", name), diff
    assert g["steps"] < o["steps"]
    check_fluence(g, o, se, plain, "f32")


def test_segment_steps_pass_a_sphere_a_beam_grazes_on_gpu(S, eng, W):
    # a beam in a clear medium runs 1e-3 cm beside a glass sphere: plain
    # steps shrink to the gap; segment steps see that the ray never meets it
    prims = [{"kind": "box", "c": [0.0, 0.0, 0.0], "half": [2.0, 2.0, 2.0]},
             {"kind": "sphere", "c": [0.0, 0.0, 0.0], "r": 0.5}]
    regions = [W._region([0], 1e-6, 0.0, 0.0, 1.0), W._region([1], 0.01, 0.0, 0.0, 1.5)]
    sc = W._scene("graze", prims, regions, None, None, pad=0.1)
    sc["source"] = {"kind": "pencil", "p": [-1.9, 0.501, 0.0], "u": [1.0, 0.0, 0.0]}
    for prec in ("f64", "f32"):
        plain = S.run(sc, 1, 1000, engine=eng, precision=prec, tally=False)
        seg = S.run(_seg(sc), 1, 1000, engine=eng, precision=prec, tally=False)
        print(f"{prec}: steps plain {plain['steps']} segment {seg['steps']}")
        assert plain["escaped_face"][1] >= 999.0 and seg["escaped_face"][1] == plain["escaped_face"][1]
        assert seg["interfaces"] == plain["interfaces"]
        assert seg["steps"] * 5 < plain["steps"], (prec, seg["steps"], plain["steps"])


def test_segment_traces_through_the_vessel_grid(S, eng, orc, W):
    # the accelerated capsule network: tangent bounds of the capsules listed
    # in a cell, the margin for the rest.  A step that jumped a capsule would
    # change the first event after it: against the plain march, every event
    # up to the first surface agrees to rounding, and the events of nearly
    # every packet agree throughout (a packet whose march meets the delta
    # band of a thin capsule elsewhere may take another valid walk after it)
    desc = W.vessel_scene(5, 1.0, n_caps=400, n_grid=32)
    n, seed = 256, 57
    print("segment vessel traces", flush=True)
    g = S.trace(dict(desc, segment=True), seed, list(range(n)), 60, engine=eng, precision="f64")
    o = [orc.trace(desc, seed, pid, 60) for pid in range(n)]
    same = 0
    for pid in range(n):
        a, b = o[pid], g[pid]
        for ea, eb in zip(a, b):
            assert (ea["type"], ea["region"], ea["event"]) == (eb["type"], eb["region"], eb["event"]), pid
            if ea["type"] in ("REFLECT", "REFRACT", "CROSS"):
                break
            if ea["type"] != "ESCAPE":
                assert np.max(np.abs(ea["p"] - eb["p"])) <= 1e-9, (pid, ea["type"])
        same += len(a) == len(b) and all((x["type"], x["region"]) == (y["type"], y["region"]) for x, y in zip(a, b))
    print(f"vessels: {same} of {n} packets take the plain march's events")
    assert same >= 0.97 * n


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_segment_steps_through_the_vessel_grid(S, eng, orc, W, prec):
    # tallies of 4000 packets against the plain march on the same packets;
    # fewer steps than the plain kernel's
    desc = W.vessel_scene(5, 1.0, n_caps=400, n_grid=32)
    n, seed = 4000, 31
    print(f"segment vessels {prec}", flush=True)
    o, se = oracle_batches(orc, desc, seed, n, 10)
    g = S.run(dict(desc, segment=True), seed, n, engine=eng, precision=prec)
    p = S.run(desc, seed, n, engine=eng, precision=prec)
    assert abs(identity_residual(g)) <= 1e-9 * n
    diff = abs(g["absorbed"].sum() - o["absorbed"].sum())
    print(f"vessels {prec}: absorbed difference {diff:.3e} of {o['absorbed'].sum():.1f}, "
          f"steps segment {g['steps']} plain {p['steps']}")
    # each packet that takes another valid walk moves the total by at most
    # its weight (<= 1): up to one packet in 500
    assert diff <= 2e-3 * n, diff
    assert g["steps"] < p["steps"]
    check_fluence(g, o, se, desc, "f32")


def _sphere_box_cloud(W, seed, n=120):
    """A scattering cube holding one accelerated union of n small plain
    spheres and boxes (the grid's general path: primitives, not capsule
    records), a beam from above."""
    rng = np.random.default_rng(seed)
    prims = [{"kind": "box", "c": [0.0, 0.0, 0.0], "half": [0.5, 0.5, 0.5]}]
    for i in range(n):
        c = rng.uniform(-0.42, 0.42, 3).tolist()
        if i % 2:
            prims.append({"kind": "sphere", "c": c, "r": float(rng.uniform(0.01, 0.05))})
        else:
            prims.append({"kind": "box", "c": c, "half": rng.uniform(0.01, 0.04, 3).tolist()})
    regions = [W._region([0], 0.2, 20.0, 0.9, 1.38), W._region(range(1, n + 1), 2.0, 60.0, 0.95, 1.45)]
    grid = {"lo": [-0.5] * 3, "hi": [0.5] * 3, "dims": [24] * 3}
    sc = W._scene("cloud", prims, regions, None, grid)
    sc["source"] = {"kind": "disc", "c": [0.0, 0.0, 0.5 + 0.5 * sc["pad"]], "r": 0.3, "u": [0.0, 0.0, -1.0]}
    sc["accel_cells"] = [16, 16, 16]
    return sc


def test_segment_steps_through_a_grid_of_spheres_and_boxes(S, eng, orc, W):
    # an accelerated union of plain spheres and boxes: the grid's general
    # path bounds the listed primitives by their tangents; in FP64 every
    # event up to the first surface is the plain march's, nearly every
    # packet takes its events throughout, and the run's tallies match the
    # plain oracle on the same packets
    desc = _sphere_box_cloud(W, 4)
    n, seed = 256, 61
    print("segment sphere/box grid traces", flush=True)
    g = S.trace(dict(desc, segment=True), seed, list(range(n)), 60, engine=eng, precision="f64")
    o = [orc.trace(desc, seed, pid, 60) for pid in range(n)]
    same = 0
    for pid in range(n):
        a, b = o[pid], g[pid]
        for ea, eb in zip(a, b):
            assert (ea["type"], ea["region"], ea["event"]) == (eb["type"], eb["region"], eb["event"]), pid
            if ea["type"] in ("REFLECT", "REFRACT", "CROSS"):
                break
            if ea["type"] != "ESCAPE":
                assert np.max(np.abs(ea["p"] - eb["p"])) <= 1e-9, (pid, ea["type"])
        same += len(a) == len(b) and all((x["type"], x["region"]) == (y["type"], y["region"]) for x, y in zip(a, b))
    print(f"sphere/box grid: {same} of {n} packets take the plain march's events")
    assert same >= 0.97 * n
    N = 4000
    ob, se = oracle_batches(orc, desc, 8, N, 10)
    for prec in ("f64", "f32"):
        gs = S.run(dict(desc, segment=True), 8, N, engine=eng, precision=prec)
        gp = S.run(desc, 8, N, engine=eng, precision=prec)
        assert abs(identity_residual(gs)) <= 1e-9 * N
        diff = abs(gs["absorbed"].sum() - ob["absorbed"].sum())
        print(f"{prec}: absorbed difference {diff:.3e} of {ob['absorbed'].sum():.1f}, steps {gs['steps']} vs {gp['steps']}")
        assert diff <= 2e-3 * N, diff
        assert gs["steps"] < gp["steps"]
        check_fluence(gs, ob, se, desc, "f32")
