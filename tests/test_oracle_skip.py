"""Pins of the ambient skip in the oracle: outside every region, a packet
whose ray enters none of the regions' surface boxes before its next step
would end moves to the first box it enters, or past the volume's boundary,
in one move.  Against the plain march (the oracle with the skip off):
- the same events, absorption, escapes and fluence, and no more SDF
  evaluations, on every workload;
- a beam that runs parallel to a face two surface thresholds away (the
  refracted ray at the critical angle) leaves in a few steps instead of one
  per 2 delta of its path;
- a beam that slopes down onto the face still meets it;
- a beam through the hole of a torus still enters its box and marches.
The escape face is the one the ray crosses, δ past it; the plain march
names the face at the point its last step reaches, which near an edge of a
widely padded volume can be the neighbouring face.
"""
import numpy as np
import pytest


def on(sc, **kw):
    """the oracle's shortcut walk with the ambient skip (and free-flight reuse)"""
    return dict(sc, reuse=True, ambient_skip=True, **kw)


def off(sc, **kw):
    """the same walk without the ambient skip"""
    return dict(sc, reuse=True, ambient_skip=False, **kw)


@pytest.mark.parametrize("name", ["slab", "cylinder", "sphere", "glass_sphere", "bottle", "gallery", "shapes"])
def test_skip_walks_the_same_packets(orc, W, name):
    desc = W.WORKLOADS[name](n_grid=12)
    n = 300 if name in ("slab", "cylinder", "bottle") else 1000
    for relax in (1.0, 1.9):
        a = orc.run(off(desc, relax=relax), 7, n)
        b = orc.run(on(desc, relax=relax), 7, n)
        for k in ("interactions", "interfaces", "reflections", "refractions", "kills", "escapes", "stalls"):
            assert a[k] == b[k], (name, relax, k)
        np.testing.assert_allclose(b["absorbed"], a["absorbed"], rtol=1e-12)
        np.testing.assert_allclose(b["escaped_face"], a["escaped_face"], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(b["fluence_raw"], a["fluence_raw"], rtol=1e-9, atol=1e-12)
        assert b["steps"] <= a["steps"]


def _plate(W, beam_p, beam_u, pad=0.1, half=1.0):
    prims = [{"kind": "box", "c": [0.0, 0.0, -0.5], "half": [half, half, 0.5]}]
    regions = [W._region([0], 1.0, 10.0, 0.9, 1.4)]
    sc = W._scene("plate", prims, regions, None, None, pad=pad)
    u = np.asarray(beam_u, float)
    sc["source"] = {"kind": "pencil", "p": list(beam_p), "u": (u / np.linalg.norm(u)).tolist()}
    return sc


def test_parallel_beam_two_thresholds_off_a_face(orc, W):
    # the beam runs along +x at 2 delta above the top face of a 1 cm plate:
    # the plain march steps by the 2e-5 cm distance, the skip leaves at once
    sc = _plate(W, [-0.55, 0.0, 2e-5], [1.0, 0.0, 0.0], half=0.5)
    plain = orc.run(off(sc), 1, 5)
    fast = orc.run(on(sc), 1, 5)
    assert plain["escaped_face"][1] == pytest.approx(5.0) and fast["escaped_face"][1] == pytest.approx(5.0)
    assert plain["steps"] > 5 * 40000
    assert fast["steps"] <= 5 * 4
    assert plain["interfaces"] == fast["interfaces"] == 0


def test_parallel_beam_beyond_the_step_cap(orc, W):
    # over 2 cm the plain march needs more steps than the cap of 1e5 per
    # event and hands the packets to the stall ledger; the skip escapes them
    sc = _plate(W, [-1.05, 0.0, 2e-5], [1.0, 0.0, 0.0])
    plain = orc.run(off(sc), 1, 5)
    fast = orc.run(on(sc), 1, 5)
    assert plain["stalls"] == 5 and plain["stalled"] == pytest.approx(5.0)
    assert fast["stalls"] == 0 and fast["escaped_face"][1] == pytest.approx(5.0)


def test_beam_sloping_onto_the_face_still_meets_it(orc, W):
    # from 2 delta above the face at a slope of 1e-5: it reaches the face
    # after 2 mm (inside the grown box every step is a plain one)
    for slope in (1e-5, 1e-4, 1e-2):
        sc = _plate(W, [-1.05, 0.0, 2e-5 + 0.05 * slope], [1.0, 0.0, -slope])
        a = orc.run(off(sc), 2, 50)
        b = orc.run(on(sc), 2, 50)
        assert a["interfaces"] == b["interfaces"] >= 50
        np.testing.assert_allclose(b["absorbed"], a["absorbed"], rtol=1e-12)
        np.testing.assert_allclose(b["escaped_face"], a["escaped_face"], rtol=1e-12, atol=1e-12)
        t = orc.trace(on(sc), 2, 0, 3)
        assert t[1]["type"] in ("REFRACT", "REFLECT")
        assert abs(t[1]["p"][2]) < 1e-4


def test_beam_through_a_torus_hole(orc, W):
    # the beam crosses the torus's box through its hole without meeting the
    # tube: it enters the box, marches across, and leaves; a second beam
    # meets the tube
    prims = [{"kind": "torus", "c": [0.0, 0.0, 0.0], "axis": [0.0, 0.0, 1.0], "R": 0.5, "r": 0.1}]
    regions = [W._region([0], 1.0, 1.0, 0.0, 1.0)]
    for x0, meets in ((0.0, False), (0.5, True)):
        sc = W._scene("ring", prims, regions, None, None, pad=0.5)
        sc["source"] = {"kind": "pencil", "p": [x0, 0.0, 0.9], "u": [0.0, 0.0, -1.0]}
        a = orc.run(off(sc), 3, 200)
        b = orc.run(on(sc), 3, 200)
        for k in ("interactions", "interfaces", "escapes"):
            assert a[k] == b[k], (x0, k)
        assert (b["interfaces"] > 0) == meets
        # the same escaped weight; with a pad of 0.5 cm the plain march's
        # last step can end past an edge of the volume, where the face it
        # names is the neighbour of the one the ray crossed, which the skip
        # names; faces are compared where the ray direction decides them
        assert b["escaped_face"].sum() == pytest.approx(a["escaped_face"].sum(), rel=1e-12)
        np.testing.assert_allclose(b["escaped_face"][4:], a["escaped_face"][4:], rtol=0.05)
        assert b["steps"] <= a["steps"]


def test_grazing_refraction_out_of_the_slab(orc, W):
    # a packet of the slab that leaves the bottom face near the critical
    # angle: the skip takes it out of the volume in a few steps, with the
    # same escape as the plain march
    desc = W.slab_scene(n_grid=8)
    a = orc.run(off(desc), 3, 1, first=9941878, threads=1)
    b = orc.run(on(desc), 3, 1, first=9941878, threads=1)
    np.testing.assert_array_equal(a["escaped_face"], b["escaped_face"])
    assert a["interactions"] == b["interactions"] and a["interfaces"] == b["interfaces"]
    assert b["steps"] < a["steps"]
