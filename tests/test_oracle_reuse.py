"""Pins of free-flight reuse in the oracle: after an interaction inside a
region, the last evaluated surface distance less the path since bounds the
distance to every surface, and an interaction inside that ball is taken
without a new SDF evaluation.  It must give the walk that evaluates before
every interaction, with or without over-relaxed steps and placed primitives,
and fewer evaluations: bit for bit where every distance is exact; to
rounding where some are only bounds (twist, displacement, ellipsoid), since
there the re-evaluated bound can be shorter than the ball and plain marching
reaches the same interaction point in two moves instead of one.  (The
oracle's default walk is the plain march; reuse and the ambient skip are
switched on here explicitly.)"""
import numpy as np
import pytest


@pytest.mark.parametrize("name", ["slab", "cylinder", "sphere", "glass_sphere", "bottle", "gallery", "shapes"])
def test_reuse_walks_the_same_packets(orc, W, name):
    desc = W.WORKLOADS[name](n_grid=12)
    n = 300 if name in ("slab", "cylinder", "bottle") else 1000
    for relax in (1.0, 1.9):
        a = orc.run(dict(desc, ambient_skip=True, relax=relax), 7, n)
        b = orc.run(dict(desc, reuse=True, ambient_skip=True, relax=relax), 7, n)
        for k in ("interactions", "interfaces", "reflections", "refractions", "kills", "escapes", "stalls"):
            assert a[k] == b[k], (name, relax, k)
        if name in ("gallery", "shapes"):   # bounded distances: equal to rounding
            np.testing.assert_allclose(b["absorbed"], a["absorbed"], rtol=1e-12)
            np.testing.assert_allclose(b["escaped_face"], a["escaped_face"], rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(b["fluence_raw"], a["fluence_raw"], rtol=1e-7, atol=1e-12)
        else:
            np.testing.assert_array_equal(b["absorbed"], a["absorbed"])
            np.testing.assert_array_equal(b["escaped_face"], a["escaped_face"])
            np.testing.assert_array_equal(b["fluence_raw"], a["fluence_raw"])
        assert b["steps"] <= a["steps"]


def test_reuse_traces_are_identical(orc, W):
    desc = W.slab_scene(n_grid=8)
    for pid in range(20):
        a = orc.trace(dict(desc, ambient_skip=True), 3, pid, 300)
        b = orc.trace(dict(desc, reuse=True, ambient_skip=True), 3, pid, 300)
        assert len(a) == len(b)
        for ea, eb in zip(a, b):
            assert (ea["type"], ea["region"], ea["event"]) == (eb["type"], eb["region"], eb["event"])
            np.testing.assert_array_equal(ea["p"], eb["p"])
            np.testing.assert_array_equal(ea["u"], eb["u"])
            assert ea["w"] == eb["w"] and ea["tau"] == eb["tau"]


def test_reuse_saves_most_evaluations_in_the_slab(orc, W):
    desc = W.slab_scene(n_grid=8)
    a = orc.run(dict(desc, ambient_skip=True), 4, 300)
    b = orc.run(dict(desc, reuse=True, ambient_skip=True), 4, 300)
    assert b["steps"] < 0.5 * a["steps"], (b["steps"], a["steps"])
