"""Pins of the oracle's step-count mirror against its plain march.

The oracle's walk is the plain step loop of Sec. 2.3.  The kernels take
shortcuts that change how many SDF evaluations a packet needs but not its
events -- free-flight reuse, the ambient skip and over-relaxed steps
(Sec. 5) -- and the oracle has a mirror of them (walk_mirror) so that tests
can compare evaluation counts.  On every workload family the mirror must
walk the plain march's packets: the same events of every kind, and the
same absorbed, escaped and fluence tallies, exactly where every distance is
exact and to rounding where some are bounds (ellipsoid, twist, bend,
displacement) or relaxed steps change the place of grazing hits (within
delta); and it must need fewer evaluations.  Every GPU parity test compares
the kernels, shortcuts on, with the plain march."""
import numpy as np
import pytest

EVENTS = ("interactions", "interfaces", "reflections", "refractions", "crossings", "kills", "escapes", "stalls")
BOUNDED = ("gallery", "shapes")


def _scene(W, name):
    if name == "vessels":
        return W.vessel_scene(3, 1.0, n_caps=150, n_grid=12)
    return W.WORKLOADS[name](n_grid=12)


@pytest.mark.parametrize("relax", [1.0, 1.9])
@pytest.mark.parametrize("name", ["sphere", "slab", "cylinder", "vessels", "glass_sphere", "bottle", "gallery",
                                  "shapes"])
def test_mirror_walks_the_plain_packets(orc, W, name, relax):
    desc = _scene(W, name)
    n = 300 if name in ("slab", "cylinder", "bottle", "vessels") else 1000
    plain = orc.run(desc, 41, n)
    fast = orc.run(dict(desc, reuse=True, ambient_skip=True, relax=relax), 41, n)
    for k in EVENTS:
        assert fast[k] == plain[k], (name, relax, k, fast[k], plain[k])
    exact = name not in BOUNDED and relax == 1.0
    if exact:
        np.testing.assert_array_equal(fast["absorbed"], plain["absorbed"])
        np.testing.assert_array_equal(fast["escaped_face"], plain["escaped_face"])
    else:
        np.testing.assert_allclose(fast["absorbed"], plain["absorbed"], rtol=1e-9)
        # the same escaped weight; the face is named at the first point the
        # march finds outside the volume, which a longer relaxed step can
        # put past an edge of the box, on the neighbouring face
        assert fast["escaped_face"].sum() == pytest.approx(plain["escaped_face"].sum(), rel=1e-9)
    F, Fp = fast["fluence_raw"], plain["fluence_raw"]
    assert np.linalg.norm(F - Fp) <= (1e-13 if exact else 1e-4) * np.linalg.norm(Fp)
    assert fast["steps"] < plain["steps"]


@pytest.mark.parametrize("name", ["slab", "cylinder", "glass_sphere"])
def test_mirror_traces_are_the_plain_traces(orc, W, name):
    desc = _scene(W, name)
    for pid in range(40):
        a = orc.trace(desc, 5, pid, 200)
        b = orc.trace(dict(desc, reuse=True, ambient_skip=True), 5, pid, 200)
        assert len(a) == len(b), pid
        for ea, eb in zip(a, b):
            assert (ea["type"], ea["region"], ea["event"]) == (eb["type"], eb["region"], eb["event"])
            d = eb["p"] - ea["p"]
            if ea["type"] == "ESCAPE":   # recorded at the first point found outside: compare off the exit ray
                d = d - (d @ ea["u"]) * ea["u"]
            assert np.max(np.abs(d)) <= 1e-12, (pid, ea["type"], d)
            np.testing.assert_allclose(eb["u"], ea["u"], rtol=0, atol=1e-12)
            assert eb["w"] == pytest.approx(ea["w"], rel=1e-12) and eb["tau"] == pytest.approx(ea["tau"], rel=1e-9, abs=1e-12)
