"""Pins of the oracle's over-relaxed sphere tracing (enhanced sphere tracing,
the remedy Sec. 5 names for slow steps along grazing surfaces).  A relaxed
step of factor w moves w times the surface distance and is kept only when
the free balls around its two ends cover it, else the plain step is taken and
the rest of the segment up to the next event marches plainly; it must find
every surface the plain march finds:

- event for event, relaxed traces equal the plain oracle's (which every other
  pin holds to closed forms), with interface points to rounding (escapes are
  recorded wherever the march first finds itself outside the volume, so
  only their directions are compared);
- the closed forms of the plain march hold with w = 1.9;
- a thin plate that one relaxed step would jump over is still crossed through
  both faces (transmission exp(-mu_a t / cos));
- grazing paths take far fewer steps.
"""
import math

import numpy as np
import pytest


def _relaxed(desc, w):
    return dict(desc, relax=w)


def _thin_plate(W, mua, thick, u):
    prims = [{"kind": "box", "c": [0.0, 0.0, 0.0], "half": [5.0, 5.0, 0.5 * thick]}]
    regions = [W._region([0], mua, 0.0, 0.0, 1.0)]
    sc = W._scene("thin_plate", prims, regions, None, None, pad=2.0)
    u = np.asarray(u, float) / np.linalg.norm(u)
    sc["source"] = {"kind": "pencil", "p": (-1.5 * u).tolist(), "u": u.tolist()}
    return sc


@pytest.mark.parametrize("name", ["glass_sphere", "cylinder", "slab", "bottle"])
def test_relaxed_traces_equal_plain_traces(orc, W, name):
    desc = W.WORKLOADS[name](n_grid=8)
    relaxed = _relaxed(desc, 1.9)
    same = 0
    n = 60
    for pid in range(n):
        a = orc.trace(desc, 4242, pid, 400)
        b = orc.trace(relaxed, 4242, pid, 400)
        if [(e["type"], e["region"], e["event"]) for e in a] != [(e["type"], e["region"], e["event"]) for e in b]:
            continue
        # an escape is recorded at the first step found outside the volume,
        # which depends on the step lengths: compare its direction only
        dp = max(np.abs(ea["p"] - eb["p"]).max() for ea, eb in zip(a, b) if ea["type"] != "ESCAPE")
        du = max(np.abs(ea["u"] - eb["u"]).max() for ea, eb in zip(a, b))
        dw = max(abs(ea["w"] - eb["w"]) for ea, eb in zip(a, b))
        if dp < 1e-6 and du < 1e-6 and dw < 1e-9:
            same += 1
    assert same >= n - 1, same


@pytest.mark.parametrize("u,thick", [([0.0, 0.0, -1.0], 0.05), ([0.6, 0.0, -0.8], 0.05), ([0.98, 0.0, -0.2], 0.02)])
def test_relaxed_step_does_not_jump_a_thin_plate(orc, W, u, thick):
    mua = 5.0
    sc = _relaxed(_thin_plate(W, mua, thick, u), 1.9)
    N = 20000
    r = orc.run(sc, seed=5, n=N)
    cos = abs(u[2]) / np.linalg.norm(u)
    want = math.exp(-mua * thick / cos)
    got = r["escaped_face"].sum() / N
    # entry face of every packet, exit face of every escaping one (without
    # scattering an interaction absorbs the whole weight)
    assert r["interfaces"] == N + r["escapes"]
    assert abs(got - want) < 4 * math.sqrt(want * (1 - want) / N) + 1e-12
    assert r["absorbed"][0] / N == pytest.approx(1 - want, abs=4 * math.sqrt(want * (1 - want) / N) + 1e-12)


def test_relaxed_closed_forms(orc, W):
    N = 100000
    # Fresnel slab at normal incidence
    mua, L, n = 2.0, 0.5, 1.5
    r = orc.run(_relaxed(W.beer_lambert_slab(mua, L, n), 1.9), seed=11, n=N)
    R = ((n - 1) / (n + 1)) ** 2
    e = math.exp(-mua * L)
    T = (1 - R) ** 2 * e / (1 - R * R * e * e)
    assert abs(r["escaped_face"][4] / N - T) < 4 * math.sqrt(T * (1 - T) / N)
    # point source in an absorbing sphere with an index step
    mua, rad, n = 1.0, 1.0, 1.38
    r = orc.run(_relaxed(W.absorbing_sphere(mua, rad, n), 1.9), seed=14, n=N)
    R0 = ((n - 1) / (n + 1)) ** 2
    e = math.exp(-mua * rad)
    want = (1 - R0) * e / (1 - R0 * e * e)
    assert abs(r["escaped_face"].sum() / N - want) < 4 * math.sqrt(want * (1 - want) / N)
    # shell (difference): radial paths see a slab twice
    mua, r_in, r_out, n = 2.0, 0.7, 1.0, 1.5
    r = orc.run(_relaxed(W.absorbing_shell(mua, r_in, r_out, n), 1.9), seed=31, n=N)
    R = ((n - 1) / (n + 1)) ** 2
    a = math.exp(-mua * (r_out - r_in))
    T_slab = (1 - R) ** 2 * a / (1 - R * R * a * a)
    R_slab = R + R * (1 - R) ** 2 * a * a / (1 - R * R * a * a)
    want = T_slab / (1 - R_slab)
    assert abs(r["escaped_face"].sum() / N - want) < 4 * math.sqrt(want * (1 - want) / N)
    # torus tube chord
    r = orc.run(_relaxed(W.torus_beam(2.0, 1.0, 0.3, x=1.0), 1.9), seed=33, n=N)
    want = math.exp(-2.0 * 2.0 * 0.3)
    assert abs(r["escaped_face"][4] / N - want) < 4 * math.sqrt(want * (1 - want) / N)


def test_relaxed_fluence_and_ledger_equal_plain(orc, W):
    # same packets, same events: the deferred crediting of relaxed steps
    # gives the plain march's fluence.  A grazing hit snaps to the foot of
    # the normal from where the march stopped (within delta of the surface),
    # so positions after one may move by up to ~delta tangentially: that is
    # the tolerance
    desc = W.slab_scene(n_grid=16)
    a = orc.run(desc, 9, 400)
    b = orc.run(_relaxed(desc, 1.9), 9, 400)
    assert a["interactions"] == b["interactions"] and a["interfaces"] == b["interfaces"]
    np.testing.assert_allclose(b["absorbed"], a["absorbed"], rtol=1e-9)
    np.testing.assert_allclose(b["fluence_raw"], a["fluence_raw"], rtol=1e-5, atol=1e-6 * a["fluence_raw"].max())
    assert b["steps"] < a["steps"]


def test_relaxed_march_saves_grazing_steps(orc, W):
    # a beam skimming 0.01 cm under the top face of a clear, index-matched
    # 10 cm block: plain steps are the depth under the face, relaxed ones w
    # times that (1/w as many steps)
    prims = [{"kind": "box", "c": [0.0, 0.0, -0.5], "half": [5.0, 5.0, 0.5]}]
    regions = [W._region([0], 1e-4, 0.0, 0.0, 1.0)]
    sc = W._scene("graze", prims, regions, None, None, pad=0.5)
    sc["source"] = {"kind": "pencil", "p": [-5.2, 0.0, -0.01], "u": [1.0, 0.0, 0.0]}
    plain = orc.run(sc, 1, 200)
    relaxed = orc.run(_relaxed(sc, 1.9), 1, 200)
    assert plain["escaped_face"][1] >= 198.0 and abs(relaxed["escaped_face"][1] - plain["escaped_face"][1]) <= 1.0
    assert relaxed["steps"] < 0.6 * plain["steps"], (relaxed["steps"], plain["steps"])


def test_relax_outside_range_is_rejected(orc, W):
    with pytest.raises(Exception):
        orc.run(_relaxed(W.sphere_scene(n_grid=4), 2.0), 1, 10)
    with pytest.raises(Exception):
        orc.run(_relaxed(W.sphere_scene(n_grid=4), 0.9), 1, 10)
