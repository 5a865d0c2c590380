"""GPU ambient skip against the oracle's (same rule, same packets): a beam
parallel to a face two surface thresholds off it leaves in a few steps (and
is not lost to the step cap), a beam sloping onto the face still meets it,
the slab packet that refracts out near the critical angle no longer marches
for 1e5 steps, and FP64 walks make the oracle's number of SDF evaluations."""
import numpy as np
import pytest

from gpu_helpers import mirror

pytestmark = pytest.mark.gpu


def _plate(W, beam_p, beam_u, half=1.0):
    prims = [{"kind": "box", "c": [0.0, 0.0, -0.5], "half": [half, half, 0.5]}]
    regions = [W._region([0], 1.0, 10.0, 0.9, 1.4)]
    sc = W._scene("plate", prims, regions, None, None, pad=0.1)
    u = np.asarray(beam_u, float)
    sc["source"] = {"kind": "pencil", "p": list(beam_p), "u": (u / np.linalg.norm(u)).tolist()}
    return sc


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_parallel_beam_leaves_in_a_few_steps(S, eng, orc, W, prec):
    for x0, half in ((-0.55, 0.5), (-1.05, 1.0)):   # the second needs > 1e5 plain steps
        sc = _plate(W, [x0, 0.0, 2e-5], [1.0, 0.0, 0.0], half=half)
        g = S.run(sc, 1, 1000, engine=eng, precision=prec, tally=False)
        # the plain march loses the second beam to the step cap; the oracle's
        # skip, the kernels' rule, lets it escape
        o = orc.run(mirror(sc), 1, 1000)
        assert g["stalls"] == 0 and g["escaped_face"][1] == pytest.approx(1000.0)
        assert g["steps"] <= 4 * 1000
        np.testing.assert_allclose(g["escaped_face"], o["escaped_face"], atol=1e-9)
        if prec == "f64":
            assert g["steps"] == o["steps"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sloping_beam_still_meets_the_face(S, eng, orc, W, prec):
    for slope in (1e-5, 1e-4, 1e-2):
        sc = _plate(W, [-1.05, 0.0, 2e-5 + 0.05 * slope], [1.0, 0.0, -slope])
        g = S.run(sc, 2, 2000, engine=eng, precision=prec, tally=False)
        o = orc.run(sc, 2, 2000)
        assert g["interfaces"] >= 2000 and abs(g["interfaces"] - o["interfaces"]) <= 2
        assert abs(g["absorbed"].sum() - o["absorbed"].sum()) <= 2.0


def test_critical_angle_exit_of_the_slab(S, eng, W):
    # packet 9941878 of seed 3 leaves the slab's bottom face 2e-5 cm below it
    # and nearly parallel in the FP32 walk; without the skip it took 81909
    # steps (one per 2e-5 cm across 1.6 cm of ambient)
    desc = W.slab_scene()
    g = S.run(desc, 3, 1, first=9941878, engine=eng, precision="f32")
    assert g["escapes"] == 1 and g["stalls"] == 0
    assert g["steps"] < 2000, g["steps"]


@pytest.mark.parametrize("name", ["glass_sphere", "bottle"])
def test_fp64_evaluations_match_oracle_with_skips(S, eng, orc, W, name):
    desc = W.WORKLOADS[name](n_grid=16)
    g = S.run(desc, 21, 3000, engine=eng, precision="f64", tally=False)
    o = orc.run(mirror(desc), 21, 3000)
    plain = orc.run(dict(desc, reuse=True), 21, 3000)
    assert o["steps"] < plain["steps"]          # the skip was taken
    assert g["interactions"] == o["interactions"]
    assert abs(g["steps"] - o["steps"]) <= 1e-5 * o["steps"], (g["steps"], o["steps"])
