"""FP32 positions as compensated sums on the GPU: a packet flying inside a
region nearly parallel to a face a few surface thresholds away moves across
the face by far less than the position's ulp per sphere-tracing step.  With
a plain FP32 sum those moves are lost and the packet slides along the face
at a fixed depth; with the compensated sum it meets the face where the FP64
oracle's walk does, in about as many steps."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _grazing_block(W):
    # clear block with its top face at z = 1 (position ulp 1.2e-7 cm); the
    # beam starts 1.9e-4 cm below the face and rises at a slope of 2.8e-3,
    # so a step of the face distance moves it up by under half an ulp
    prims = [{"kind": "box", "c": [0.0, 0.0, 0.5], "half": [1.0, 1.0, 0.5]}]
    regions = [W._region([0], 1e-4, 0.0, 0.0, 1.4)]
    sc = W._scene("graze_top", prims, regions, None, None, pad=0.1)
    u = np.array([1.0, 0.0, 0.0028])
    sc["source"] = {"kind": "pencil", "p": [-0.9, 0.0, 1.0 - 1.9e-4], "u": (u / np.linalg.norm(u)).tolist()}
    return sc


def test_grazing_beam_meets_the_face_like_the_oracle(S, eng, orc, W):
    sc = _grazing_block(W)
    o = orc.run(sc, 1, 20)
    ot = orc.trace(sc, 1, 0, 4)
    assert ot[1]["type"] == "REFLECT"            # total internal reflection at the top face
    g = S.run(sc, 1, 20, engine=eng, precision="f32", tally=False)
    gt = S.trace(sc, 1, [0], 4, engine=eng, precision="f32")[0]
    print(f"oracle reflects at x {ot[1]['p'][0]:.6f}, FP32 walk event 1 {gt[1]['type']} at {gt[1]['p']}; "
          f"steps {g['steps']} vs {o['steps']}")
    assert gt[1]["type"] == "REFLECT"
    assert abs(gt[1]["p"][0] - ot[1]["p"][0]) < 2e-3
    assert g["interfaces"] == o["interfaces"] and g["reflections"] == o["reflections"]
    assert g["steps"] <= 1.5 * o["steps"]


def test_slow_packet_of_the_shapes_scene(S, eng, W):
    # packet 828869 of seed 3 flies 0.5 cm just under the top face of the
    # scene's tissue block at a slope of 2.8e-3: with a plain FP32 sum it
    # took 43169 steps (a quarter of a second on one lane, the launch's tail)
    g = S.run(W.WORKLOADS["shapes"](), 3, 1, first=828869, engine=eng, precision="f32", tally=False)
    assert g["escapes"] + g["kills"] == 1 and g["stalls"] == 0
    assert g["steps"] < 5000, g["steps"]
