"""Scene dictionaries round-trip through JSON files unchanged, and the
oracle walks a loaded scene exactly as the original (every family and the
random scenes, whose parameters are numpy values)."""
import numpy as np
import pytest


@pytest.mark.parametrize("make", ["sphere", "slab", "cylinder", "bottle", "gallery", "shapes", "vessels", "random"])
def test_scene_json_round_trip(W, orc, tmp_path, make):
    if make == "vessels":
        d = W.vessel_scene(3, 1.0, n_caps=60, n_grid=8)
    elif make == "random":
        d = W.random_scene(7, n_grid=8)
    else:
        d = W.WORKLOADS[make](n_grid=8)
    p = tmp_path / "scene.json"
    W.save_scene(d, p)
    e = W.load_scene(p)
    assert e == W._plain(d)
    a, b = orc.run(d, 3, 500), orc.run(e, 3, 500)
    assert np.array_equal(a["absorbed"], b["absorbed"]) and np.array_equal(a["fluence_raw"], b["fluence_raw"])
