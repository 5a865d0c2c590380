"""Property pins of the oracle on seeded random scenes (every primitive kind,
placements, modifiers, repetition, region operations, sources; see
workloads.random_scene): the shortcuts that leave the plain march's walk as
it is (free-flight reuse, the ambient skip) must do so on all of them, the
energy identity must hold, and voxelising must give the region of every
voxel centre that the region test gives."""
import numpy as np
import pytest

SEEDS = list(range(12))


@pytest.mark.parametrize("seed", SEEDS)
def test_shortcuts_keep_the_walk(orc, W, seed):
    desc = W.random_scene(seed)
    plain = orc.run(dict(desc, reuse=False, ambient_skip=False), 5, 300)
    fast = orc.run(dict(desc, reuse=True, ambient_skip=True), 5, 300)
    for k in ("interactions", "interfaces", "reflections", "refractions", "kills", "escapes", "stalls"):
        # a bounded distance (twist, bend, displacement, ellipsoid) can be
        # re-evaluated shorter by the plain march and reach an interface
        # point by another rounding: events agree to a few in a thousand
        assert abs(plain[k] - fast[k]) <= max(2, 3e-3 * plain[k]), (seed, k, plain[k], fast[k])
    assert abs(fast["absorbed"].sum() - plain["absorbed"].sum()) <= 1.0      # one packet's weight
    assert abs(fast["escaped_face"].sum() - plain["escaped_face"].sum()) <= 1.0
    assert fast["steps"] <= plain["steps"]


@pytest.mark.parametrize("seed", SEEDS)
def test_energy_identity(orc, W, seed):
    r = orc.run(W.random_scene(seed), 9, 500)
    total = r["absorbed"].sum() + r["escaped_face"].sum() + r["stalled"] + r["roulette_loss"] - r["roulette_gain"]
    assert abs(total - 500.0) <= 1e-9 * 500


@pytest.mark.parametrize("seed", SEEDS[:6])
def test_voxelisation_is_the_region_test(orc, W, seed):
    desc = W.random_scene(seed, n_grid=8)
    vox = orc.voxelize(desc)
    lo, hi, n = np.array(desc["grid"]["lo"]), np.array(desc["grid"]["hi"]), np.array(desc["grid"]["dims"])
    h = (hi - lo) / n
    for idx in np.ndindex(*n[::-1]):
        z, y, x = idx
        c = lo + (np.array([x, y, z]) + 0.5) * h
        assert vox[z, y, x] == orc.region_of(desc, c), (seed, idx)
