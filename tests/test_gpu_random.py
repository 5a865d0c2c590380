"""GPU parity with the oracle on seeded random scenes (every primitive kind,
placements, modifiers, repetition, region operations and sources; see
workloads.random_scene), through the C ABI: event traces, run totals,
fluence and voxelisation.  Same tolerances as the fixed scenes' parity
tests; scenes with bounded distances (twist, bend, displacement,
ellipsoid) are held to one packet's weight, as there."""
import numpy as np
import pytest

from gpu_helpers import check_fluence, compare_traces, extent_of, identity_residual, oracle_batches

pytestmark = pytest.mark.gpu

SEEDS = list(range(12))


@pytest.mark.parametrize("seed", SEEDS)
def test_random_scene_runs_match_oracle(S, eng, orc, W, seed):
    desc = W.random_scene(seed)
    n, B = 4000, 8
    o, se = oracle_batches(orc, desc, 11, n, B)
    # Monte Carlo standard error of the absorbed total, from the batches
    per = [orc.run(desc, 11, n // B, first=b * (n // B))["absorbed"].sum() for b in range(B)]
    se_abs = float(np.sqrt(B * np.var(per, ddof=1)))
    for prec in ("f64", "f32"):
        g = S.run(desc, 11, n, engine=eng, precision=prec)
        assert g["launched"] == n
        assert abs(identity_residual(g)) <= 1e-9 * n
        diff = abs(g["absorbed"].sum() - o["absorbed"].sum())
        print(f"random {seed} {prec}: absorbed difference {diff:.3f} (SE {se_abs:.3f}), "
              f"interfaces {g['interfaces']} vs {o['interfaces']}")
        if prec == "f64":   # the same walks, up to one packet a rounding flip sends elsewhere
            assert diff <= 1.0 + 1e-9 * n, seed
            assert abs(g["interfaces"] - o["interfaces"]) <= max(2, 2e-3 * o["interfaces"]), seed
        else:               # FP32: 1e-4, or 2 packets per 1e4 where reflections are chaotic
            assert diff <= max(1e-4 * o["absorbed"].sum(), 2.0 * n / 1e4), seed
            assert abs(g["interfaces"] - o["interfaces"]) <= max(5, 0.02 * o["interfaces"]), seed
        check_fluence(g, o, se, desc, "f32", n_batches=B)


@pytest.mark.parametrize("prec,tol,need", [("f64", 1e-6, 0.97), ("f32", 1e-4, 0.97)])
@pytest.mark.parametrize("seed", SEEDS[:6])
def test_random_scene_traces_match_oracle(S, eng, orc, W, seed, prec, tol, need):
    # FP32: the tolerance of the placed and modified shapes' scenes (their
    # rotations, twists and bends round in FP32 at every evaluation)
    desc = W.random_scene(seed)
    n = 128
    g = S.trace(desc, 13, list(range(n)), 40, engine=eng, precision=prec)
    o = [orc.trace(desc, 13, pid, 40) for pid in range(n)]
    mut = [rg["mua"] + rg["mus"] for rg in desc["regions"]]
    frac, worst, bad = compare_traces(o, g, extent_of(S, desc), tol, cap=40, mut=mut)
    print(f"random {seed} {prec}: agree {frac:.4f} worst {worst} first disagreements {bad[:5]}")
    assert frac >= need, (seed, frac, worst, bad[:10])


@pytest.mark.parametrize("seed", SEEDS)
def test_random_scene_voxelises_like_the_oracle(S, eng, orc, W, seed):
    desc = W.random_scene(seed, n_grid=32)
    gv, ov = S.voxelize(desc, engine=eng), orc.voxelize(desc)
    assert len(np.argwhere(gv != ov)) <= max(2, 1e-4 * ov.size), seed


@pytest.mark.parametrize("seed", SEEDS[:6])
def test_random_scene_escape_images(S, eng, orc, W, seed):
    # a 12 x 12 escape image on a face that changes with the seed, against
    # the oracle's on the same packets: per pixel within 3 Monte Carlo SE
    # (floored at one packet's weight), totals within one packet
    from gpu_helpers import batch_se
    desc = W.random_scene(seed)
    desc["detector"] = {"face": seed % 6, "lo": [-1.0, -1.0], "hi": [1.0, 1.0], "dims": [12, 12]}
    n, B = 6000, 8
    imgs = [orc.run(desc, 17, n // B, first=b * (n // B))["image"] for b in range(B)]
    o, se = sum(imgs), batch_se(imgs)
    for prec in ("f64", "f32"):
        g = S.run(desc, 17, n, engine=eng, precision=prec)["image"]
        z = np.abs(g - o) / np.maximum(se, 1.0)
        print(f"random {seed} face {seed % 6} {prec}: image total {g.sum():.3f} vs {o.sum():.3f}, "
              f"pixels within 3 SE {np.mean(z <= 3):.4f}")
        assert np.mean(z <= 3.0) >= 0.99, seed
        assert abs(g.sum() - o.sum()) <= 1.0 + 1e-9 * n or prec == "f32" and abs(g.sum() - o.sum()) <= 3.0, seed


@pytest.mark.parametrize("seed", SEEDS[:6])
def test_random_scene_relaxed_runs_match_oracle(S, eng, orc, W, seed):
    # over-relaxed steps (w = 1.9) on the random scenes: the FP64 walk takes
    # the plain march's decisions (to one packet where distances are bounds)
    desc = dict(W.random_scene(seed), relax=1.9)
    n = 3000
    o = orc.run(W.random_scene(seed), 23, n)
    g = S.run(desc, 23, n, engine=eng, precision="f64")
    assert abs(g["absorbed"].sum() - o["absorbed"].sum()) <= 1.0 + 1e-9 * n, seed
    assert abs(g["interfaces"] - o["interfaces"]) <= max(2, 2e-3 * o["interfaces"]), seed
    assert abs(identity_residual(g)) <= 1e-9 * n
    # FP32 with over-relaxed steps: as the plain FP32 walk on these scenes
    # (1e-4, or 2 packets per 1e4 where reflections are chaotic)
    g = S.run(desc, 23, n, engine=eng, precision="f32")
    diff = abs(g["absorbed"].sum() - o["absorbed"].sum())
    assert diff <= max(1e-4 * o["absorbed"].sum(), 2.0 * n / 1e4), (seed, diff)
    assert abs(g["interfaces"] - o["interfaces"]) <= max(5, 0.02 * o["interfaces"]), seed
    assert abs(identity_residual(g)) <= 1e-9 * n


def _with_union(desc):
    """The scene itself when it has a union region of several primitives;
    else its first two inner regions merged into one union (the first's
    properties), so every seed has a region to accelerate."""
    if any(rg["op"] == "union" and len(rg["prims"]) >= 2 for rg in desc["regions"]):
        return desc
    r = [dict(rg) for rg in desc["regions"]]
    r[1] = dict(r[1], prims=r[1]["prims"] + r[2]["prims"], op="union", k=0.0)
    del r[2]
    return dict(desc, regions=r)


@pytest.mark.parametrize("seed", SEEDS)
def test_random_scene_acceleration_grid(S, eng, W, seed):
    # the uniform grid over a union region of placed and modified primitives
    # changes how far steps go, never a decision
    desc = _with_union(W.random_scene(seed))
    assert any(rg["op"] == "union" and len(rg["prims"]) >= 2 for rg in desc["regions"])
    desc = dict(desc, accel_cells=[8, 8, 8])   # the binding takes the union region with most primitives
    plain = S.run(dict(desc, accel_cells=None), 29, 3000, engine=eng, precision="f64")
    accel = S.run(desc, 29, 3000, engine=eng, precision="f64")
    for k in ("interactions", "interfaces", "reflections", "refractions", "kills", "escapes"):
        assert abs(accel[k] - plain[k]) <= max(1, 1e-3 * plain[k]), (seed, k, accel[k], plain[k])
    assert abs(accel["absorbed"].sum() - plain["absorbed"].sum()) <= 1.0 + 1e-9 * 3000
