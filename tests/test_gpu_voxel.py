"""GPU parity of the voxelised comparison model (Sec. 3): the device
voxelisation and the voxel walk, through the C ABI, against the oracle's
voxel model on shared seeds, plus its closed forms and batching with SDF
jobs.

Tolerances are those of the SDF walk's parity tests: FP64 transport to
1e-6 relative per event record, 1e-9 on totals; FP32 to 1e-5 per record
for 97% of packets, 1e-4 on totals, fluence within 3 Monte Carlo SE.
Voxelisation is an integer result decided in FP64 on both sides; it must
agree exactly except at voxel centres that lie on a surface to rounding,
where either region is a correct reading.
"""
import math

import numpy as np
import pytest

from gpu_helpers import check_fluence, compare_traces, extent_of, identity_residual, oracle_batches

pytestmark = pytest.mark.gpu


def _vox(desc):
    return dict(desc, geometry="voxel")


def _scenes(W):
    return {
        "sphere": W.sphere_scene(n_grid=24),
        "cylinder": W.cylinder_scene(n_grid=32),
        "stack": W.stack_scene([(0.1, 1.0, 1.5), (0.2, 0.5, 1.4), (0.3, 0.2, 1.4)], nz=12),
        "vessels": W.vessel_scene(7, 1.0, n_caps=150, n_grid=24),
    }


@pytest.mark.parametrize("name", ["sphere", "cylinder", "stack", "vessels"])
def test_voxelize_matches_oracle(S, eng, orc, W, name):
    desc = _scenes(W)[name]
    g = S.voxelize(desc, engine=eng)
    o = orc.voxelize(desc)
    assert g.shape == o.shape
    bad = np.argwhere(g != o)
    print(f"{name}: {len(bad)} of {o.size} voxels differ")
    assert len(bad) <= max(2, 1e-4 * o.size)
    lo, hi = np.array(desc["grid"]["lo"]), np.array(desc["grid"]["hi"])
    d = (hi - lo) / np.array(desc["grid"]["dims"])
    for k, j, i in bad:
        c = lo + (np.array([i, j, k]) + 0.5) * d
        dmin = min(abs(orc.region_sdf(desc, r, c)) for r in range(len(desc["regions"])))
        assert dmin < 1e-12, (i, j, k, dmin)
    assert len(np.unique(g)) > 1


@pytest.mark.parametrize("prec,need", [("f64", 0.99), ("f32", 0.97)])
@pytest.mark.parametrize("name", ["sphere", "cylinder", "stack", "vessels"])
def test_voxel_traces_match_oracle(S, eng, orc, W, name, prec, need):
    desc = _scenes(W)[name]
    tol = 1e-6 if prec == "f64" else 1e-5
    n, seed = 256, 31337
    g = S.trace(_vox(desc), seed, list(range(n)), 50, engine=eng, precision=prec)
    o = [orc.trace(desc, seed, pid, 50, voxel=True) for pid in range(n)]
    mut = [rg["mua"] + rg["mus"] for rg in desc["regions"]]
    frac, worst, bad = compare_traces(o, g, extent_of(S, desc), tol, mut=mut)
    print(f"{name} {prec}: agree {frac:.4f} worst {worst} first disagreements {bad[:5]}")
    assert frac >= need, (frac, worst, bad[:10])


@pytest.mark.parametrize("prec,abs_tol", [("f64", 1e-9), ("f32", 1e-4)])
def test_voxel_run_parity(S, eng, orc, W, prec, abs_tol):
    """Curved scene at 64^3 (several voxels per vessel radius, a ragged
    disc beam entering the grid from outside)."""
    desc = W.cylinder_scene(n_grid=64)
    n, seed = 10000, 2718
    o, se = oracle_batches(orc, desc, seed, n, 10, voxel=True)
    g = S.run(_vox(desc), seed, n, engine=eng, precision=prec)
    assert g["launched"] == n
    assert abs(identity_residual(g)) <= 1e-9 * n
    diff = abs(g["absorbed"].sum() - o["absorbed"].sum())
    rel = diff / o["absorbed"].sum()
    print(f"{prec}: absorbed relative difference {rel:.3e} ({diff:.3e} in packet weights)")
    assert rel <= abs_tol
    assert np.allclose(g["escaped_face"], o["escaped_face"], rtol=10 * abs_tol, atol=1e-9 * n if prec == "f64" else 1.0)
    if prec == "f64":
        assert g["interfaces"] == o["interfaces"]
    check_fluence(g, o, se, desc, prec)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_voxel_beer_lambert_on_gpu(S, eng, W, prec):
    mua, L, n = 2.0, 0.5, 1.5
    N = 1000000
    g = S.run(_vox(W.beer_lambert_slab(mua, L, n)), 5, N, engine=eng, precision=prec)
    R = ((n - 1) / (n + 1)) ** 2
    e = math.exp(-mua * L)
    T = (1 - R) ** 2 * e / (1 - R * R * e * e)
    Rt = R + R * (1 - R) ** 2 * e * e / (1 - R * R * e * e)
    for got, want in ((g["escaped_face"][4] / N, T), (g["escaped_face"][5] / N, Rt)):
        assert abs(got - want) < 4 * math.sqrt(want * (1 - want) / N)
    assert g["escaped_face"][:4].sum() == 0


def _close(a, b, rtol):
    np.testing.assert_allclose(a["absorbed"], b["absorbed"], rtol=rtol)
    np.testing.assert_allclose(a["escaped_face"], b["escaped_face"], rtol=rtol, atol=1e-12)
    np.testing.assert_allclose(a["fluence_raw"], b["fluence_raw"], rtol=rtol, atol=1e-12)
    for k in ("launched", "interactions", "interfaces", "voxel_pieces", "kills"):
        assert a[k] == b[k], k


@pytest.mark.parametrize("graph", [0, 1])
def test_mixed_geometry_batch_equals_runs_alone(S, W, graph):
    """SDF and voxel jobs in one batch: the launch runs one kernel per
    geometry over the shared job table; each job equals its run alone,
    also when the sequence is captured and replayed."""
    import torch
    descs = [W.sphere_scene(n_grid=20), _vox(W.cylinder_scene(n_grid=32)), _vox(W.slab_scene(n_grid=24)),
             W.vessel_scene(3, 0.7, n_caps=200, n_grid=16), _vox(W.sphere_scene(n_grid=20))]
    seeds = [21, 22, 23, 24, 25]
    ns = [8000, 3000, 2000, 1500, 8000]
    e = S.Engine(0, precision="f64", use_graph=graph)
    e_alone = S.Engine(0)
    scenes = [S.Scene(d) for d in descs]
    for rep in range(2 if graph else 1):
        outs = S.launch_batch(e, scenes, seeds, ns)
        torch.cuda.synchronize()
        for sc, sd, n, b in zip(scenes, seeds, ns, outs):
            alone = S.run(sc, sd, n, engine=e_alone, precision="f64")
            _close(b.host(), alone, 1e-11)
    e.close()
    e_alone.close()


def test_voxel_model_converges_with_resolution(S, eng, W):
    """The paper's accuracy comparison in miniature: on the curved vessel
    scene the voxel model's absorbed energy approaches the SDF model's as
    the grid refines (same packets, same seeds)."""
    N, seed = 200000, 5
    sdf = S.run(W.cylinder_scene(n_grid=64), seed, N, engine=eng, precision="f32")["absorbed"] / N
    err = {}
    for ng in (16, 128):
        v = S.run(_vox(W.cylinder_scene(n_grid=ng)), seed, N, engine=eng, precision="f32")["absorbed"] / N
        err[ng] = float(np.abs(v - sdf).sum())
    print("voxel-model absorbed error vs SDF:", err)
    assert err[128] < 0.5 * err[16]
