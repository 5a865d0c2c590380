"""GPU parity of the further gallery shapes (Sec. 2.2: capped cone,
octahedron, hexagonal prism, ellipsoid, and a bent rod) against the oracle
on a scene holding all five, and escape closed forms on the GPU.  Same tolerances
as the SDF walk's parity tests.  The scene's glass shapes make long
chains of internal reflections, a chaotic billiard: FP32 runs have the
allowance of gpu_helpers.absorbed_agrees.  The ellipsoid's distance is a
bound, so in FP64 an interface hit can land up to delta apart from the
oracle's (a step more or less): FP64 runs are held to one packet's weight."""
import math

import numpy as np
import pytest

from gpu_helpers import absorbed_agrees, check_fluence, compare_traces, extent_of, identity_residual, oracle_batches

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,need", [("f64", 0.99), ("f32", 0.97)])
def test_shapes_traces_match_oracle(S, eng, orc, W, prec, need):
    desc = W.shapes_scene(n_grid=32)
    tol = 1e-6 if prec == "f64" else 1e-4
    n, seed = 256, 1618
    g = S.trace(desc, seed, list(range(n)), 50, engine=eng, precision=prec)
    o = [orc.trace(desc, seed, pid, 50) for pid in range(n)]
    mut = [rg["mua"] + rg["mus"] for rg in desc["regions"]]
    frac, worst, bad = compare_traces(o, g, extent_of(S, desc), tol, mut=mut)
    print(f"shapes {prec}: agree {frac:.4f} worst {worst} first disagreements {bad[:5]}")
    assert frac >= need, (frac, worst, bad[:10])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_shapes_run_parity(S, eng, orc, W, prec):
    desc = W.shapes_scene(n_grid=48)
    n, seed = 10000, 27
    o, se = oracle_batches(orc, desc, seed, n, 10)
    g = S.run(desc, seed, n, engine=eng, precision=prec)
    assert g["launched"] == n
    assert abs(identity_residual(g)) <= 1e-9 * n
    diff = abs(g["absorbed"].sum() - o["absorbed"].sum())
    print(f"shapes {prec}: absorbed relative difference {diff / o['absorbed'].sum():.3e}")
    if prec == "f32":
        assert absorbed_agrees(g["absorbed"].sum(), o["absorbed"].sum(), n, prec, "shapes"), diff
    else:
        assert diff <= 1.0
    assert abs(g["interfaces"] - o["interfaces"]) <= 1e-3 * o["interfaces"]
    check_fluence(g, o, se, desc, "f32")


def test_shapes_voxelise_like_the_oracle(S, eng, orc, W):
    desc = W.shapes_scene(n_grid=48)
    gv, ov = S.voxelize(desc, engine=eng), orc.voxelize(desc)
    assert len(np.argwhere(gv != ov)) <= max(2, 1e-4 * ov.size)
    assert set(np.unique(gv)) == {0, 1, 2, 3, 4, 5}


def _fib(n):
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    phi = math.pi * (1 + 5 ** 0.5) * i
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def test_octahedron_and_hexprism_escape_on_gpu(S, eng, W):
    N, mua = 1_000_000, 2.0
    u = _fib(200000)
    cases = []
    s = 0.6
    cases.append(({"kind": "octahedron", "c": [0, 0, 0], "s": s}, s / np.abs(u).sum(1)))
    h, hz = 0.4, 0.3
    nrm = np.array([[math.cos(a), math.sin(a)] for a in (math.pi / 6 + k * math.pi / 3 for k in range(6))])
    dots = u[:, :2] @ nrm.T
    t = np.minimum(hz / np.maximum(np.abs(u[:, 2]), 1e-300),
                   np.min(np.where(dots > 0, h / np.maximum(dots, 1e-300), np.inf), axis=1))
    cases.append(({"kind": "hexprism", "c": [0, 0, 0], "h": h, "hz": hz}, t))
    for prim, texit in cases:
        sc = W._scene("one", [prim], [W._region([0], mua, 0.0, 0.0, 1.0)], {"kind": "point", "p": [0.0, 0.0, 0.0]}, None)
        g = S.run(sc, 11, N, engine=eng, precision="f32", tally=False)
        want = float(np.mean(np.exp(-mua * texit)))
        got = g["escaped_face"].sum() / N
        assert abs(got - want) < 4 * math.sqrt(want * (1 - want) / N), (prim["kind"], got, want)
