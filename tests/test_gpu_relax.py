"""GPU over-relaxed sphere tracing against the oracle's plain march (same
packets: relaxed steps change no event), its step counts against the
oracle's mirror of the same rule, and its closed forms on the GPU: a thin
plate that one relaxed step would jump is crossed through both faces, a
grazing beam takes about 1/w as many steps, and relaxed runs tally what
plain runs tally.  Same tolerances as the plain walk's parity tests."""
import math

import numpy as np
import pytest

from gpu_helpers import absorbed_agrees, check_fluence, compare_traces, extent_of, identity_residual, mirror, oracle_batches

pytestmark = pytest.mark.gpu

W_RELAX = 1.9


def _relaxed(desc, w=W_RELAX):
    return dict(desc, relax=w)


@pytest.mark.parametrize("prec,need", [("f64", 0.99), ("f32", 0.97)])
@pytest.mark.parametrize("name", ["slab", "cylinder", "glass_sphere", "bottle"])
def test_relaxed_traces_match_oracle(S, eng, orc, W, name, prec, need):
    plain = W.WORKLOADS[name](n_grid=32)
    desc = _relaxed(plain)
    tol = 1e-6 if prec == "f64" else 1e-5
    n, seed = 256, 777
    g = S.trace(desc, seed, list(range(n)), 50, engine=eng, precision=prec)
    o = [orc.trace(plain, seed, pid, 50) for pid in range(n)]
    mut = [rg["mua"] + rg["mus"] for rg in desc["regions"]]
    frac, worst, bad = compare_traces(o, g, extent_of(S, desc), tol, mut=mut)
    print(f"{name} {prec}: agree {frac:.4f} worst {worst} first disagreements {bad[:5]}")
    assert frac >= need, (frac, worst, bad[:10])


@pytest.mark.parametrize("prec,abs_tol", [("f64", 1e-9), ("f32", 1e-4)])
@pytest.mark.parametrize("name", ["slab", "bottle"])
def test_relaxed_run_parity(S, eng, orc, W, name, prec, abs_tol):
    plain = W.WORKLOADS[name](n_grid=48)
    desc = _relaxed(plain)
    n, seed = 10000, 99
    o, se = oracle_batches(orc, plain, seed, n, 10)
    g = S.run(desc, seed, n, engine=eng, precision=prec)
    assert g["launched"] == n
    assert abs(identity_residual(g)) <= 1e-9 * n
    diff = abs(g["absorbed"].sum() - o["absorbed"].sum())
    rel = diff / o["absorbed"].sum()
    print(f"{name} {prec}: absorbed relative difference {rel:.3e}, steps {g['steps']} vs oracle {o['steps']}")
    assert absorbed_agrees(g["absorbed"].sum(), o["absorbed"].sum(), n, prec, name), (rel, diff)
    if prec == "f64":
        assert g["interfaces"] == o["interfaces"]
        m = orc.run(mirror(desc), seed, n, with_grid=False)   # the same rule's step count
        assert m["steps"] < o["steps"]
        assert abs(g["steps"] - m["steps"]) <= 1e-4 * m["steps"]
    check_fluence(g, o, se, desc, prec)


def test_relaxed_and_plain_runs_agree(S, eng, W):
    # same packets, relaxed or not: every tally but the step count agrees,
    # and the relaxed run takes fewer steps
    desc = W.WORKLOADS["glass_sphere"](n_grid=32)
    a = S.run(desc, 5, 50000, engine=eng, precision="f64")
    b = S.run(_relaxed(desc), 5, 50000, engine=eng, precision="f64")
    assert a["interactions"] == b["interactions"] and a["interfaces"] == b["interfaces"]
    np.testing.assert_allclose(b["absorbed"], a["absorbed"], rtol=1e-7)
    np.testing.assert_allclose(b["escaped_face"], a["escaped_face"], rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(b["fluence_raw"], a["fluence_raw"], rtol=1e-4, atol=1e-6 * a["fluence_raw"].max())
    assert b["steps"] < 0.9 * a["steps"], (b["steps"], a["steps"])


@pytest.mark.parametrize("u,thick", [([0.0, 0.0, -1.0], 0.05), ([0.98, 0.0, -0.2], 0.02)])
def test_relaxed_step_does_not_jump_a_thin_plate_on_gpu(S, eng, W, u, thick):
    mua = 5.0
    prims = [{"kind": "box", "c": [0.0, 0.0, 0.0], "half": [5.0, 5.0, 0.5 * thick]}]
    regions = [W._region([0], mua, 0.0, 0.0, 1.0)]
    sc = W._scene("thin_plate", prims, regions, None, None, pad=2.0)
    uu = np.asarray(u, float) / np.linalg.norm(u)
    sc["source"] = {"kind": "pencil", "p": (-1.5 * uu).tolist(), "u": uu.tolist()}
    N = 1_000_000
    g = S.run(_relaxed(sc), 6, N, engine=eng, precision="f32", tally=False)
    want = math.exp(-mua * thick / abs(uu[2]))
    assert g["interfaces"] == N + g["escapes"]
    assert abs(g["escaped_face"].sum() / N - want) < 4 * math.sqrt(want * (1 - want) / N)


def test_relaxed_grazing_beam_steps_on_gpu(S, eng, W):
    # a beam skimming 0.01 cm under the top face of a clear, index-matched
    # 10 cm block
    prims = [{"kind": "box", "c": [0.0, 0.0, -0.5], "half": [5.0, 5.0, 0.5]}]
    regions = [W._region([0], 1e-4, 0.0, 0.0, 1.0)]
    sc = W._scene("graze", prims, regions, None, None, pad=0.5)
    sc["source"] = {"kind": "pencil", "p": [-5.2, 0.0, -0.01], "u": [1.0, 0.0, 0.0]}
    for prec in ("f64", "f32"):
        plain = S.run(sc, 1, 1000, engine=eng, precision=prec, tally=False)
        relaxed = S.run(_relaxed(sc), 1, 1000, engine=eng, precision=prec, tally=False)
        assert plain["escaped_face"][1] >= 990.0 and abs(relaxed["escaped_face"][1] - plain["escaped_face"][1]) <= 1.0
        assert relaxed["steps"] < 0.6 * plain["steps"], (prec, relaxed["steps"], plain["steps"])


@pytest.mark.parametrize("name,relax", [("slab", 1.0), ("cylinder", 1.0), ("slab", 1.9)])
def test_fp64_evaluations_match_oracle(S, eng, orc, W, name, relax):
    # free-flight reuse and relaxed steps decide the same way on both sides:
    # the FP64 walk makes the oracle's number of SDF evaluations
    desc = dict(W.WORKLOADS[name](n_grid=16), relax=relax)
    g = S.run(desc, 21, 3000, engine=eng, precision="f64", tally=False)
    o = orc.run(mirror(desc), 21, 3000)
    assert g["interactions"] == o["interactions"]
    assert abs(g["steps"] - o["steps"]) <= 1e-5 * o["steps"], (g["steps"], o["steps"])
