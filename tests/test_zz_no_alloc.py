"""smcrt_run_ex_static (the run that allocates no device memory: its scratch
is a fixed device array) against smcrt_run_ex on the same scenes, seeds and
packets, through the C ABI.  Two calls in a row, the second with a smaller
input, so the second runs in scratch the first left behind.  The walks are
the same kernels: counts of events, steps and voxel pieces agree exactly;
absorbed, escaped and fluence to the order of FP64 sums (the static run
tallies straight into the caller's grid, smcrt_run_ex into bricks for FP32
cubic voxels).  Scenes: an accelerated vessel network (grid-build buffers in
the scratch) and the voxel model (region grid in the scratch), then a small
sphere and a small slab.  A scene that needs more scratch than the array is
refused before any work is queued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(S, eng, sc, seed, n, static):
    import torch
    out = S.Outputs(sc, eng.device)
    fn = S.smcrt_run_ex_static if static else S.smcrt_run_ex
    fn(eng.h, sc.h, seed, 0, n, out.struct(), S._stream_ptr(None))
    torch.cuda.synchronize()
    return out.host()


def _same(a, b):
    for k in ("launched", "interactions", "interfaces", "reflections", "refractions", "crossings", "kills",
              "escapes", "stalls", "steps", "voxel_pieces"):
        assert a[k] == b[k], k
    np.testing.assert_allclose(a["absorbed"], b["absorbed"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(a["escaped_face"], b["escaped_face"], rtol=1e-12, atol=1e-12)
    if b["fluence_raw"] is not None:
        F, G = a["fluence_raw"], b["fluence_raw"]
        np.testing.assert_allclose(F, G, rtol=1e-9, atol=1e-12 * G.max())
        assert G.sum() > 0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_static_run_equals_run_ex_twice(S, W, prec):
    eng = S.Engine(0, precision=prec)
    try:
        pairs = [
            (W.vessel_scene(7, 1.0, n_caps=300, n_grid=48), 5000),
            (W.vessel_scene(8, 0.7, n_caps=120, n_grid=24), 2000),   # smaller: the scratch holds the first's leftovers
            (dict(W.cylinder_scene(n_grid=96), geometry="voxel"), 20000),
            (dict(W.cylinder_scene(n_grid=40), geometry="voxel"), 3000),
            (W.sphere_scene(n_grid=40), 20000),
            (W.slab_scene(n_grid=16), 1000),
        ]
        for desc, n in pairs:
            sc = S.Scene(desc)
            print(f"{prec} {desc['name']} {desc.get('geometry', 'sdf')} n={n}", flush=True)
            a = _run(S, eng, sc, 77, n, static=True)
            b = _run(S, eng, sc, 77, n, static=False)
            _same(a, b)
    finally:
        eng.close()


def test_static_run_refuses_a_scene_beyond_its_scratch(S, W):
    import torch
    eng = S.Engine(0)
    try:
        big = S.Scene(dict(W.cylinder_scene(n_grid=8), geometry="voxel",
                           grid={"lo": [-0.5] * 3, "hi": [0.5] * 3, "dims": [512, 512, 160]}))
        out = S.Outputs(big, 0, tally=False)
        with pytest.raises(S.SmcrtError, match="static scratch"):
            S.smcrt_run_ex_static(eng.h, big.h, 1, 0, 10, out.struct(), S._stream_ptr(None))
        torch.cuda.synchronize()
        assert out.host()["launched"] == 0      # nothing was queued
    finally:
        eng.close()
