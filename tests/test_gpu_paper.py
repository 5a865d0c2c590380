"""GPU runs of the paper's validation experiment E1 and of the tally-free
mode its speed test uses.

- Tally-free runs (no fluence buffer) walk the same packets as tallied runs:
  every scalar tally is the same, in both geometry models.
- The isotropic scattering sphere of Eq. 4 over the optical depths the
  paper sweeps: FP64 runs agree with the oracle packet for packet (same
  scattering counts, escapes to 1e-9), and the mean number of scatterings
  meets Eq. 4 in its thick limit and the first-flight probability in its
  thin limit.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _close_scalars(a, b, rtol):
    np.testing.assert_allclose(a["absorbed"], b["absorbed"], rtol=rtol)
    np.testing.assert_allclose(a["escaped_face"], b["escaped_face"], rtol=rtol, atol=1e-12)
    for k in ("launched", "interactions", "interfaces", "reflections", "refractions", "kills", "escapes", "steps"):
        assert a[k] == b[k], k


@pytest.mark.parametrize("geometry", ["sdf", "voxel"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tally_free_run_walks_the_same_packets(S, eng, W, geometry, prec):
    desc = dict(W.cylinder_scene(n_grid=48), geometry=geometry)
    with_tally = S.run(desc, 7, 20000, engine=eng, precision=prec)
    free = S.run(desc, 7, 20000, engine=eng, precision=prec, tally=False)
    assert free["fluence_raw"] is None and with_tally["fluence_raw"].sum() > 0
    assert free["voxel_pieces"] == 0 and with_tally["voxel_pieces"] > 0
    _close_scalars(free, with_tally, 1e-11 if prec == "f64" else 1e-6)


@pytest.mark.parametrize("tau,n", [(0.1, 20000), (1.0, 20000), (10.0, 4000), (100.0, 200)])
def test_eq4_sweep_matches_oracle(S, eng, orc, W, tau, n):
    desc = W.scattering_sphere(tau)
    g = S.run(desc, 2112, n, engine=eng, precision="f64", tally=False)
    o = orc.run(desc, 2112, n)
    assert g["interactions"] == o["interactions"]
    np.testing.assert_allclose(g["escaped_face"], o["escaped_face"], rtol=1e-9, atol=1e-9)
    assert g["absorbed"].sum() == 0.0


def test_eq4_thin_limit_on_gpu(S, eng, W):
    tau, N = 0.01, 1_000_000
    g = S.run(W.scattering_sphere(tau), 17, N, engine=eng, precision="f32", tally=False)
    first = 1 - math.exp(-tau)  # exact first-flight probability
    assert abs(g["interactions"] / N - first) < 4 * math.sqrt(first / N) + tau * tau


# Eq. 4 is the diffusion-limit estimate: 6 % above the exact mean at tau = 10
# (the oracle gives 56.4 against 60), under 2 % at tau = 100
@pytest.mark.parametrize("tau,N,rel", [(10.0, 200_000, 0.10), (100.0, 20_000, 0.03)])
def test_eq4_thick_limit_on_gpu(S, eng, W, tau, N, rel):
    g = S.run(W.scattering_sphere(tau), 18, N, engine=eng, precision="f32", tally=False)
    assert g["interactions"] / N == pytest.approx(tau * tau / 2 + tau, rel=rel)
