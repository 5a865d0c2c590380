"""The z-score summary that bench.py reports beside the headline fluence
error, checked with the oracle standing in for the GPU runner: batches of
the oracle over the oracle's own packets must sum to its run (chi-square per
degree of freedom near 0), an independent packet range must look like the
same distribution (near 1), and a tally 10 % too large must not."""
import numpy as np
import pytest

import bench


class _OracleRunner:
    """The one call fluence_z_scores makes of the binding, served by the
    oracle (optionally with every tally scaled)."""

    def __init__(self, orc, scale=1.0):
        self.orc, self.scale = orc, scale

    def run(self, desc, seed, n, first=0, engine=None, precision=None):
        r = self.orc.run(desc, seed, n, first=first)
        return {"fluence_raw": self.scale * r["fluence_raw"]}


@pytest.mark.parametrize("name,ng,n", [("sphere", 24, 40000), ("cylinder", 32, 20000)])
def test_fluence_z_scores_on_the_oracle(orc, W, name, ng, n):
    d = W.WORKLOADS[name](n_grid=ng)
    Fo = orc.run(d, 0, n)["fluence_raw"]
    z = bench.fluence_z_scores(_OracleRunner(orc), d, None, "f64", d, n, Fo)
    same, ind = z["same_packets"], z["independent_packets"]
    assert same["within_3se"] == 1.0 and same["chi2_per_dof"] < 1e-6, same
    assert ind["voxels"] >= 2000, ind
    assert ind["within_3se"] >= 0.99 and 0.9 <= ind["chi2_per_dof"] <= 1.1, ind
    bad = bench.fluence_z_scores(_OracleRunner(orc, 1.1), d, None, "f64", d, n, Fo)["independent_packets"]
    assert bad["chi2_per_dof"] > 1.2, bad  # outside the [0.9, 1.1] the bench reads as agreement
