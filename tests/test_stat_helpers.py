"""The statistical comparison the GPU parity tests use on independent
samples (gpu_helpers.independent_fluence_check), checked on the oracle
itself: two disjoint packet-id ranges of the same scene are two samples of
one distribution and must pass (fraction within 3 SE and chi-square per
degree of freedom near 1); a sample scaled by 1.1 -- a 10 % error in the
tally -- must fail."""
import pytest

from gpu_helpers import independent_fluence_check


@pytest.mark.parametrize("name,ng,N", [("sphere", 24, 40000), ("cylinder", 32, 20000)])
def test_independent_check_accepts_two_samples_of_one_walk(orc, W, name, ng, N):
    d = W.WORKLOADS[name](n_grid=ng)
    B, st = 20, N // 20
    a = [orc.run(d, 5, st, first=b * st)["fluence_raw"] for b in range(B)]
    c = [orc.run(d, 5, st, first=N + b * st)["fluence_raw"] for b in range(B)]
    independent_fluence_check(c, a)
    with pytest.raises(AssertionError):
        independent_fluence_check([1.1 * x for x in c], a)
