"""Section 5.2 studies on the GPU path, small: both tests are valid under the null
(near-uniform p-values, type-I error near the level), both detect a clear alternative,
and the first replications of each study equal the FP64 oracle's efficient permutation
test and cross-ED test on the same data."""
import numpy as np
import pytest
from scipy.stats import kstest

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_null_p_values_uniform_for_both_tests():
    from paper_2406_06488_amd import studies
    say("studies: null, 300 replications")
    e, c = studies.pvalues(60, 60, 20, 300, B=200, seed=5)
    for name, p in (("efficient", e), ("cross", c)):
        assert kstest(p, "uniform").pvalue > 1e-3, name
        assert abs(np.mean(p <= 0.05) - 0.05) < 0.05, name


def test_both_tests_detect_a_clear_alternative():
    from paper_2406_06488_amd import studies
    say("studies: alternative, 100 replications")
    e, c = studies.pvalues(150, 150, 50, 100, j=10, eps=0.5, B=200, seed=6)
    assert np.mean(e <= 0.05) > 0.95 and np.mean(c <= 0.05) > 0.9


@pytest.mark.parametrize("eps", [0.0, 0.5])
def test_study_replications_match_the_oracle(eps):
    """The first replications of a null and of an alternative study, against the oracle's
    efficient permutation test (same split seed) and cross-ED test on the same data (FP32
    form: statistic within 1e-5; exceedance counts equal except for splits within 1e-5 of
    the threshold; cross-ED p-values within 1e-5)."""
    import oracle
    from paper_2406_06488_amd import studies
    say("studies: oracle check, eps %g" % eps)
    res, cross, kept = studies.pvalues(90, 70, 30, 6, j=10, eps=eps, B=200, seed=9, keep=6,
                                       detail=True)
    assert len(kept) == 6
    for r, c, (X, Y, sd) in zip(res, cross, kept):
        o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), 200, sd, oracle.ED)
        ps, thr = o["perm_stats"], o["threshold"]
        floor = float(np.mean(np.abs(ps)))
        assert abs(r["statistic"] - o["statistic"]) <= 1e-5 * max(abs(o["statistic"]), floor)
        near = int(np.sum(np.abs(ps - thr) <= 1e-5 * max(abs(thr), floor)))
        assert abs(r["count_ge"] - o["count_ge"]) <= near, (r, o["count_ge"], near)
        if near == 0:
            assert r["p_value"] == o["p_value"]
        oc = oracle.cross(X.astype(np.float64), Y.astype(np.float64), oracle.ED)
        assert abs(c - oc["p_value"]) <= 1e-5, (c, oc["p_value"])
