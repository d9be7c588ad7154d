"""Section 5.2 studies on the GPU path, small: both tests are valid under the null
(near-uniform p-values, type-I error near the level) and both detect a clear
alternative."""
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
