"""Host pieces of the Section 5.2 studies: the bootstrap spread drawn around the power
curves (one standard deviation of the power estimate over 200 resamples of the
replications)."""
import numpy as np

from paper_2406_06488_amd import studies


def test_bootstrap_sd_matches_the_binomial_standard_error():
    # the bootstrap SD of a mean of n 0/1 outcomes with mean m tends to sqrt(m (1 - m) / n);
    # with 200 resamples the estimate itself is within about 5 % of it (20 % allowed)
    g = np.random.Generator(np.random.PCG64(11))
    for n, m in ((500, 0.3), (500, 0.9), (200, 0.5)):
        hits = g.random(n) < m
        mh = hits.mean()
        ref = np.sqrt(mh * (1 - mh) / n)
        sd = studies.bootstrap_sd(hits, nboot=200, seed=3)
        assert abs(sd - ref) < 0.2 * ref, (n, m, sd, ref)


def test_bootstrap_sd_of_constant_outcomes_is_zero_and_seeded():
    assert studies.bootstrap_sd(np.ones(100, dtype=bool)) == 0.0
    assert studies.bootstrap_sd(np.zeros(50, dtype=bool)) == 0.0
    h = np.arange(100) % 3 == 0
    assert studies.bootstrap_sd(h, seed=7) == studies.bootstrap_sd(h, seed=7)
    assert studies.bootstrap_sd(h, seed=7) != studies.bootstrap_sd(h, seed=8)
