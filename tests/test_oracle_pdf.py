"""Pins of the oracle's velocity statistics (Test 7, Fig. 8) against what
does not depend on it: the velocity an equilibrium state carries by
construction, scipy's sample moments, and numpy's edge-based histogram."""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle import pdf as P
from paper_2602_16486_amd import workloads as W


@pytest.mark.parametrize("q,shape", [(9, (12, 7)), (27, (5, 4, 3))])
def test_velocity_of_an_equilibrium_is_its_velocity(q, shape):
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, 3, umax=0.04, dims=2 if q == 9 else 3)
    f = O.init_equilibrium(q, n, rho=rho, u=u)
    assert np.abs(P.velocity(q, f) - u).max() < 1e-15


def test_moments_match_scipy():
    rng = np.random.default_rng(5)
    u = np.stack([rng.normal(0.1, 2.0, 5000), rng.exponential(1.0, 5000), rng.uniform(-1, 1, 5000)])
    m = P.velocity_moments(u)
    for a in range(3):
        assert np.isclose(m[a, 0], np.mean(u[a]), rtol=1e-13)
        assert np.isclose(m[a, 1], np.var(u[a]), rtol=1e-13)
        assert np.isclose(m[a, 2], stats.skew(u[a]), rtol=1e-10)
        assert np.isclose(m[a, 3], stats.kurtosis(u[a], fisher=False), rtol=1e-10)
    # exponential: skewness 2, kurtosis 9; uniform: 0 and 9/5 (large-sample)
    assert abs(m[1, 2] - 2) < 0.3 and abs(m[2, 3] - 1.8) < 0.05


def test_histogram_matches_numpy_edges():
    rng = np.random.default_rng(6)
    u = np.stack([rng.normal(0, 1e-2, 4000), rng.standard_t(3, 4000), np.zeros(4000)])
    counts, xs = P.velocity_histogram(u, 2, 30, 3.0)
    for a in range(2):
        edges = np.linspace(-3.0, 3.0, 31)
        h, _ = np.histogram(xs[a], bins=edges)
        assert np.array_equal(counts[a, 1:-1], h)
        assert counts[a, 0] == np.sum(xs[a] < -3.0)
        assert counts[a, -1] == np.sum(xs[a] >= 3.0)
        assert counts[a].sum() == 4000
    assert not counts[2].any()
