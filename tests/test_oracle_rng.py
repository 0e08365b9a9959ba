"""Pins of the oracle's random numbers: Philox4x32-10 against its published
known-answer vectors, and the distribution of the derived move quantities
(particle index, Metropolis variable, Gaussian displacement; Sec. 2, Sec. 5.1)."""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from conftest import read_golden


def test_philox_known_answers():
    rows = read_golden("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        assert O.philox(w[0:4], w[4:6]) == tuple(w[6:10])


def _draws(n, count, sigma=1.0, order=0, seed=1, t=3, w=5):
    sys_ = O.system(n, 10.0, 2.9, step_sigma=sigma, seed=seed, order=order)
    s = np.zeros(count, np.int64)
    xi = np.zeros(count)
    d = np.zeros((count, 3))
    for i in range(count):
        s[i], xi[i], d[i] = O.draw_move(sys_, i % 4096, t + i // 4096, w)
    return s, xi, d


def test_move_index_uniform_and_in_range():
    n = 37
    s, _, _ = _draws(n, 40000)
    assert s.min() >= 0 and s.max() < n
    counts = np.bincount(s, minlength=n)
    p = stats.chisquare(counts).pvalue
    assert p > 1e-3, p


def test_sequential_order_is_micro_step():
    sys_ = O.system(11, 10.0, 2.9, step_sigma=1.0, order=1)
    for k in range(40):
        assert O.draw_move(sys_, k, 0, 0)[0] == k % 11


def test_xi_open_unit_interval_uniform():
    _, xi, _ = _draws(16, 40000)
    assert xi.min() > 0.0 and xi.max() < 1.0
    assert stats.kstest(xi, "uniform").pvalue > 1e-3


def test_gaussian_displacement_moments():
    sigma = 0.7
    _, _, d = _draws(16, 60000, sigma=sigma)
    x = d.ravel() / sigma
    n = x.size
    assert abs(x.mean()) < 5 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(stats.kurtosis(x, fisher=False) - 3.0) < 5 * np.sqrt(24.0 / n)
    # components are uncorrelated
    c = np.corrcoef(d.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5 / np.sqrt(len(d)))
    assert stats.kstest(x, "norm").pvalue > 1e-3


def test_stream_keyed_by_walker_sweep_step():
    sys_ = O.system(64, 10.0, 2.9, step_sigma=1.0, seed=9)
    a = O.draw_move(sys_, 3, 4, 5)
    assert O.draw_move(sys_, 3, 4, 5)[1] == a[1]
    assert O.draw_move(sys_, 3, 4, 6)[1] != a[1]
    assert O.draw_move(sys_, 3, 5, 5)[1] != a[1]
    assert O.draw_move(sys_, 4, 4, 5)[1] != a[1]
    other_seed = O.system(64, 10.0, 2.9, step_sigma=1.0, seed=10)
    assert O.draw_move(other_seed, 3, 4, 5)[1] != a[1]
