"""Pins of the host statistics (Sec. 4.1, Eq. (10)): reblocking and the
autocorrelation time on sequences whose answers are known in closed form.

* Independent samples: every reblocking level estimates sigma/sqrt(n), and
  m_c is zero (within noise).
* AR(1), A_{i+1} = rho A_i + sqrt(1 - rho^2) eps_i: R(k) = rho^k, so
  m_c = rho / (1 - rho), and the standard error of the mean of n samples is
  sigma/sqrt(n) * sqrt((1 + rho) / (1 - rho)) = sigma/sqrt(n) sqrt(1 + 2 m_c)
  (Eq. (10) with m = 1); the blocking plateau reaches it.
"""
import numpy as np
import pytest

from paper_1312_1282_amd import observables as ob


def ar1(n, rho, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    c = np.sqrt(1.0 - rho * rho)
    for i in range(1, n):
        x[i] = rho * x[i - 1] + c * e[i]
    return x


def test_independent_samples():
    rng = np.random.default_rng(3)
    x = 2.0 + 0.5 * rng.standard_normal(1 << 16)
    exact = 0.5 / np.sqrt(len(x))
    lv = ob.blocking(x)
    assert lv[0][0] == len(x)
    for n, se, dse in lv[:10]:
        assert abs(se - exact) <= 4 * dse + 0.02 * exact, (n, se, exact)
    se, level = ob.blocking_se(x)
    assert se == pytest.approx(exact, rel=0.05)
    R, mc = ob.autocorrelation(x, kmax=50)
    assert R[0] == pytest.approx(1.0)
    assert abs(mc) < 0.05


@pytest.mark.parametrize("rho", [0.5, 0.8, 0.95])
def test_ar1_error_and_autocorrelation_time(rho):
    n = 1 << 18
    x = ar1(n, rho, seed=int(rho * 100))
    mc_exact = rho / (1.0 - rho)
    se_exact = 1.0 / np.sqrt(n) * np.sqrt((1.0 + rho) / (1.0 - rho))
    R, mc = ob.autocorrelation(x, kmax=400)
    assert R[1] == pytest.approx(rho, abs=0.01)
    assert R[3] == pytest.approx(rho ** 3, abs=0.02)
    assert mc == pytest.approx(mc_exact, rel=0.1)
    se, level = ob.blocking_se(x)
    assert se == pytest.approx(se_exact, rel=0.15), (se, se_exact, level)
    # the naive (level 0) estimate is too small by sqrt(1 + 2 m_c)
    assert ob.blocking(x)[0][1] == pytest.approx(se_exact / np.sqrt(1 + 2 * mc_exact), rel=0.05)


def test_short_and_odd_sequences():
    assert ob.blocking([1.0, 2.0, 3.0]) == []
    lv = ob.blocking(np.arange(9.0))
    assert [n for n, _, _ in lv] == [9, 4]
