"""Pins of the oracle's pair functions: minimum image (Sec. 5.1), the Jastrow
factor of Eqs. (8)-(9) under the multiplicative-symmetrization reading, and the
HFD-B(HE) potential named in Sec. 2 against its published well and zero."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle as O
from conftest import read_golden

B = 1.15 * 2.556


def test_min_image_is_nearest_of_27_images():
    rng = np.random.default_rng(3)
    L = 13.7
    for _ in range(20000):
        a = rng.uniform(0, L, 3)
        b = rng.uniform(0, L, 3)
        d = np.array([O.min_image(a[i] - b[i], L) for i in range(3)])
        best = min(
            np.linalg.norm(a - b + L * np.array([i, j, k]))
            for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)
        )
        assert abs(np.linalg.norm(d) - best) <= 1e-12 * L
        assert np.all(np.abs(d) <= L / 2)


def test_f_is_schiff_verlet_fifth_power():
    s = O.system(2, 20.0, B)
    # at r = b: f = -1/2 exactly; at r = 2b: -1/64
    assert O.f(s, B) == -0.5
    assert O.f(s, 2 * B) == pytest.approx(-0.5 / 32, rel=1e-15)


def test_u_vanishes_with_zero_slope_at_half_box():
    L = 17.0
    s = O.system(2, L, B)
    h = L / 2
    assert abs(O.u(s, h)) < 1e-15
    eps = 1e-6
    slope = (O.u(s, h) - O.u(s, h - eps)) / eps   # one-sided: O(u'' eps) ~ 1e-9
    assert abs(slope) < 1e-8
    u, du, d2u = O.u_derivs(s, h)
    assert abs(du) < 1e-15
    # zero beyond the cutoff, negative (repulsive core) inside
    assert O.u(s, h + 1e-9) == 0.0 and O.u(s, 12.0) == 0.0
    assert O.u(s, 2.0) < O.u(s, 3.0) < O.u(s, 5.0) < 0.0


@pytest.mark.parametrize("r", [2.2, 2.9, 3.7, 5.0, 6.6, 8.1])
def test_u_derivatives_match_central_differences(r):
    s = O.system(2, 17.0, B)
    u, du, d2u = O.u_derivs(s, r)
    assert u == O.u(s, r)
    h = 1e-4
    fd1 = (O.u(s, r + h) - O.u(s, r - h)) / (2 * h)
    fd2 = (O.u(s, r + h) - 2 * O.u(s, r) + O.u(s, r - h)) / (h * h)
    assert du == pytest.approx(fd1, rel=1e-7, abs=1e-12)
    assert d2u == pytest.approx(fd2, rel=2e-5, abs=1e-9)


def _golden_hfdb():
    return {r[0]: float(r[1]) for r in read_golden("hfdb_he_properties.txt")}


def test_hfdb_well_depth_and_position():
    g = _golden_hfdb()
    eps, rm = g["epsilon_K"], g["r_m_A"]
    assert O.aziz(rm) == pytest.approx(-eps, rel=1e-6)
    h = 1e-5
    slope = (O.aziz(rm + h) - O.aziz(rm - h)) / (2 * h)
    assert abs(slope) < 1e-4          # K / Angstrom: the minimum sits at r_m
    # it is a minimum
    assert O.aziz(rm - 0.05) > O.aziz(rm) and O.aziz(rm + 0.05) > O.aziz(rm)


def test_hfdb_zero_crossing():
    g = _golden_hfdb()
    r0 = brentq(O.aziz, 2.3, 2.9, xtol=1e-12)
    assert abs(r0 - g["sigma_A"]) < 5e-5


def test_hfdb_limits():
    # finite repulsive core (damping switches the dispersion off at short range)
    v0 = O.aziz(1e-3)
    assert math.isfinite(v0) and 1e6 < v0 < 1e7
    # attractive tail, tending to the C6 dispersion term -eps C6 (r_m / r)^6
    assert O.aziz(6.0) < 0 and O.aziz(12.0) < 0
    r = 60.0
    assert O.aziz(r) == pytest.approx(-10.948 * 1.36745214 * (2.963 / r) ** 6, rel=1e-3)
