"""Pins of the oracle's per-configuration quantities:
  * Eq. (7) single-move sums against the brute-force difference of two full
    O(N^2) totals;
  * the local energy (Sec. 2, local value of the Hamiltonian) against the
    two-particle closed form, against finite differences of ln psi, under
    translation and permutation, and at b = 0 (ideal-gas wavefunction)."""
import numpy as np
import pytest

import oracle as O
from inputs import grid_config, moves

B = 1.15 * 2.556
RHO = 0.02186
HB = 12.1194


def _sys(n, b=B, rho=RHO):
    L = (n / rho) ** (1 / 3)
    return O.system(n, L, b, hbar2_over_m=HB), L


@pytest.mark.parametrize("n", [2, 4, 27, 108])
def test_delta_equals_difference_of_totals(n):
    s, L = _sys(n)
    x = grid_config(n, L, seed=n)
    ss, dd = moves(n, 12, 0.9, seed=100 + n)
    for k in range(len(ss)):
        rnew = O.trial_position(s, x, ss[k], dd[k])
        du, dv, su, sv = O.delta(s, x, ss[k], rnew)
        x2 = x.copy()
        x2[:, ss[k]] = rnew
        U0, V0 = O.totals(s, x)
        U1, V1 = O.totals(s, x2)
        tu = 1e-12 * max(abs(du), su, 1e-300) + 1e-13 * max(abs(U0), abs(U1))
        tv = 1e-12 * max(abs(dv), sv, 1e-300) + 1e-13 * max(abs(V0), abs(V1))
        assert abs((U1 - U0) - du) <= tu, (k, U1 - U0, du)
        assert abs((V1 - V0) - dv) <= tv, (k, V1 - V0, dv)


def test_trial_position_wraps_into_box():
    s, L = _sys(4)
    x = grid_config(4, L, seed=1)
    x[:, 0] = [0.01, L - 0.01, 3.0]
    r = O.trial_position(s, x, 0, np.array([-0.02, 0.02, 0.5]))
    assert 0 <= r[0] < L and 0 <= r[1] < L
    assert r[0] == pytest.approx(L - 0.01, abs=1e-12)
    assert r[1] == pytest.approx(0.01, abs=1e-12)
    assert r[2] == 3.5


@pytest.mark.parametrize("r", [2.4, 2.963, 3.5, 4.5, 6.0])
def test_two_particle_local_energy_closed_form(r):
    """N=2: G_1 = -G_2 = u' rhat, L_1 = L_2 = u'' + 2u'/r, so
    E_L = V(r) - 2 kappa (u'' + 2u'/r + u'^2) with kappa = hbar^2/2m.
    u' and u'' are taken from central differences of u (pinned separately)."""
    L = 14.0
    s = O.system(2, L, B, hbar2_over_m=HB)
    x = np.array([[1.0, 1.0 + r * 0.6], [2.0, 2.0 + r * 0.8], [3.0, 3.0]])
    h = 1e-4
    du = (O.u(s, r + h) - O.u(s, r - h)) / (2 * h)
    d2u = (O.u(s, r + h) - 2 * O.u(s, r) + O.u(s, r - h)) / h ** 2
    kappa = HB / 2
    expect_t = -2 * kappa * (d2u + 2 * du / r + du ** 2)
    out, scale = O.local_energy(s, x)
    assert out[1] == O.aziz(r) or out[1] == pytest.approx(O.aziz(r), rel=1e-14)
    assert out[2] == pytest.approx(expect_t, rel=1e-5, abs=1e-9)
    assert out[0] == pytest.approx(out[1] + out[2], rel=1e-14)
    # the three kinetic estimators for a single pair
    assert out[3] == pytest.approx(-kappa * (d2u + 2 * du / r), rel=1e-5)
    assert out[4] == pytest.approx(2 * kappa * du ** 2, rel=1e-6)
    assert out[5] == pytest.approx(O.u(s, r), rel=1e-13)


def test_two_particles_beyond_cutoff_have_no_energy():
    L = 14.0
    s = O.system(2, L, B, hbar2_over_m=HB)
    x = np.array([[0.5, 7.6], [0.5, 7.6], [0.5, 0.5]])   # r = 7.1 * sqrt(2) > L/2
    out, _ = O.local_energy(s, x)
    assert np.all(out == 0.0)


@pytest.mark.parametrize("n", [4, 32])
def test_gradient_and_laplacian_match_finite_differences(n):
    s, L = _sys(n)
    x = grid_config(n, L, seed=7 + n)
    out, scale, G, Lap = O.local_energy(s, x, want_derivs=True)
    h = 2e-4
    U0 = O.totals(s, x)[0]
    for i in range(n):
        lap = 0.0
        for a in range(3):
            xp = x.copy(); xp[a, i] += h
            xm = x.copy(); xm[a, i] -= h
            Up = O.totals(s, xp)[0]
            Um = O.totals(s, xm)[0]
            g = (Up - Um) / (2 * h)
            lap += (Up - 2 * U0 + Um) / h ** 2
            assert G[a, i] == pytest.approx(g, rel=1e-6, abs=1e-7)
        assert Lap[i] == pytest.approx(lap, rel=2e-4, abs=2e-5)
    # U reported by the local-energy pass is the same ln psi
    assert out[5] == pytest.approx(U0, rel=1e-13)
    # assembly of the estimators
    kappa = HB / 2
    assert out[2] == pytest.approx(-kappa * (Lap.sum() + (G ** 2).sum()), rel=1e-12)
    assert out[3] == pytest.approx(-kappa / 2 * Lap.sum(), rel=1e-12)
    assert out[4] == pytest.approx(kappa * (G ** 2).sum(), rel=1e-12)


def test_local_energy_translation_and_permutation_invariant():
    n = 108
    s, L = _sys(n)
    x = grid_config(n, L, seed=5)
    ref, scale = O.local_energy(s, x)
    shifted = np.mod(x + np.array([[3.3], [-7.1], [11.9]]), L)
    out, _ = O.local_energy(s, shifted)
    assert np.allclose(out, ref, rtol=0, atol=1e-11 * scale)
    perm = np.random.default_rng(2).permutation(n)
    out, _ = O.local_energy(s, x[:, perm])
    assert np.allclose(out, ref, rtol=0, atol=1e-12 * scale)


def test_b_zero_has_no_kinetic_energy():
    n = 27
    s, L = _sys(n, b=0.0)
    x = grid_config(n, L, seed=11)
    out, _ = O.local_energy(s, x)
    assert out[2] == 0.0 and out[3] == 0.0 and out[4] == 0.0 and out[5] == 0.0
    assert out[0] == out[1]


def test_sum_of_pair_potential_matches_totals():
    n = 64
    s, L = _sys(n)
    x = grid_config(n, L, seed=21)
    out, _ = O.local_energy(s, x)
    U, V = O.totals(s, x)
    assert out[1] == pytest.approx(V, rel=1e-13)
    assert out[5] == pytest.approx(U, rel=1e-13)


def test_fcc_start():
    n = 108
    s, L = _sys(n)
    x = O.fcc_start(s, 0)
    assert x.min() > 0 and x.max() < L
    a = L / 3
    # nearest neighbour distance of fcc is a / sqrt(2), up to the 1e-3 a jitter
    d = np.array([np.linalg.norm([O.min_image(x[c, 0] - x[c, j], L) for c in range(3)]) for j in range(1, n)])
    assert np.isclose(d.min(), a / np.sqrt(2), rtol=3e-3)
    assert np.sum(np.abs(d - a / np.sqrt(2)) < 3e-3 * a) == 12
    # distinct walkers get distinct jitter, same lattice
    y = O.fcc_start(s, 1)
    assert not np.array_equal(x, y)
    assert np.max(np.abs(x - y)) < 1.001e-3 * a
