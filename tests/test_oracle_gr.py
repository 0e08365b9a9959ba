"""Pins of the oracle's pair distribution histogram (the g(r) of the paper's
host analysis, Sec. 5.4), against facts fixed by geometry:

* a perfect fcc lattice: every bin below L/2 holds N/2 times the number of
  lattice vectors of that length, counted here by integer enumeration;
* a second implementation (numpy, vectorised minimum image and np.histogram)
  on random configurations;
* the ideal gas: expected counts are N(N-1)/2 times the shell volume over L^3.
"""
import numpy as np
import pytest

import oracle as O
from inputs import uniform_config

RHO = 0.02186


def osys(n, L=None):
    return O.system(n, L if L is not None else O.box_side(n, RHO), 2.94, hbar2_over_m=12.1194, step_sigma=0.6,
                    seed=1)


def fcc_lattice(nc, a):
    base = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    pts = [(np.array([i, j, k]) + b + 0.25) * a for i in range(nc) for j in range(nc) for k in range(nc)
           for b in base]
    return np.array(pts).T.copy()


@pytest.mark.parametrize("nc,nb", [(4, 37), (5, 61)])
def test_perfect_fcc_shells(nc, nb):
    a = 5.0
    L = nc * a
    n = 4 * nc ** 3
    s = osys(n, L)
    counts, _ = O.pair_histogram(s, fcc_lattice(nc, a), nb)
    # lattice vectors (x, y, z) a/2 with x + y + z even, enumerated in integers
    h = L / 2
    width = h / nb
    expect = np.zeros(nb, dtype=np.int64)
    m = 2 * nc
    for x in range(-m, m + 1):
        for y in range(-m, m + 1):
            for z in range(-m, m + 1):
                if (x + y + z) % 2 or (x == y == z == 0):
                    continue
                q = x * x + y * y + z * z          # |v|^2 = q a^2 / 4
                if 4 * q < (2 * nc) ** 2:          # strictly inside L/2 = nc a / 2
                    expect[int(np.floor(np.sqrt(q) * a / 2 / width))] += 1
    expect = expect * n // 2
    # every bin but the last (which may hold the shell at exactly L/2, where a
    # vector and its periodic image are the same neighbour)
    assert np.array_equal(counts[:-1].astype(np.int64), expect[:-1])
    assert (expect > 0).sum() >= 6


def _numpy_histogram(x, L, nb):
    d = x[:, :, None] - x[:, None, :]
    d -= L * np.rint(d / L)
    r = np.sqrt((d * d).sum(0))
    iu = np.triu_indices(x.shape[1], 1)
    r = r[iu]
    r = r[r <= L / 2]
    c, _ = np.histogram(np.minimum(r, np.nextafter(L / 2, 0)), bins=nb, range=(0.0, L / 2))
    return c


@pytest.mark.parametrize("n,nb,seed", [(2, 10, 1), (27, 20, 2), (108, 50, 3), (257, 100, 4)])
def test_matches_a_second_implementation(n, nb, seed):
    s = osys(n)
    x = uniform_config(n, s.L, seed=seed)
    counts, edge = O.pair_histogram(s, x, nb, rel_window=1e-9)
    ref = _numpy_histogram(x, s.L, nb)
    assert edge.sum() == 0          # no pair so close to an edge that roundings could disagree
    assert np.array_equal(counts.astype(np.int64), ref)


def test_ideal_gas_shell_volumes():
    n, nb, reps = 64, 16, 200
    s = osys(n)
    tot = np.zeros(nb)
    for k in range(reps):
        counts, _ = O.pair_histogram(s, uniform_config(n, s.L, seed=1000 + k), nb)
        tot += counts
    w = s.L / 2 / nb
    shell = 4.0 / 3.0 * np.pi * ((np.arange(1, nb + 1) * w) ** 3 - (np.arange(nb) * w) ** 3)
    expect = reps * n * (n - 1) / 2 * shell / s.L ** 3
    chi2 = ((tot - expect) ** 2 / expect).sum()
    assert chi2 < 45.0, chi2        # 16 bins: p ~ 1e-4 at 45
    assert tot.sum() == pytest.approx(reps * n * (n - 1) / 2 * np.pi / 6, rel=0.02)


def test_cutoff_pair_goes_to_last_bin_and_edges_are_flagged():
    L = 10.0
    s = osys(2, L)
    x = np.array([[1.0, 6.0], [2.0, 2.0], [3.0, 3.0]])     # r = L/2 exactly
    counts, edge = O.pair_histogram(s, x, 5, rel_window=1e-12)
    assert counts.tolist() == [0, 0, 0, 0, 1] and edge[5] == 1
    x = np.array([[1.0, 3.0], [2.0, 2.0], [3.0, 3.0]])     # r = 2 = edge between bins 1 and 2
    counts, edge = O.pair_histogram(s, x, 5, rel_window=1e-12)
    assert counts.tolist() == [0, 0, 1, 0, 0] and edge[2] == 1
    x = np.array([[1.0, 7.5], [2.0, 2.0], [3.0, 3.0]])     # min image: r = 3.5
    counts, _ = O.pair_histogram(s, x, 5)
    assert counts.tolist() == [0, 0, 0, 1, 0]


def test_pair_distribution_of_the_ideal_gas_is_one():
    from paper_1312_1282_amd import observables
    n, nb, reps = 64, 8, 300
    s = osys(n)
    tot = np.zeros(nb)
    for k in range(reps):
        tot += O.pair_histogram(s, uniform_config(n, s.L, seed=5000 + k), nb)[0]
    r, g = observables.pair_distribution(tot, n, s.L, reps)
    assert np.allclose(r, (np.arange(nb) + 0.5) * s.L / 2 / nb)
    assert np.all(np.abs(g - 1.0) < 0.1) and abs(g[2:].mean() - 1.0) < 0.02
