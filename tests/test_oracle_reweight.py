"""Correlated sampling over the Jastrow parameter b, on the CPU.

* The identity the reweighting rests on: f of Eq. (9) scales as b^5, so the
  oracle's local energy evaluated directly at b' equals V + 2 lam T_JF -
  lam^2 T_F of its evaluation at b, and U(b') = lam U(b), lam = (b'/b)^5.
* The estimator: energies reweighted from an oracle chain at b agree with an
  oracle chain run at b' itself, within their standard errors.
"""
import numpy as np
import pytest

import oracle as O
from inputs import grid_config
from paper_1312_1282_amd import configs, observables

RHO = configs.RHO_EQ
STEP = configs.C1_SMALL_FP64.step_sigma


def osys(n, b, seed=1):
    return O.system(n, O.box_side(n, RHO), b, hbar2_over_m=configs.HBAR2_OVER_M, step_sigma=STEP, seed=seed)


@pytest.mark.parametrize("n,b,bp", [(2, 2.9, 3.1), (32, 2.94, 2.80), (108, 2.94, 3.07), (108, 3.0, 3.0)])
def test_local_energy_scales_with_b_to_the_fifth(n, b, bp):
    s_b, s_bp = osys(n, b), osys(n, bp)
    x = grid_config(n, s_b.L, seed=90 + n)
    el_b, scale_b = O.local_energy(s_b, x)
    el_bp, scale_bp = O.local_energy(s_bp, x)
    lam = (bp / b) ** 5
    e, lw = observables.energy_at_b(el_b, lam)
    tol = 1e-12 * max(scale_b, scale_bp)
    assert abs(e - el_bp[0]) <= tol, (e, el_bp[0])
    assert abs(lam * el_b[5] - el_bp[5]) <= 1e-12 * abs(el_bp[5]) + 1e-12
    assert lw == pytest.approx(2.0 * (el_bp[5] - el_b[5]), rel=1e-12, abs=1e-12)


def _records(s_, w, equil, n_sweeps, m):
    """Oracle chain from the fcc start; the local-energy record of every m-th
    measured configuration."""
    x = O.fcc_start(s_, w)
    a = O.walker_init(s_, x)
    O.run_walker(s_, w, x, a, 0, equil, 0xFFFFFFFF, 0)
    rec = []
    t = equil
    for _ in range(n_sweeps // m):
        O.run_walker(s_, w, x, a, t, m, 0xFFFFFFFF, 0)
        t += m
        rec.append(O.local_energy(s_, x)[0])
    return np.array(rec)


def test_reweighted_energy_matches_a_direct_run():
    n, b, bp = 32, 2.94, 2.94 * 1.03
    W, equil, sweeps, m = 8, 200, 1500, 5
    rec_b = np.stack([_records(osys(n, b, seed=3), w, equil, sweeps, m) for w in range(W)])
    rec_bp = np.stack([_records(osys(n, bp, seed=4), w, equil, sweeps, m) for w in range(W)])
    est = observables.reweight_b(rec_b, b, [b, bp], n)
    # at b itself the estimate is the plain mean
    assert est[0]["E_per_atom"] == pytest.approx(rec_b[..., 0].mean() / n, rel=1e-12)
    assert est[0]["ess"] == pytest.approx(rec_b[..., 0].size)
    direct = rec_bp[..., 0].mean(axis=1) / n
    se_direct = direct.std(ddof=1) / np.sqrt(W)
    # walker-level spread of the reweighted estimate
    per_w = np.array([observables.reweight_b(rec_b[w:w + 1], b, [bp], n)[0]["E_per_atom"] for w in range(W)])
    se_rw = per_w.std(ddof=1) / np.sqrt(W)
    assert est[1]["ess"] > 0.3 * rec_b[..., 0].size
    assert abs(est[1]["E_per_atom"] - direct.mean()) < 4.0 * np.hypot(se_direct, se_rw), \
        (est[1]["E_per_atom"], direct.mean(), se_direct, se_rw)
