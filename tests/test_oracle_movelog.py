"""Pins of the oracle's per-move record and of its FP32-coordinate storage.

The record (s, accepted, dU, dV, scales) of every micro-update is what the GPU
parity tests compare the sweep kernel's own record with, move by move.  It is
pinned to quantities computed independently of it: the random stream, the
Eq. (5) decision, and the brute-force totals of Eq. (6) (the accepted moves'
dU must telescope to U(final) - U(start)).

FP32 storage (the precision form's coordinates, arithmetic still FP64): every
stored position is the nearest FP32 number to the FP64 one, inside [0, L).
"""
import numpy as np

import oracle as O

B = 1.15 * 2.556
HB = 12.1194
RHO = 0.02186


def _sys(n, fp32=False, seed=7, step=0.63, order=0):
    L = O.box_side(n, RHO, fp32)
    return O.system(n, L, B, hbar2_over_m=HB, step_sigma=step, seed=seed, order=order, fp32_coords=fp32)


def test_logged_chain_is_the_chain():
    """Recording changes nothing: same configuration and accumulators, bit for bit."""
    s_ = _sys(32)
    x1 = O.fcc_start(s_, 3)
    a1 = O.walker_init(s_, x1)
    O.run_walker(s_, 3, x1, a1, 0, 12, 4, 2)
    x2 = O.fcc_start(s_, 3)
    a2 = O.walker_init(s_, x2)
    O.run_walker_log(s_, 3, x2, a2, 0, 12, 4, 2)
    assert np.array_equal(x1, x2)
    assert bytes(a1) == bytes(a2)


def test_move_log_follows_stream_decision_and_totals():
    """Each record's s is the stream's s for (k, t, w); its decision is Eq. (5)
    on the stream's xi; the accepted moves' dU and dV add up to the change of
    the brute-force totals between the start and the end (no sample resets the
    running totals here); every dU and dV is within its own scale."""
    n, sweeps, w, t0 = 48, 10, 5, 100
    s_ = _sys(n)
    x = O.fcc_start(s_, w)
    U0, V0 = O.totals(s_, x)
    a = O.walker_init(s_, x)
    log = O.run_walker_log(s_, w, x, a, t0, sweeps, 0xFFFFFFFF, 0)
    assert log.shape == (n * sweeps, 8)
    for q in range(n * sweeps):
        k, t = q % n, t0 + q // n
        s, xi, _ = O.draw_move(s_, k, t, w)
        assert log[q, 0] == s
        assert bool(log[q, 1]) == O.metropolis_accept(log[q, 2], xi)
        assert abs(log[q, 2]) <= log[q, 4] and abs(log[q, 3]) <= log[q, 5]
    acc = log[:, 1] == 1
    assert 0.3 < acc.mean() < 0.8
    U1, V1 = O.totals(s_, x)
    su, sv = log[acc, 4].sum(), log[acc, 5].sum()
    assert abs(log[acc, 2].sum() - (U1 - U0)) <= 1e-12 * su
    assert abs(log[acc, 3].sum() - (V1 - V0)) <= 1e-12 * sv


def test_log_capacity_truncates():
    s_ = _sys(16)
    x = O.fcc_start(s_, 0)
    a = O.walker_init(s_, x)
    full = O.run_walker_log(s_, 0, x.copy(), O.walker_init(s_, x), 0, 3, 0, 0)
    part = O.run_walker_log(s_, 0, x, a, 0, 3, 0, 0, cap=20)
    assert np.array_equal(full[:20], part)


def test_fp32_storage_rounds_every_stored_position():
    """Start and every accepted position are FP32 numbers in [0, L), each the
    nearest FP32 number to the FP64 position the move computed; the running
    totals still equal a fresh evaluation."""
    n = 32
    s32 = _sys(n, fp32=True)
    s64 = _sys(n, fp32=False)
    s64.L = s32.L   # same (FP32-representable) box, FP64 storage
    x32 = O.fcc_start(s32, 2)
    x64 = O.fcc_start(s64, 2)
    assert np.array_equal(x32, x64.astype(np.float32).astype(np.float64))
    a = O.walker_init(s32, x32)
    log = O.run_walker_log(s32, 2, x32, a, 0, 15, 0xFFFFFFFF, 0)
    assert np.array_equal(x32, x32.astype(np.float32).astype(np.float64))
    assert np.all((x32 >= 0) & (x32 < s32.L))
    assert 0.3 < log[:, 1].mean() < 0.8
    U, V = O.totals(s32, x32)
    assert abs(a.u_run - U) <= 1e-10 * max(1.0, abs(U))
    assert abs(a.v_run - V) <= 1e-10 * max(1.0, abs(V))
    # one trial move against its FP64 counterpart: at most half an FP32 ulp apart
    s, _, d = O.draw_move(s32, 0, 99, 2)
    r32 = O.trial_position(s32, x32, s, d)
    r64 = O.trial_position(s64, x32, s, d)
    assert np.array_equal(r32, r64.astype(np.float32).astype(np.float64))
    ulp = np.spacing(np.abs(r64).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(r32 - r64) <= 0.5 * ulp)


def test_fp32_storage_value_rounding_to_L_is_zero():
    """A position just below L whose nearest FP32 number is L itself is the
    point 0 of the periodic box."""
    n = 4
    s32 = _sys(n, fp32=True)
    L = s32.L
    x = np.ascontiguousarray(np.full((3, n), 1.0))
    x[0, 1] = np.nextafter(L, 0.0)   # an FP64 number that rounds up to L in FP32
    assert float(np.float32(x[0, 1])) == L
    r = O.trial_position(s32, x, 1, np.zeros(3))
    assert r[0] == 0.0 and r[1] == 1.0 and r[2] == 1.0


def test_aziz_slope_is_the_derivative_of_the_potential():
    """dV/dr against central differences of the potential itself, across the
    damping region (x < D), the well and the dispersion tail."""
    for r in (2.3, 2.7, 2.963, 3.4, 4.0, 4.39, 4.5, 6.0, 9.0, 15.0):
        h = 1e-5 * r
        fd = (O.aziz(r + h) - O.aziz(r - h)) / (2 * h)
        assert abs(O.aziz_deriv(r) - fd) <= 1e-7 * max(1.0, abs(fd)), r
    # the well's minimum at r_m: the slope changes sign there
    assert O.aziz_deriv(2.95) < 0.0 < O.aziz_deriv(2.98)


def test_move_slopes_sum_the_pair_slopes():
    """N = 3: the slopes of a move are the sums over the two other atoms of
    |du/dr| and |dV/dr| at the old and the trial distance, each taken here by
    central differences of u and V (the pair beyond L/2 adds nothing)."""
    n = 3
    s_ = _sys(n)
    L = s_.L
    x = np.ascontiguousarray(np.array([[0.3, 2.9, 5.1], [0.2, 0.4, 3.0], [0.1, 0.3, 0.2]]) * (L / 6.0))
    s, rnew = 0, x[:, 0] + np.array([0.7, -0.2, 0.4])
    su, sv = O.delta_slopes(s_, x, s, rnew)
    want_u = want_v = 0.0
    for i in (1, 2):
        for p in (rnew, x[:, 0]):
            d = p - x[:, i]
            d -= L * np.round(d / L)
            r = float(np.sqrt(d @ d))
            h = 1e-6 * r
            want_u += abs(O.u(s_, r + h) - O.u(s_, r - h)) / (2 * h)
            if r <= L / 2:
                want_v += abs(O.aziz(r + h) - O.aziz(r - h)) / (2 * h)
    assert su == __import__("pytest").approx(want_u, rel=1e-6)
    assert sv == __import__("pytest").approx(want_v, rel=1e-6)
