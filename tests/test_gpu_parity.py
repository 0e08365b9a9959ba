"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (FP64):
  * Eq. (7) sums:  |dU_gpu - dU_or| <= 1e-12 max(|dU_or|, sum_i |u'_i| + |u_i|),
    same for dV with |V| terms (relative 1e-12 is ill-posed when dU ~ 0, so
    the scale is the sum of the magnitudes that are added);
  * local energy: each of (E_L, V, T_PB, T_JF, T_F, U) within 1e-12 x the
    oracle's scale sum |V_ij| + kappa sum_i (|L_i| + |G_i|^2);
  * random numbers: s and xi bit for bit, delta within 1e-14 relative
    (Box-Muller uses log, sqrt, sin, cos whose last bit may differ between the
    device and host math libraries);
  * chains in lockstep: identical accept counts, coordinates within 1e-9 A,
    accumulators within 1e-10 relative.
"""
import threading

import numpy as np
import pytest

import oracle as O
from inputs import grid_config, moves
from paper_1312_1282_amd import abi, configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RHO = configs.RHO_EQ
B = configs.C1_SMALL_FP64.b
STEP = configs.C1_SMALL_FP64.step_sigma


def osys(n, rho=RHO, b=B, step=STEP, seed=1, fp32=False, order=0):
    return O.system(n, O.box_side(n, rho, fp32), b, hbar2_over_m=configs.HBAR2_OVER_M, step_sigma=step,
                    seed=seed, order=order)


def gparams(n, W, precision=abi.FP64, threads=0, seed=1, wbase=0, order=0, b=B, rho=RHO, step=STEP,
            variant=abi.VARIANT_AUTO):
    return abi.make_params(n, W, precision=precision, density=rho, b=b, step_sigma=step, seed=seed,
                           walker_id_base=wbase, threads=threads, order=order, variant=variant)


def within(got, ref, scale, rel):
    return abs(got - ref) <= rel * max(abs(ref), scale)


def _dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


# ---------------------------------------------------------------------------
# per-configuration quantities

@pytest.mark.parametrize("n,threads", [(2, 64), (4, 128), (27, 256), (108, 64), (108, 128), (500, 64), (500, 512),
                                       (1100, 1024), (2048, 256), (2048, 512)])
def test_move_sums_fp64(n, threads):
    W = 6
    s_ = osys(n)
    L = s_.L
    xs = np.stack([grid_config(n, L, seed=1000 + n + w) for w in range(W)])
    ss, dd = moves(n, W, 0.8, seed=77 + n)
    p = gparams(n, W, threads=threads)
    out = torch.zeros((W, 2), dtype=torch.float64, device="cuda")
    abi.move_delta(p, _dev(xs), _dev(ss, torch.int32), _dev(dd), out)
    out = out.cpu().numpy()
    for w in range(W):
        rnew = O.trial_position(s_, xs[w], ss[w], dd[w])
        du, dv, su, sv = O.delta(s_, xs[w], ss[w], rnew)
        assert within(out[w, 0], du, su, 1e-12), (w, out[w, 0], du, su)
        assert within(out[w, 1], dv, sv, 1e-12), (w, out[w, 1], dv, sv)


@pytest.mark.parametrize("n,threads", [(2, 64), (4, 128), (27, 128), (108, 64), (108, 256), (500, 128),
                                       (1100, 1024), (2048, 256), (4000, 512)])
def test_local_energy_fp64(n, threads):
    W = 3
    s_ = osys(n)
    xs = np.stack([grid_config(n, s_.L, seed=2000 + n + w) for w in range(W)])
    p = gparams(n, W, threads=threads)
    out = torch.zeros((W, 6), dtype=torch.float64, device="cuda")
    abi.local_energy(p, _dev(xs), out)
    out = out.cpu().numpy()
    for w in range(W):
        ref, scale = O.local_energy(s_, xs[w])
        for q in range(6):
            assert within(out[w, q], ref[q], scale, 1e-12), (w, q, out[w, q], ref[q], scale)


def test_eval_config_host_entry():
    n = 108
    s_ = osys(n)
    x = grid_config(n, s_.L, seed=5)
    p = gparams(n, 1)
    ss, dd = moves(n, 4, 1.0, seed=3)
    for k in range(4):
        du, dv, el = abi.eval_config(p, x, int(ss[k]), dd[k])
        rnew = O.trial_position(s_, x, ss[k], dd[k])
        rdu, rdv, su, sv = O.delta(s_, x, ss[k], rnew)
        ref, scale = O.local_energy(s_, x)
        assert within(du, rdu, su, 1e-12) and within(dv, rdv, sv, 1e-12)
        assert all(within(el[q], ref[q], scale, 1e-12) for q in range(6))


def test_invalid_move_index_gives_nan_and_eval_rejects():
    n, W = 27, 2
    s_ = osys(n)
    xs = np.stack([grid_config(n, s_.L, seed=w) for w in range(W)])
    p = gparams(n, W)
    out = torch.zeros((W, 2), dtype=torch.float64, device="cuda")
    abi.move_delta(p, _dev(xs), _dev(np.array([-1, n], np.int32), torch.int32), _dev(np.zeros((W, 3))), out)
    assert torch.isnan(out).all()
    with pytest.raises(abi.HevmcError):
        abi.eval_config(gparams(n, 1), xs[0], n, np.zeros(3))


def test_fp64_walker_too_large_for_lds():
    """An FP64 walker of 10976 atoms (263 KB) fits in no workgroup's LDS: the
    plan spreads it over two workgroups, and the entry points without a
    spread form refuse it."""
    p = gparams(10976, 1)
    plan = abi.plan_launch(p)
    assert plan["slices"] == 2 and plan["variant"] == abi.VARIANT_PLAIN
    lds, _ = abi.footprint(p)
    assert lds == 2 * plan["lds_per_group"]
    coords, acc = abi.alloc_state(p)
    with pytest.raises(abi.HevmcError) as ei:
        abi.pair_histogram(p, coords, torch.zeros((1, 16), dtype=torch.int64, device="cuda"))
    assert ei.value.code == -3


def _largest_fitting_n(precision, lo, hi):
    """Largest N whose walker fits one workgroup's LDS (bisection on the plan)."""
    def fits(n):
        return abi.plan_launch(gparams(n, 1, precision=precision))["slices"] == 1
    assert fits(lo) and not fits(hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        lo, hi = (mid, hi) if fits(mid) else (lo, mid)
    return lo


def test_largest_fp64_walker_follows_the_oracle():
    """The largest FP64 walker that fits in one workgroup's LDS (plain
    variant, about 6800 atoms): one sweep with a local-energy sample, against
    the oracle; one atom more is spread over two workgroups."""
    n = _largest_fitting_n(abi.FP64, 4000, 10976)
    assert 6000 < n < 7000
    assert abi.plan_launch(gparams(n + 1, 1))["slices"] == 2
    p = gparams(n, 2, seed=12)
    plan = abi.plan_launch(p)
    assert plan["variant"] == abi.VARIANT_PLAIN and plan["lds_per_walker"] >= 24 * n
    xg, ag = _gpu_chain(p, [1], 0, 1)
    s_ = osys(n, seed=12)
    res = {}

    def work(w):
        res[w] = _oracle_chain(s_, w, 1, 0, 1)

    th = [threading.Thread(target=work, args=(w,)) for w in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for w in range(2):
        _compare_walker(xg[w], ag[w], *res[w])


# ---------------------------------------------------------------------------
# random numbers and start

@pytest.mark.parametrize("order", [0, 1])
def test_draw_moves_match_oracle(order):
    n, W, t = 97, 3, 12345
    p = gparams(n, W, seed=0x1234567890ABCDEF, wbase=7, order=order)
    s_ = osys(n, seed=0x1234567890ABCDEF, order=order)
    so = torch.zeros((W, n), dtype=torch.int32, device="cuda")
    xo = torch.zeros((W, n), dtype=torch.float64, device="cuda")
    do = torch.zeros((W, n, 3), dtype=torch.float64, device="cuda")
    abi.draw_moves(p, t, so, xo, do)
    so, xo, do = so.cpu().numpy(), xo.cpu().numpy(), do.cpu().numpy()
    for w in range(W):
        for k in range(n):
            s, xi, d = O.draw_move(s_, k, t, 7 + w)
            assert so[w, k] == s
            assert xo[w, k] == xi
            assert np.allclose(do[w, k], d, rtol=1e-14, atol=1e-15 * STEP)


@pytest.mark.parametrize("n,precision", [(108, abi.FP64), (500, abi.FP64), (256, abi.FP32)])
def test_fcc_start_and_initial_totals(n, precision):
    W = 4
    p = gparams(n, W, precision=precision, wbase=3)
    coords, acc = abi.alloc_state(p)
    abi.init_walkers(p, coords, acc, fcc_start=True)
    xs = coords.cpu().numpy().astype(np.float64)
    a = abi.acc_to_numpy(acc)
    fp32 = precision == abi.FP32
    s_ = osys(n, fp32=fp32)
    for w in range(W):
        ref = O.fcc_start(s_, 3 + w)
        tol = 1e-6 * s_.L if fp32 else 1e-13 * s_.L
        assert np.max(np.abs(xs[w] - ref)) <= tol
        U, V = O.totals(s_, xs[w])
        rel = 1e-5 if fp32 else 1e-12
        assert a["u_run"][w] == pytest.approx(U, rel=rel)
        assert a["v_run"][w] == pytest.approx(V, rel=rel)
        assert a["n_try"][w] == 0 and a["sum_e"][w] == 0


# ---------------------------------------------------------------------------
# chains in lockstep

def _gpu_chain(p, splits, measure_start, m, keep_rows=True, rows_fill=None):
    """Run the GPU chain from the fcc start in launches of the given lengths.
    keep_rows: keep the row sums in a device buffer between launches (else the
    kernel recomputes them at each launch); rows_fill: overwrite that buffer
    with this value after initialisation (a stale buffer)."""
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p) if keep_rows else None
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    if rows is not None and rows_fill is not None:
        rows.fill_(rows_fill)
    t = 0
    for k in splits:
        abi.sweep(p, coords, acc, t, k, measure_start, m, rows=rows)
        t += k
    torch.cuda.synchronize()
    return coords.cpu().numpy(), abi.acc_to_numpy(acc)


def _oracle_chain(s_, w, n_sweeps, measure_start, m):
    x = O.fcc_start(s_, w)
    a = O.walker_init(s_, x)
    el = O.run_walker(s_, w, x, a, 0, n_sweeps, measure_start, m, record_el=False)
    return x, a


def _compare_walker(xg, ag, xo, ao):
    assert ag["n_acc"] == ao.n_acc and ag["n_try"] == ao.n_try
    assert ag["n_samples"] == ao.n_samples and ag["n_sweeps_meas"] == ao.n_sweeps_meas
    assert np.max(np.abs(xg - xo)) < 1e-9
    for f in ("sum_e", "sum_e2", "sum_v", "sum_tpb", "sum_tjf", "sum_tf", "sum_vs"):
        c = "c_" + f[4:]
        g = ag[f] + ag[c]
        o = getattr(ao, f) + getattr(ao, c)
        assert g == pytest.approx(o, rel=1e-10, abs=1e-8), f
    assert ag["u_run"] == pytest.approx(ao.u_run, rel=1e-10, abs=1e-9)
    assert ag["v_run"] == pytest.approx(ao.v_run, rel=1e-10, abs=1e-9)


VARIANTS = [abi.VARIANT_PLAIN, abi.VARIANT_ROWS]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("keep_rows", [True, False])
def test_lockstep_chain_n108_full_run(variant, keep_rows):
    """N=108, one walker, 200 equilibration + 1000 measured sweeps, local energy
    every sweep, split over launches of different lengths."""
    wl = configs.C1_SMALL_FP64
    p = abi.params_for(wl, variant=variant)
    total = wl.equil + wl.measured
    xg, ag = _gpu_chain(p, [150, 50, 400, 600], wl.equil, wl.m, keep_rows=keep_rows)
    s_ = osys(wl.n, seed=wl.seed)
    xo, ao = _oracle_chain(s_, 0, total, wl.equil, wl.m)
    _compare_walker(xg[0], ag[0], xo, ao)
    assert ao.n_samples == 1000


@pytest.mark.parametrize("variant", VARIANTS)
def test_lockstep_without_energy_refresh(variant):
    """Sweeps with no local-energy pass: the running totals (and, for the row
    variant, the rows) are only updated incrementally for 60 sweeps."""
    n, W = 256, 2
    p = gparams(n, W, seed=21, variant=variant)
    xg, ag = _gpu_chain(p, [25, 35], 0, 0)
    s_ = osys(n, seed=21)
    for w in range(W):
        xo, ao = _oracle_chain(s_, w, 60, 0, 0)
        _compare_walker(xg[w], ag[w], xo, ao)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("threads", [64, 128, 256])
def test_lockstep_sequential_order_and_threads(variant, threads):
    n, W = 256, 3
    p = gparams(n, W, threads=threads, order=1, seed=9, wbase=40, variant=variant)
    xg, ag = _gpu_chain(p, [7, 5], 4, 2)
    s_ = osys(n, seed=9, order=1)
    for w in range(W):
        xo, ao = _oracle_chain(s_, 40 + w, 12, 4, 2)
        _compare_walker(xg[w], ag[w], xo, ao)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("threads", [64, 128])
def test_split_launches_bitwise_identical(variant, threads):
    n, W = 256, 5
    p = gparams(n, W, seed=3, variant=variant, threads=threads)
    x1, a1 = _gpu_chain(p, [10], 2, 3)
    x2, a2 = _gpu_chain(p, [3, 4, 3], 2, 3)
    assert np.array_equal(x1, x2)
    assert a1.tobytes() == a2.tobytes()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n", [3, 65, 300])
def test_lockstep_spatial_order_ragged_n(variant, n):
    """N = 3, 65, 300 (the sort pads its keys to a power of two; at N < 128
    most lanes own no atom) with atoms re-sorted by cell every sweep: the chain
    still follows the oracle move for move, and a split run is bitwise the same
    as one launch."""
    W = 3
    p = gparams(n, W, threads=128, seed=17, wbase=7, variant=variant)
    assert abi.plan_launch(p)["spatial_order"] == 1
    xg, ag = _gpu_chain(p, [4, 5], 3, 2)
    s_ = osys(n, seed=17)
    for w in range(W):
        xo, ao = _oracle_chain(s_, 7 + w, 9, 3, 2)
        _compare_walker(xg[w], ag[w], xo, ao)
    x1, a1 = _gpu_chain(p, [9], 3, 2)
    assert np.array_equal(x1, xg) and a1.tobytes() == ag.tobytes()


@pytest.mark.parametrize("n,threads", [(512, 64), (1024, 128)])
def test_lockstep_dense_lanes(n, threads):
    """N = 8 x threads: every lane owns eight atoms and the row-sum passes run
    without per-lane bounds checks; the chain still follows the oracle."""
    W = 2
    p = gparams(n, W, threads=threads, seed=23, variant=abi.VARIANT_ROWS)
    xg, ag = _gpu_chain(p, [2, 2], 1, 3)
    s_ = osys(n, seed=23)
    for w in range(W):
        xo, ao = _oracle_chain(s_, w, 4, 1, 3)
        _compare_walker(xg[w], ag[w], xo, ao)


def test_stale_rows_buffer_is_recomputed():
    """A rows buffer that disagrees with u_run is detected and rebuilt: the
    result equals a run that recomputes the rows at every launch."""
    n, W = 256, 2
    p = gparams(n, W, seed=5, variant=abi.VARIANT_ROWS)
    x1, a1 = _gpu_chain(p, [6], 0, 3, keep_rows=False)
    x2, a2 = _gpu_chain(p, [6], 0, 3, keep_rows=True, rows_fill=0.25)
    assert np.array_equal(x1, x2)
    assert a1.tobytes() == a2.tobytes()


@pytest.mark.parametrize("variant", VARIANTS)
def test_n2048_w512_launch_sampled_walkers(variant):
    """The benchmark's launch: N=2048, 512 walkers, FP64, five sweeps with a
    local-energy sample after the fifth; walkers 0, 255 and 511 are replayed by
    the oracle."""
    wl = configs.C2_N2048_FP64
    p = abi.params_for(wl, variant=variant)
    xg, ag = _gpu_chain(p, [5], 0, 5)
    s_ = osys(wl.n, seed=wl.seed)
    picks = [0, 255, 511]
    res = {}

    def work(w):
        res[w] = _oracle_chain(s_, w, 5, 0, 5)

    th = [threading.Thread(target=work, args=(w,)) for w in picks]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for w in picks:
        _compare_walker(xg[w], ag[w], *res[w])
    # every walker moved and sampled once
    assert np.all(ag["n_samples"] == 1) and np.all(ag["n_try"] == 5 * wl.n)
    assert 0.3 < ag["n_acc"].sum() / ag["n_try"].sum() < 0.8


# ---------------------------------------------------------------------------
# ensemble layer

def test_ensemble_matches_stateless_calls():
    n, W = 108, 2
    p = gparams(n, W, seed=4)
    e = abi.Ensemble(p)
    e.run(5)
    e.run(10, energy_every=2, measure=True)
    a = e.acc()
    x = e.coords()
    assert e.sweep_index() == 15
    e.close()
    xg, ag = _gpu_chain(p, [5, 10], 5, 2)
    assert np.array_equal(x, xg)
    assert a.tobytes() == ag.tobytes()


def test_ensemble_from_host_coordinates():
    n, W = 64, 2
    s_ = osys(n)
    xs = np.stack([grid_config(n, s_.L, seed=50 + w) for w in range(W)])
    p = gparams(n, W, seed=2)
    e = abi.Ensemble(p, init_xyz=xs)
    a0 = e.acc()
    for w in range(W):
        U, V = O.totals(s_, xs[w])
        assert a0["u_run"][w] == pytest.approx(U, rel=1e-12)
        assert a0["v_run"][w] == pytest.approx(V, rel=1e-12)
    bad = xs.copy()
    bad[0, 0, 0] = s_.L + 1.0
    with pytest.raises(abi.HevmcError):
        abi.Ensemble(p, init_xyz=bad)
    e.close()


# ---------------------------------------------------------------------------
# checkpoint / resume and failure reporting

@pytest.mark.parametrize("variant", VARIANTS)
def test_checkpoint_through_host_resumes_bitwise(variant):
    """Walker state copied to host memory (coordinates, accumulators, row sums)
    and back into fresh device buffers continues exactly as if never stopped:
    the random stream is keyed by the sweep index, so the sweep counter is the
    only other state (restart as in Sec. 5.4)."""
    n, W = 256, 6
    p = gparams(n, W, seed=17, variant=variant)
    x_ref, a_ref = _gpu_chain(p, [8, 6], 3, 2)
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    abi.sweep(p, coords, acc, 0, 8, 3, 2, rows=rows)
    torch.cuda.synchronize()
    saved = (coords.cpu().numpy().copy(), acc.cpu().numpy().copy(), rows.cpu().numpy().copy())
    del coords, acc, rows
    c2 = torch.from_numpy(saved[0]).cuda()
    a2 = torch.from_numpy(saved[1]).cuda()
    r2 = torch.from_numpy(saved[2]).cuda()
    abi.sweep(p, c2, a2, 8, 6, 3, 2, rows=r2)
    torch.cuda.synchronize()
    assert np.array_equal(c2.cpu().numpy(), x_ref)
    assert abi.acc_to_numpy(a2).tobytes() == a_ref.tobytes()


@pytest.mark.parametrize("threads", [64, 128])
def test_non_finite_state_is_reported(threads):
    """A configuration holding NaN gives non-finite running totals (its pairs
    fail every cutoff test, so without a check they would drop out of the sums
    unnoticed); the ensemble layer reports HEVMC_ESTATE when it synchronises,
    and the stateless calls leave NaN totals on that walker only."""
    n, W = 64, 2
    s_ = osys(n)
    xs = np.stack([grid_config(n, s_.L, seed=w) for w in range(W)])
    xs[1, 0, 5] = np.nan
    p = gparams(n, W, threads=threads)
    c2, a2 = torch.from_numpy(xs).cuda(), torch.zeros((W, abi.ACC_BYTES), dtype=torch.uint8, device="cuda")
    abi.init_walkers(p, c2, a2, fcc_start=False)
    torch.cuda.synchronize()
    a = abi.acc_to_numpy(a2)
    assert np.isfinite(a["u_run"][0]) and np.isnan(a["u_run"][1]) and np.isnan(a["v_run"][1])
    abi.sweep(p, c2, a2, 0, 2, 0, 1)
    torch.cuda.synchronize()
    a = abi.acc_to_numpy(a2)
    assert np.isfinite(a["u_run"][0]) and np.isnan(a["u_run"][1]) and np.isnan(a["v_run"][1])
    coords = torch.from_numpy(xs).cuda()
    acc = torch.zeros((W, abi.ACC_BYTES), dtype=torch.uint8, device="cuda")
    import ctypes as C
    h = C.c_void_p()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert abi.lib().hevmc_create_on(C.byref(p), C.c_void_p(coords.data_ptr()), C.c_void_p(acc.data_ptr()), st,
                                     C.byref(h)) == 0
    assert abi.lib().hevmc_run(h, 3, 0, 0) == 0
    assert abi.lib().hevmc_sync(h) == -5
    assert b"non-finite" in abi.lib().hevmc_last_error()
    assert abi.lib().hevmc_destroy(h) == 0


def test_create_on_keeps_its_row_sums_between_runs():
    """An ensemble on caller-owned buffers keeps the row sums of the row-sum
    sweep in a buffer of its own between runs, as hevmc_create does: two runs
    give the bits of the stateless calls with one rows buffer carried through
    (rebuilding the rows from scratch would change the last bits)."""
    import ctypes as C
    n, W = 256, 4
    p = gparams(n, W, threads=128)
    assert abi.plan_uses_rows(p)
    s_ = osys(n)
    xs = np.stack([grid_config(n, s_.L, seed=w) for w in range(W)])
    c1, a1 = torch.from_numpy(xs).cuda(), torch.zeros((W, abi.ACC_BYTES), dtype=torch.uint8, device="cuda")
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, c1, a1, fcc_start=False, rows=rows)
    abi.sweep(p, c1, a1, 0, 3, abi.NO_MEASURE, 0, rows=rows)
    abi.sweep(p, c1, a1, 3, 4, 3, 2, rows=rows)
    c2, a2 = torch.from_numpy(xs).cuda(), torch.zeros((W, abi.ACC_BYTES), dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert abi.lib().hevmc_create_on(C.byref(p), C.c_void_p(c2.data_ptr()), C.c_void_p(a2.data_ptr()), st,
                                     C.byref(h)) == 0
    assert abi.lib().hevmc_run(h, 3, 0, 0) == 0
    assert abi.lib().hevmc_run(h, 4, 2, 1) == 0
    assert abi.lib().hevmc_sync(h) == 0
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(a1, a2)
    assert abi.lib().hevmc_destroy(h) == 0


def test_a_second_thread_on_a_busy_ensemble_gets_ebusy():
    """While one thread waits in hevmc_sync for a long run, a call on the same
    ensemble from another thread returns HEVMC_EBUSY and does nothing; once the
    first call returns, the ensemble answers again."""
    import ctypes as C
    import threading
    import time
    wl = configs.C2_N2048_FP64
    e = abi.Ensemble(abi.params_for(wl))
    e.run(300)
    res = {}
    th = threading.Thread(target=lambda: res.setdefault("sync", abi.lib().hevmc_sync(e._h)))
    th.start()
    time.sleep(0.3)
    s = C.c_uint32()
    busy = abi.lib().hevmc_get_sweep(e._h, C.byref(s))
    th.join()
    assert busy == -6 and b"in use" in abi.lib().hevmc_last_error()
    assert res["sync"] == 0
    assert e.sweep_index() == 300
    e.close()


@pytest.mark.parametrize("precision,threads", [(abi.FP64, 64), (abi.FP64, 256), (abi.FP32, 128)])
def test_ideal_gas_b_zero_accepts_every_move(precision, threads):
    """The degenerate trial function b = 0 (u = 0, psi constant): every
    Eq. (7) sum is zero, so Eq. (5) accepts every move, and the walkers do
    the oracle's random walk; the local energy is V alone (T = 0)."""
    n, W, sweeps = 108, 4, 3
    p = gparams(n, W, precision=precision, threads=threads, b=0.0)
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    abi.sweep(p, coords, acc, 0, sweeps, 0, 1, rows=rows)
    torch.cuda.synchronize()
    a = abi.acc_to_numpy(acc)
    assert np.all(a["n_acc"] == n * sweeps) and np.all(a["n_try"] == n * sweeps)
    assert np.all(a["sum_tpb"] == 0.0) and np.all(a["sum_tjf"] == 0.0) and np.all(a["sum_tf"] == 0.0)
    fp32 = precision == abi.FP32
    s_ = osys(n, b=0.0, fp32=fp32)
    xs = coords.cpu().numpy().astype(np.float64)
    for w in range(W):
        x = O.fcc_start(s_, w)
        if fp32:
            x = x.astype(np.float32).astype(np.float64)
        for t in range(sweeps):
            for k in range(n):
                sk, _, d = O.draw_move(s_, k, t, w)
                x[:, sk] = O.trial_position(s_, x, sk, d)
                if fp32:
                    x[:, sk] = x[:, sk].astype(np.float32).astype(np.float64)
        tol = 1e-9 if not fp32 else 1e-4
        gap = np.abs(xs[w] - x)
        gap = np.minimum(gap, s_.L - gap)
        assert gap.max() < tol, (w, gap.max())
        el, scale = O.local_energy(s_, xs[w])
        assert el[2] == 0.0 and el[3] == 0.0 and el[4] == 0.0


def test_zero_sweeps_change_nothing():
    """A sweep call of zero sweeps leaves coordinates, accumulators and rows
    as they were, bit for bit."""
    p = gparams(256, 8, threads=128)
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    abi.sweep(p, coords, acc, 0, 2, 0, 1, rows=rows)
    torch.cuda.synchronize()
    c0, a0, r0 = coords.clone(), acc.clone(), rows.clone()
    abi.sweep(p, coords, acc, 2, 0, 0, 1, rows=rows)
    torch.cuda.synchronize()
    assert torch.equal(coords, c0) and torch.equal(acc, a0) and torch.equal(rows, r0)


@pytest.mark.parametrize("wl,threads,variant,spatial", [
    (configs.C2_N2048_FP64, 256, abi.VARIANT_ROWS, 1),
    (configs.C3_N2048_FP32, 256, abi.VARIANT_ROWS, 1),
    (configs.C5_N10976_FP32, 512, abi.VARIANT_ROWS, 0),
    (configs.C1_SMALL_FP64, 64, abi.VARIANT_ROWS, 0),
])
def test_launch_plans_of_the_workloads(wl, threads, variant, spatial):
    """The plans the parity and bench runs rely on: row sums where they fit
    (in registers for N = 10976 FP32, whose LDS holds only the coordinates),
    spatial order where it costs no residency, one wave per small walker."""
    plan = abi.plan_launch(abi.params_for(wl))
    assert (plan["threads"], plan["variant"], plan["spatial_order"]) == (threads, variant, spatial), plan
    assert plan["walkers_per_cu"] >= 1 and plan["lds_per_group"] >= plan["lds_per_walker"]
    if wl is configs.C5_N10976_FP32:
        assert plan["lds_per_walker"] == 3 * 4 * wl.n



@pytest.mark.parametrize("wl", [configs.C2_N2048_FP64, configs.C3_N2048_FP32])
def test_walkers_do_not_depend_on_compute_unit_sharing(wl):
    """In the full launch two walkers share each compute unit and trade issue
    priority by progress; launched four at a time, a walker has a compute unit
    to itself.  Scheduling is all that differs: walkers 0-3 leave both launches
    with the same bits."""
    out = []
    for W in (wl.walkers, 4):
        p = abi.params_for(wl, n_walkers=W)
        assert abi.plan_launch(p)["walkers_per_cu"] == (2 if W == wl.walkers else 1)
        coords, acc = abi.alloc_state(p)
        rows = abi.alloc_rows(p)
        abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
        abi.sweep(p, coords, acc, 0, 2, 0, 2, rows=rows)
        torch.cuda.synchronize()
        out.append((coords[:4].cpu().numpy(), abi.acc_to_numpy(acc)[:4], rows[:4].cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1].tobytes() == out[1][1].tobytes()
    assert np.array_equal(out[0][2], out[1][2])
