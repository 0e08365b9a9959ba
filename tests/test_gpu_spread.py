"""Spread walkers: one walker over several workgroups of a cooperative launch
(the cooperative kernel of Sec. 3, across compute units), for walkers whose
coordinates fit in no workgroup's LDS.  Held to the oracle like the
single-workgroup sweep:

  * start and local energy: FP64 values within 1e-12 of the oracle's scale;
  * every micro-update of an FP64 sweep (plain form: dU and dV of every move)
    in lockstep with the oracle's own chain, at 1e-12 of the summed
    magnitudes, and the sample that ends it;
  * an FP32 walker beyond one workgroup (coordinates in FP32) move by move
    within the FP32 bounds, up to the first decision that rounding could flip;
  * a wait that gives up (forced from the host by a zero poll limit) ends
    the call with HEVMC_EDEVICE, every workgroup having left the kernel, and
    the library works normally afterwards.
"""
import threading

import numpy as np
import pytest

import oracle as O
from paper_1312_1282_amd import abi, configs
from test_gpu_movelog import compare_fp32, compare_fp64, _xi_logs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RHO = configs.RHO_EQ
B = configs.C1_SMALL_FP64.b
STEP = configs.C1_SMALL_FP64.step_sigma


def params(n, W, precision=abi.FP64, seed=17, threads=0):
    return abi.make_params(n, W, precision=precision, density=RHO, b=B, step_sigma=STEP, seed=seed,
                           threads=threads)


def osys(n, seed=17, fp32=False):
    return O.system(n, O.box_side(n, RHO, fp32), B, hbar2_over_m=configs.HBAR2_OVER_M, step_sigma=STEP,
                    seed=seed, fp32_coords=fp32)


def test_spread_plans():
    p = params(8000, 2)
    plan = abi.plan_launch(p)
    assert (plan["slices"], plan["threads"], plan["variant"], plan["spatial_order"]) == (2, 512, abi.VARIANT_PLAIN, 0)
    assert plan["lds_per_group"] >= 3 * 4000 * 8 and plan["lds_per_group"] <= 160 * 1024
    for t in (256, 1024):
        assert abi.plan_launch(params(8000, 2, threads=t))["threads"] == t
    assert abi.plan_launch(params(40960, 1, abi.FP32))["slices"] == 4
    # beyond 14 slices' LDS the walker does not fit at all
    with pytest.raises(abi.HevmcError) as ei:
        abi.plan_launch(params(100000, 1))
    assert ei.value.code == -3
    assert abi.plan_launch(params(14000, 1, abi.FP32))["slices"] == 2
    assert abi.plan_launch(params(2048, 1))["slices"] == 1
    assert abi.plan_launch(params(13000, 1, abi.FP32))["slices"] == 1   # rows in registers, one workgroup


def test_spread_start_and_local_energy_follow_the_oracle():
    n, W = 8000, 2
    p = params(n, W)
    coords, acc = abi.alloc_state(p)
    abi.init_walkers(p, coords, acc, fcc_start=True)
    out = torch.zeros((W, 6), dtype=torch.float64, device="cuda")
    abi.local_energy(p, coords, out)
    torch.cuda.synchronize()
    xs = coords.cpu().numpy()
    a = abi.acc_to_numpy(acc)
    el_g = out.cpu().numpy()
    s_ = osys(n)
    for w in range(W):
        ref = O.fcc_start(s_, w)
        assert np.max(np.abs(xs[w] - ref)) <= 1e-13 * s_.L
        el, scale = O.local_energy(s_, xs[w])
        assert np.all(np.abs(el_g[w] - el) <= 1e-12 * scale), (el_g[w], el)
        U, V = el[5], el[1]
        assert a["u_run"][w] == pytest.approx(U, rel=1e-12)
        assert a["v_run"][w] == pytest.approx(V, rel=1e-12)
        assert a["n_try"][w] == 0 and a["sum_e"][w] == 0


def _oracle_logs(s_, walkers, n_sweeps, measure_start, m):
    res = {}

    def work(w):
        x = O.fcc_start(s_, w)
        a = O.walker_init(s_, x)
        res[w] = (O.run_walker_log(s_, w, x, a, 0, n_sweeps, measure_start, m), a, x)

    th = [threading.Thread(target=work, args=(w,)) for w in walkers]
    for t in th:
        t.start()
    for t in th:
        t.join()
    return res


@pytest.mark.parametrize("threads", [0, 256, 1024])
def test_spread_every_move_follows_the_oracle_fp64(threads):
    """N = 8000 in FP64 (192 KB of coordinates, two workgroups), two walkers,
    one measured sweep with the local-energy sample that ends it; workgroups
    of the library's size (512 threads), of 256 and of 1024."""
    n, W = 8000, 2
    p = params(n, W, threads=threads)
    coords, acc = abi.alloc_state(p)
    abi.init_walkers(p, coords, acc, fcc_start=True)
    log = torch.full((W, n, 4), float("nan"), dtype=torch.float64, device="cuda")
    abi.sweep(p, coords, acc, 0, 1, 0, 1, movelog=log)
    torch.cuda.synchronize()
    g = log.cpu().numpy()
    xs = coords.cpu().numpy()
    ag = abi.acc_to_numpy(acc)
    o = _oracle_logs(osys(n), range(W), 1, 0, 1)
    for w in range(W):
        rec, a, x = o[w]
        compare_fp64(g[w], rec, rows_form=False)
        assert ag["n_acc"][w] == a.n_acc and ag["n_try"][w] == a.n_try == n
        assert ag["n_samples"][w] == a.n_samples == 1
        assert np.max(np.abs(xs[w] - x)) < 1e-9
        assert ag["sum_e"][w] + ag["c_e"][w] == pytest.approx(a.sum_e + a.c_e, rel=1e-10)
        assert ag["sum_vs"][w] + ag["c_vs"][w] == pytest.approx(a.sum_vs + a.c_vs, rel=1e-10)
    assert 0.35 < g[:, :, 1].mean() < 0.7


def _repeat_counts(s_, wid, n):
    """Moves of sweep 0 of walker id wid whose atom is the previous move's
    (s_{m+1} = s_m) or the one before (s_{m+1} = s_{m-1})."""
    s = [O.draw_move(s_, k, 0, wid)[0] for k in range(n)]
    same = sum(s[m + 1] == s[m] for m in range(n - 1))
    back = sum(s[m + 1] == s[m - 1] != s[m] for m in range(1, n - 1))
    return same, back


def test_spread_repeated_atoms_follow_the_oracle():
    """A move of the same atom again takes its old position from the outcome
    of the move before (nobody publishes it), and a move of the atom two
    moves back reads the position its holder published after that move's
    decision.  Walkers whose sweep has several of each are picked from the
    move stream and run move by move against the oracle."""
    n = 8000
    s_ = osys(n)
    picked = []
    for wid in range(400):
        same, back = _repeat_counts(s_, wid, n)
        if same >= 2 and back >= 2:
            picked.append(wid)
        if len(picked) == 2:
            break
    assert len(picked) == 2
    for wid in picked:
        p = abi.make_params(n, 1, precision=abi.FP64, density=RHO, b=B, step_sigma=STEP, seed=17,
                            walker_id_base=wid)
        assert abi.plan_launch(p)["slices"] == 2
        coords, acc = abi.alloc_state(p)
        x0 = O.fcc_start(s_, wid)
        coords.copy_(torch.from_numpy(x0[None]).cuda())
        abi.init_walkers(p, coords, acc, fcc_start=False)
        log = torch.full((1, n, 4), float("nan"), dtype=torch.float64, device="cuda")
        abi.sweep(p, coords, acc, 0, 1, movelog=log)
        torch.cuda.synchronize()
        a = O.walker_init(s_, x0.copy())
        x = x0.copy()
        rec = O.run_walker_log(s_, wid, x, a, 0, 1, 0xFFFFFFFF, 0)
        compare_fp64(log.cpu().numpy()[0], rec, rows_form=False)
        assert np.max(np.abs(coords.cpu().numpy()[0] - x)) < 1e-9


def test_spread_sequential_order_follows_the_oracle():
    """Atoms moved in label order (s = k, Sec. 2's alternative to random
    selection): the next move's atom is always another one, so every old
    position comes from the mailbox; one sweep move by move."""
    n = 8000
    p = abi.make_params(n, 1, precision=abi.FP64, density=RHO, b=B, step_sigma=STEP, seed=17,
                        order=abi.SELECT_SEQUENTIAL)
    assert abi.plan_launch(p)["slices"] == 2
    coords, acc = abi.alloc_state(p)
    abi.init_walkers(p, coords, acc, fcc_start=True)
    log = torch.full((1, n, 4), float("nan"), dtype=torch.float64, device="cuda")
    abi.sweep(p, coords, acc, 0, 1, movelog=log)
    torch.cuda.synchronize()
    s_ = O.system(n, O.box_side(n, RHO), B, hbar2_over_m=configs.HBAR2_OVER_M, step_sigma=STEP, seed=17,
                  order=1)
    x = O.fcc_start(s_, 0)
    a = O.walker_init(s_, x)
    rec = O.run_walker_log(s_, 0, x, a, 0, 1, 0xFFFFFFFF, 0)
    g = log.cpu().numpy()[0]
    assert np.array_equal(g[:, 0], np.arange(n, dtype=np.float64))
    compare_fp64(g, rec, rows_form=False)
    assert np.max(np.abs(coords.cpu().numpy()[0] - x)) < 1e-9


def test_spread_every_move_follows_the_oracle_fp32():
    """N = 14000 in FP32 (168 KB of coordinates, two workgroups), one walker,
    one sweep, move by move within the FP32 bounds."""
    n = 14000
    p = params(n, 1, abi.FP32)
    assert abi.plan_launch(p)["slices"] == 2
    coords, acc = abi.alloc_state(p)
    abi.init_walkers(p, coords, acc, fcc_start=True)
    log = torch.full((1, n, 4), float("nan"), dtype=torch.float64, device="cuda")
    abi.sweep(p, coords, acc, 0, 1, movelog=log)
    torch.cuda.synchronize()
    s_ = osys(n, fp32=True)
    o = _oracle_logs(s_, [0], 1, 0xFFFFFFFF, 0)
    xl = _xi_logs(s_, 0, n, n)
    end, _ = compare_fp32(log.cpu().numpy()[0], o[0][0], xl, False, min_moves=n // 4, L=s_.L)


def test_spread_ensemble_matches_the_stateless_calls():
    """The ensemble layer runs spread walkers through the same calls: an
    owning ensemble started from given coordinates gives the bits of
    hevmc_init_walkers + hevmc_sweep on the same coordinates."""
    n, W = 8000, 2
    p = params(n, W)
    s_ = osys(n)
    xs = np.stack([O.fcc_start(s_, w) for w in range(W)])
    e = abi.Ensemble(p, init_xyz=xs)
    e.run(1, energy_every=1, measure=True)
    e.sync()
    a_e, x_e = e.acc(), e.coords()
    e.close()
    coords, acc = abi.alloc_state(p)
    coords.copy_(torch.from_numpy(xs).cuda())
    abi.init_walkers(p, coords, acc, fcc_start=False)
    abi.sweep(p, coords, acc, 0, 1, 0, 1)
    torch.cuda.synchronize()
    a_s = abi.acc_to_numpy(acc)
    assert np.array_equal(x_e, coords.cpu().numpy())
    for f in abi.ACC_FIELDS + abi.ACC_INT_FIELDS:
        assert np.array_equal(a_e[f], a_s[f]), f
    assert np.all(a_s["n_samples"] == 1) and np.all(a_s["n_try"] == n)


def test_spread_trace_and_pair_histogram_follow_the_oracle():
    """Per-sample records (hevmc_sweep_trace) and the pair histogram
    (hevmc_sweep_gr) of spread walkers come from their local-energy kernels:
    both follow the oracle's chain over two sampled sweeps, and neither
    changes the chain."""
    n, W, sweeps, nb, cap = 8000, 2, 2, 80, 4
    p = params(n, W)

    def run(trace=None, gr=None):
        coords, acc = abi.alloc_state(p)
        abi.init_walkers(p, coords, acc, fcc_start=True)
        abi.sweep(p, coords, acc, 0, sweeps, 0, 1, trace=trace, gr=gr)
        torch.cuda.synchronize()
        return coords.cpu().numpy(), abi.acc_to_numpy(acc)

    tr = torch.full((W, cap, 6), -1.0, dtype=torch.float64, device="cuda")
    gr = torch.zeros((W, nb), dtype=torch.int64, device="cuda")
    x_t, a_t = run(trace=tr)
    x_g, a_g = run(gr=gr)
    x_0, a_0 = run()
    assert np.array_equal(x_t, x_0) and np.array_equal(x_g, x_0)
    assert a_t.tobytes() == a_0.tobytes() and a_g.tobytes() == a_0.tobytes()
    tr, gr = tr.cpu().numpy(), gr.cpu().numpy()
    s_ = osys(n)
    for w in range(W):
        x = O.fcc_start(s_, w)
        a = O.walker_init(s_, x)
        rec, ref, edge = [], np.zeros(nb, dtype=np.int64), np.zeros(nb + 1, dtype=np.int64)
        for t in range(sweeps):
            O.run_walker(s_, w, x, a, t, 1, 0, 1)
            rec.append(O.local_energy(s_, x)[0])
            h, e = O.pair_histogram(s_, x, nb, rel_window=1e-8)
            ref += np.asarray(h, dtype=np.int64)
            edge += np.asarray(e, dtype=np.int64)
        np.testing.assert_allclose(tr[w, :sweeps], np.array(rec), rtol=1e-10, atol=1e-8)
        assert np.all(tr[w, sweeps:] == -1.0)
        slack = edge[:-1] + edge[1:]
        assert np.all(np.abs(gr[w] - ref) <= slack), (w, np.nonzero(np.abs(gr[w] - ref) > slack)[0][:5])
        assert ref.sum() > 0 and abs(int(gr[w].sum()) - int(ref.sum())) <= int(edge[-1])


def test_spread_wait_that_gives_up_is_reported(monkeypatch):
    """A zero poll limit (forced from the host): a workgroup that finds the
    others not yet arrived gives up at once, the others give up in turn, and
    the call reports HEVMC_EDEVICE; a normal call then runs."""
    n, W = 8000, 2
    p = params(n, W)
    coords, acc = abi.alloc_state(p)
    abi.init_walkers(p, coords, acc, fcc_start=True)
    monkeypatch.setenv("HEVMC_SPREAD_SPIN_CAP", "0")
    with pytest.raises(abi.HevmcError) as ei:
        abi.sweep(p, coords, acc, 0, 1)
    assert ei.value.code == -4 and "gave up" in str(ei.value)
    monkeypatch.delenv("HEVMC_SPREAD_SPIN_CAP")
    abi.init_walkers(p, coords, acc, fcc_start=True)
    abi.sweep(p, coords, acc, 0, 1)
    torch.cuda.synchronize()
    a = abi.acc_to_numpy(acc)
    assert np.all(np.isfinite(a["u_run"]))
