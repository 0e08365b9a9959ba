"""Move-by-move parity of the sweep kernel against the oracle (Eqs. (5), (7)).

The sweep runs through hevmc_sweep_log, the same kernel and launch plan that
hevmc_sweep (and bench.py) use, with a record of every micro-update of the
first walkers: (s, accepted, dU, dV).  The oracle runs its own chain from the
same start with the same random stream (or_run_walker_log) and records the
same quantities at the configurations it generates itself.  Nothing from the
GPU enters the oracle: the two chains agree move for move because they make
the same decisions.

Bars:
  * FP64: every move in lockstep (same atom, same decision), and
      |dU_gpu - dU_or| <= 1e-12 max(|dU_or|, sum_i |u'_i| + |u_i|)
    for every move, dV likewise with |V| terms (for every move in the PLAIN
    form, for accepted moves in the row-sum forms, which form dV only there).
    In the row-sum forms dU is the forward sum minus the moved atom's row,
    updated move by move: the runs here take 60 or more sweeps with no
    local-energy pass, so no row is ever refreshed, and a drifting row fails.
  * FP32 form (pair terms in FP32, sums in FP64, coordinates FP32): the
    oracle keeps its coordinates in FP32 too (fp32_coords) and computes in
    FP64.  Two error sources per pair term:
      - the FP32 arithmetic on a given distance (reciprocal square root and
        reciprocal to an ulp, a few roundings): within ~1e-6 of the term;
      - the distance itself: a coordinate difference is rounded in FP32
        before the image is taken, so a pair that meets across the box (the
        difference near L, its image L - |d| small) carries an absolute
        error of up to half an FP32 ulp of L per component, about one ulp of
        L in r.  The term then moves by |du/dr| times that.
    Hence, with the oracle's scales and slopes of the same move,
      |dU_gpu - dU_or| <= 2e-6 max(|dU_or|, scale_u) + 2 ulp(L) slope_u,
      |dV_gpu - dV_or| <= 1e-5 max(|dV_or|, scale_v) + 2 ulp(L) slope_v
    (the potential adds two exponentials in FP32).  A decision can then flip
    where 2 dU lies within that bound of ln xi: the chains are compared up to
    the first differing decision, which must be such a near tie.
"""
import math
import threading

import numpy as np
import pytest

import oracle as O
from paper_1312_1282_amd import abi, configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RHO = configs.RHO_EQ
B = configs.C1_SMALL_FP64.b
STEP = configs.C1_SMALL_FP64.step_sigma


def osys(n, seed, fp32=False, b=B, rho=RHO, step=STEP):
    return O.system(n, O.box_side(n, rho, fp32), b, hbar2_over_m=configs.HBAR2_OVER_M, step_sigma=step,
                    seed=seed, fp32_coords=fp32)


def gpu_log(p, n_sweeps, log_walkers, measure_start=abi.NO_MEASURE, m=0):
    """Fresh fcc start, one logged launch of n_sweeps sweeps; (log, acc)."""
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    log = torch.full((log_walkers, n_sweeps * p.n, 4), float("nan"), dtype=torch.float64, device="cuda")
    abi.sweep(p, coords, acc, 0, n_sweeps, measure_start, m, rows=rows, movelog=log)
    torch.cuda.synchronize()
    return log.cpu().numpy(), abi.acc_to_numpy(acc)


def oracle_logs(s_, walkers, n_sweeps, measure_start=0xFFFFFFFF, m=0):
    """Oracle chains of the given walker ids from their fcc starts, in threads."""
    res = {}

    def work(w):
        x = O.fcc_start(s_, w)
        a = O.walker_init(s_, x)
        res[w] = (O.run_walker_log(s_, w, x, a, 0, n_sweeps, measure_start, m), a)

    th = [threading.Thread(target=work, args=(w,)) for w in walkers]
    for t in th:
        t.start()
    for t in th:
        t.join()
    return res


def compare_fp64(g, o, rows_form):
    """g: GPU records (moves, 4); o: oracle records (moves, 8)."""
    assert np.array_equal(g[:, 0], o[:, 0]), "moved atoms differ"
    assert np.array_equal(g[:, 1], o[:, 1]), f"decisions differ at {np.nonzero(g[:, 1] != o[:, 1])[0][:5]}"
    err_u = np.abs(g[:, 2] - o[:, 2]) / np.maximum(np.abs(o[:, 2]), o[:, 4])
    assert err_u.max() <= 1e-12, (int(err_u.argmax()), float(err_u.max()))
    acc = o[:, 1] == 1
    sel = acc if rows_form else np.ones(len(o), bool)
    err_v = np.abs(g[sel, 3] - o[sel, 3]) / np.maximum(np.abs(o[sel, 3]), o[sel, 5])
    assert err_v.max() <= 1e-12, float(err_v.max())
    if rows_form:
        assert np.all(np.isnan(g[~acc, 3])), "the row-sum forms form no dV for rejected moves"
    return float(err_u.max()), float(err_v.max())


@pytest.mark.parametrize("n,W,threads,sweeps,variant", [
    (108, 4, 64, 200, abi.VARIANT_ROWS),    # one wavefront per walker, few-chunk row passes
    (108, 4, 64, 200, abi.VARIANT_PLAIN),
    (256, 3, 128, 100, abi.VARIANT_ROWS),   # spatial order
    (256, 3, 128, 100, abi.VARIANT_PLAIN),
    (300, 2, 256, 60, abi.VARIANT_ROWS),    # ragged: some lanes own fewer atoms
    (1024, 2, 128, 60, abi.VARIANT_ROWS),   # eight atoms per lane (dense passes)
    (4096, 1, 512, 2, abi.VARIANT_ROWS),    # eight atoms per lane at 512 threads: accept pass in pairs
])
def test_every_move_follows_the_oracle_fp64(n, W, threads, sweeps, variant):
    p = abi.make_params(n, W, density=RHO, b=B, step_sigma=STEP, seed=31, threads=threads, variant=variant)
    plan = abi.plan_launch(p)
    assert plan["variant"] == variant
    g, _ = gpu_log(p, sweeps, W)
    o = oracle_logs(osys(n, 31), range(W), sweeps)
    for w in range(W):
        compare_fp64(g[w], o[w][0], variant == abi.VARIANT_ROWS)
    assert 0.35 < g[:, :, 1].mean() < 0.7


def test_every_move_of_the_benchmark_launch_fp64():
    """The benchmark's plan (N=2048, 512 walkers, FP64, 256 threads, row sums,
    spatial order, dense lanes, two walkers per compute unit): 60 sweeps with
    no local-energy pass, walkers 0 and 1 replayed move by move (245 760
    micro-updates, none of whose rows is refreshed)."""
    wl = configs.C2_N2048_FP64
    p = abi.params_for(wl)
    plan = abi.plan_launch(p)
    assert (plan["threads"], plan["variant"], plan["spatial_order"], plan["walkers_per_cu"]) == \
        (256, abi.VARIANT_ROWS, 1, 2), plan
    sweeps = 60
    g, ag = gpu_log(p, sweeps, 2, measure_start=0, m=0)
    o = oracle_logs(osys(wl.n, wl.seed), [0, 1], sweeps, measure_start=0, m=0)
    for w in (0, 1):
        compare_fp64(g[w], o[w][0], True)
        assert ag["n_acc"][w] == o[w][1].n_acc and ag["n_try"][w] == o[w][1].n_try == sweeps * wl.n
        assert ag["u_run"][w] == pytest.approx(o[w][1].u_run, rel=1e-10, abs=1e-9)


def test_plain_sweep_odd_n_across_sweep_ends():
    """N = 4099 (odd, beyond the row-sum and spatial-order limits of 512
    threads): the plain form with eight waves per walker, whose reduction
    buffers alternate move by move across sweep ends; three sweeps, the only
    local-energy sample after the third, every move compared."""
    n, W = 4099, 2
    p = abi.make_params(n, W, density=RHO, b=B, step_sigma=STEP, seed=41, threads=512)
    plan = abi.plan_launch(p)
    assert (plan["variant"], plan["spatial_order"]) == (abi.VARIANT_PLAIN, 0), plan
    g, ag = gpu_log(p, 3, W, measure_start=0, m=3)
    o = oracle_logs(osys(n, 41), range(W), 3, measure_start=0, m=3)
    for w in range(W):
        compare_fp64(g[w], o[w][0], False)
        a = o[w][1]
        assert ag["n_samples"][w] == a.n_samples == 1
        assert ag["sum_e"][w] + ag["c_e"][w] == pytest.approx(a.sum_e + a.c_e, rel=1e-10)


def test_log_leaves_the_chain_unchanged():
    """Recording is an output only: coordinates and accumulators are bitwise
    those of hevmc_sweep, and walkers past log_walkers are not written."""
    n, W = 256, 4
    p = abi.make_params(n, W, density=RHO, b=B, step_sigma=STEP, seed=8, threads=128)
    out = []
    for logged in (False, True):
        coords, acc = abi.alloc_state(p)
        rows = abi.alloc_rows(p)
        abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
        log = torch.full((2, 5 * n, 4), -7.0, dtype=torch.float64, device="cuda") if logged else None
        abi.sweep(p, coords, acc, 0, 5, 1, 2, rows=rows, movelog=log)
        torch.cuda.synchronize()
        out.append((coords.cpu().numpy(), abi.acc_to_numpy(acc).tobytes()))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_log_capacity_and_arguments():
    n, W = 64, 2
    p = abi.make_params(n, W, density=RHO, b=B, step_sigma=STEP, seed=8, threads=64)
    coords, acc = abi.alloc_state(p)
    abi.init_walkers(p, coords, acc, fcc_start=True)
    log = torch.full((1, 100, 4), -7.0, dtype=torch.float64, device="cuda")
    abi.sweep(p, coords, acc, 0, 3, movelog=log)
    torch.cuda.synchronize()
    l = log.cpu().numpy()
    assert np.all(l[0, :, 0] >= 0) and np.all(l[0, :, 0] < n)   # all 100 records written
    with pytest.raises(abi.HevmcError):
        abi.sweep(p, coords, acc, 0, 1, movelog=torch.zeros((3, 10, 4), dtype=torch.float64, device="cuda"))


# ---------------------------------------------------------------------------
# FP32 form

def fp32_bounds(o, L):
    """Per-move FP32 bounds on dU and dV (see the module docstring)."""
    ulp_L = float(np.spacing(np.float32(L)))
    bu = 2e-6 * np.maximum(np.abs(o[:, 2]), o[:, 4]) + 2.0 * ulp_L * o[:, 6]
    bv = 1e-5 * np.maximum(np.abs(o[:, 3]), o[:, 5]) + 2.0 * ulp_L * o[:, 7]
    return bu, bv


def compare_fp32(g, o, xi_log, rows_form, min_moves, L):
    """Compare up to the first differing decision, which must be a near tie.
    xi_log: ln xi of every move (from the oracle's stream)."""
    bu, bv = fp32_bounds(o, L)
    diff = np.nonzero((g[:, 0] != o[:, 0]) | (g[:, 1] != o[:, 1]))[0]
    end = int(diff[0]) if len(diff) else len(o)
    if end < len(o):
        q = end
        assert g[q, 0] == o[q, 0], "the moved atoms differ before any decision did"
        margin = abs(2.0 * o[q, 2] - xi_log[q])
        assert margin <= 2.0 * bu[q], ("a decision flipped away from a tie", q, margin)
    assert end >= min_moves, (end, min_moves)
    g, o, bu, bv = g[:end], o[:end], bu[:end], bv[:end]
    ratio_u = np.abs(g[:, 2] - o[:, 2]) / bu
    assert ratio_u.max() <= 1.0, (int(ratio_u.argmax()), float(ratio_u.max()))
    acc = o[:, 1] == 1
    sel = acc if rows_form else np.ones(len(o), bool)
    ratio_v = np.abs(g[sel, 3] - o[sel, 3]) / bv[sel]
    assert ratio_v.max() <= 1.0, float(ratio_v.max())
    return end, float(ratio_u.max())


def _xi_logs(s_, w, moves, n):
    return np.array([math.log(O.draw_move(s_, q % n, q // n, w)[1]) for q in range(moves)])


@pytest.mark.parametrize("wl,sweeps,walkers", [
    (configs.C3_N2048_FP32, 20, [0, 1]),     # the FP32 benchmark plan: rows in LDS, register copies
    (configs.C5_N10976_FP32, 2, [0]),        # rows in registers (512 threads, 22 rows per lane)
])
def test_every_move_follows_the_oracle_fp32(wl, sweeps, walkers):
    p = abi.params_for(wl)
    plan = abi.plan_launch(p)
    assert plan["variant"] == abi.VARIANT_ROWS
    g, _ = gpu_log(p, sweeps, len(walkers))
    s_ = osys(wl.n, wl.seed, fp32=True)
    o = oracle_logs(s_, walkers, sweeps)
    for i, w in enumerate(walkers):
        xl = _xi_logs(s_, w, sweeps * wl.n, wl.n)
        end, _ = compare_fp32(g[i], o[w][0], xl, True, min_moves=wl.n, L=s_.L)
