"""GPU tests of the FP32 precision form against the FP64 oracle.

The FP32 form keeps coordinates and pair terms (distances, u, V and their
derivatives) in FP32 and every sum in FP64.  The oracle is evaluated on the same
float-rounded coordinates, in the box whose side is rounded to FP32.

Tolerances, from the FP32 arithmetic (unit roundoff u32 = 2^-24 = 6.0e-8):
  * a rational pair term (u, its derivatives, the dispersion part of V) passes
    through ~10 roundings and the hardware reciprocal / reciprocal square root
    (1 ulp each): relative error <= ~16 u32 = 1e-6, so sums of such terms are
    within 2e-6 of the sum of their magnitudes;
  * the exponentials of V take an argument with error ~|arg| u32, |arg| up to
    ~100 inside the cutoff: V sums within 1e-5 of the sum of |V|;
  * local-energy components within 2e-6 of the oracle's scale, and the local
    energy per atom within 0.5 mK (the form's target is 1 mK/atom).
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
KELVIN_TO_MK = 1e3


def osys32(n, seed=1, step=STEP):
    return O.system(n, O.box_side(n, RHO, fp32=True), B, hbar2_over_m=configs.HBAR2_OVER_M, step_sigma=step,
                    seed=seed)


def within(got, ref, scale, rel):
    return abs(got - ref) <= rel * max(abs(ref), scale)


@pytest.mark.parametrize("n,threads", [(108, 128), (500, 128), (2048, 256), (2048, 512)])
def test_fp32_move_sums(n, threads):
    W = 6
    s_ = osys32(n)
    xs = np.stack([grid_config(n, s_.L, seed=300 + n + w, dtype=np.float32) for w in range(W)])
    ss, dd = moves(n, W, 0.8, seed=31 + n)
    p = abi.make_params(n, W, precision=abi.FP32, threads=threads)
    out = torch.zeros((W, 2), dtype=torch.float64, device="cuda")
    abi.move_delta(p, torch.from_numpy(xs).cuda(), torch.from_numpy(ss).cuda(), torch.from_numpy(dd).cuda(), out)
    out = out.cpu().numpy()
    for w in range(W):
        x64 = xs[w].astype(np.float64)
        rnew = O.trial_position(s_, x64, ss[w], dd[w]).astype(np.float32).astype(np.float64)
        du, dv, su, sv = O.delta(s_, x64, ss[w], rnew)
        assert within(out[w, 0], du, su, 2e-6), (w, out[w, 0], du, su)
        assert within(out[w, 1], dv, sv, 1e-5), (w, out[w, 1], dv, sv)


@pytest.mark.parametrize("n,threads", [(108, 128), (864, 128), (2048, 256), (14000, 0)])
def test_fp32_local_energy(n, threads):
    """Also N = 14000, a walker spread over two workgroups, whose local energy
    runs in the split kernels (blocks of atoms, then the per-walker finish)."""
    W = 4 if n <= 2048 else 2
    s_ = osys32(n)
    xs = np.stack([grid_config(n, s_.L, seed=400 + n + w, dtype=np.float32) for w in range(W)])
    p = abi.make_params(n, W, precision=abi.FP32, threads=threads)
    out = torch.zeros((W, 6), dtype=torch.float64, device="cuda")
    abi.local_energy(p, torch.from_numpy(xs).cuda(), out)
    out = out.cpu().numpy()
    worst = 0.0
    for w in range(W):
        ref, scale = O.local_energy(s_, xs[w].astype(np.float64))
        for q in range(6):
            assert within(out[w, q], ref[q], scale, 2e-6), (w, q, out[w, q], ref[q], scale)
        worst = max(worst, abs(out[w, 0] - ref[0]) / n * KELVIN_TO_MK)
    assert worst < 0.5, f"E_L error {worst:.3f} mK/atom"


def _launch_and_check_samples(wl, picks, sweeps, threads=0, variant=abi.VARIANT_AUTO):
    """One launch of `sweeps` sweeps with a local-energy sample after the last,
    at the workload's full size; the sampled walkers' E_L, V and U are checked
    against the oracle evaluated on the walkers' final coordinates."""
    p = abi.params_for(wl, threads=threads, variant=variant)
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    abi.sweep(p, coords, acc, 0, sweeps, 0, sweeps, rows=rows)
    torch.cuda.synchronize()
    a = abi.acc_to_numpy(acc)
    assert np.all(a["n_samples"] == 1) and np.all(a["n_try"] == sweeps * wl.n)
    x = coords.cpu().numpy()
    s_ = osys32(wl.n)
    res = {}

    def work(w):
        res[w] = O.local_energy(s_, x[w].astype(np.float64))

    th = [threading.Thread(target=work, args=(w,)) for w in picks]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for w in picks:
        ref, scale = res[w]
        e = a["sum_e"][w] + a["c_e"][w]
        assert within(e, ref[0], scale, 2e-6)
        assert abs(e - ref[0]) / wl.n * KELVIN_TO_MK < 0.5
        assert within(a["v_run"][w], ref[1], scale, 2e-6)
        assert within(a["u_run"][w], ref[5], scale, 2e-6)
    return a


@pytest.mark.parametrize("n,threads", [(1024, 128), (2048, 256), (2048, 512), (8192, 512), (10976, 512)])
def test_fp32_running_totals_follow_the_moves(n, threads):
    """Sweeps with no sample, so u_run and v_run are the initial sums plus every
    accepted move's dU and dV.  The FP32 pair value of a pair is the same from
    either atom and until one of them moves, so the running totals telescope to
    the FP32 sums over the final configuration: each is within the static
    tolerance of the oracle's U and V there.  A stale copy of any atom's
    position or row in any pass would break the telescoping by a whole pair
    term (covers the register copies of the dense-lane passes, N = 8 x threads,
    the LDS passes, N = 4 x threads, and the rows kept in registers because
    they do not fit in LDS, N = 8192 and 10976 at 512 threads)."""
    W, sweeps = (3, 3) if n <= 2048 else (2, 2)
    p = abi.make_params(n, W, precision=abi.FP32, threads=threads, variant=abi.VARIANT_ROWS, density=RHO, b=B,
                        step_sigma=STEP, seed=11)
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    abi.sweep(p, coords, acc, 0, 1, abi.NO_MEASURE, 0, rows=rows)
    abi.sweep(p, coords, acc, 1, sweeps - 1, abi.NO_MEASURE, 0, rows=rows)
    torch.cuda.synchronize()
    a = abi.acc_to_numpy(acc)
    assert np.all(a["n_samples"] == 0)
    x = coords.cpu().numpy()
    s_ = osys32(n, seed=11)
    res = {}

    def work(w):
        res[w] = O.local_energy(s_, x[w].astype(np.float64))

    th = [threading.Thread(target=work, args=(w,)) for w in range(W)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for w in range(W):
        ref, scale = res[w]
        assert within(a["u_run"][w], ref[5], scale, 2e-6), (w, a["u_run"][w], ref[5], scale)
        assert within(a["v_run"][w], ref[1], scale, 1e-5), (w, a["v_run"][w], ref[1], scale)


def test_fp32_n2048_w1024_launch_sampled_walkers():
    wl = configs.C3_N2048_FP32
    a = _launch_and_check_samples(wl, [0, 511, 1023], 5)
    assert 0.3 < a["n_acc"].sum() / a["n_try"].sum() < 0.8


def test_fp32_n10976_w256_launch_sampled_walkers():
    wl = configs.C5_N10976_FP32
    _launch_and_check_samples(wl, [0, 255], 1)


def test_fp32_chain_against_fp64_chain():
    """FP32 and FP64 chains on identical seeds and walker ids sample the same
    distribution: the ensemble energies per atom agree within 3 combined
    (walker-paired) standard errors.  The chains share their first moves and
    part ways at the first decision that the FP32 rounding flips, so this is a
    statistical check; the FP32 form's own error in mK/atom is bounded per
    configuration by the tests above."""
    n, W = 256, 1024
    res = {}
    for prec in (abi.FP64, abi.FP32):
        p = abi.make_params(n, W, precision=prec, step_sigma=STEP, seed=11)
        coords, acc = abi.alloc_state(p)
        rows = abi.alloc_rows(p)
        abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
        abi.sweep(p, coords, acc, 0, 100, abi.NO_MEASURE, 0, rows=rows)
        abi.sweep(p, coords, acc, 100, 200, 100, 5, rows=rows)
        torch.cuda.synchronize()
        a = abi.acc_to_numpy(acc)
        res[prec] = (a["sum_e"] + a["c_e"]) / a["n_samples"] / n
    d = res[abi.FP32] - res[abi.FP64]
    se = d.std(ddof=1) / np.sqrt(W)
    assert abs(d.mean()) <= 3 * se + 1e-9, (d.mean() * KELVIN_TO_MK, se * KELVIN_TO_MK)


def test_fp32_form_against_fp64_at_benchmark_size():
    """The precision-form workload (N=2048, 1024 walkers) in FP32 and in FP64
    on identical seeds and walker ids, 40 + 60 sweeps with a sample every 5:
      * the FP32 local energy of every FP64 chain's final configuration
        (rounded to FP32) is within 1 mK/atom of its FP64 local energy (the
        form's target; measured ~0.01 mK/atom);
      * the chain energies per atom agree within 2 combined standard errors
        (the bar for chains), and within 4 walker-paired ones."""
    wl = configs.C3_N2048_FP32
    equil, measured = 40, 60
    res = {}
    for prec in (abi.FP64, abi.FP32):
        p = abi.params_for(wl, precision=prec)
        coords, acc = abi.alloc_state(p)
        rows = abi.alloc_rows(p)
        abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
        abi.sweep(p, coords, acc, 0, equil, abi.NO_MEASURE, 0, rows=rows)
        abi.sweep(p, coords, acc, equil, measured, equil, wl.m, rows=rows)
        torch.cuda.synchronize()
        a = abi.acc_to_numpy(acc)
        assert np.all(a["n_samples"] == measured // wl.m)
        res[prec] = ((a["sum_e"] + a["c_e"]) / a["n_samples"] / wl.n, coords)
    e64, e32 = res[abi.FP64][0], res[abi.FP32][0]
    W = wl.walkers
    se64, se32 = e64.std(ddof=1) / np.sqrt(W), e32.std(ddof=1) / np.sqrt(W)
    assert abs(e32.mean() - e64.mean()) <= 2 * np.hypot(se64, se32), (e32.mean(), e64.mean(), se64, se32)
    d = e32 - e64
    assert abs(d.mean()) <= 4 * d.std(ddof=1) / np.sqrt(W) + 1e-9
    x32 = res[abi.FP64][1].to(torch.float32)
    out64 = torch.zeros((W, 6), dtype=torch.float64, device="cuda")
    out32 = torch.zeros((W, 6), dtype=torch.float64, device="cuda")
    abi.local_energy(abi.params_for(wl, precision=abi.FP64), x32.to(torch.float64), out64)
    abi.local_energy(abi.params_for(wl, precision=abi.FP32), x32, out32)
    torch.cuda.synchronize()
    err_mk = (out32[:, 0] - out64[:, 0]).abs().cpu().numpy() / wl.n * KELVIN_TO_MK
    assert err_mk.max() <= 1.0, err_mk.max()
