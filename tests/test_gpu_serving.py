"""GPU tests of the batched sweep and the continuous-batching server: a
request's result is the same alone and in a mix, bit for bit."""
import numpy as np
import pytest

import oracle as O
from paper_1312_1282_amd import abi, configs, serving

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _req(rid, n, W, precision, density, b, seed):
    return serving.Request(rid=rid, arrival=0.0, n=n, walkers=W, precision=precision, density=density, b=b,
                           seed=seed)


def _acc_diff(a, b):
    """The accumulator fields that differ, with their largest relative difference."""
    out = []
    for f in abi.ACC_FIELDS + abi.ACC_INT_FIELDS:
        if not np.array_equal(a[f], b[f]):
            d = np.abs(a[f] - b[f]) / np.maximum(np.abs(a[f]), 1e-300)
            w = int(np.argmax(np.where(np.isnan(d), np.inf, d)))
            out.append(f"{f}: {d.max():.2e} at walker {w} ({a[f][w]!r} vs {b[f][w]!r})")
    return "; ".join(out)


@pytest.mark.parametrize("n,precision", [(256, abi.FP64), (256, abi.FP32), (1100, abi.FP64), (2048, abi.FP64),
                                         (2048, abi.FP32), (4000, abi.FP32)])
def test_batched_launch_equals_single_requests(n, precision):
    """Three requests with the same N and precision but their own density, b
    and seed share slot pools with gaps; after three launches of 7 sweeps each
    (the first equilibration only) every request equals its own hevmc_sweep run."""
    reqs = [_req(0, n, 5, precision, 0.0190, 2.6, 11), _req(1, n, 3, precision, 0.0220, 3.0, 12),
            _req(2, n, 4, precision, 0.0255, 3.3, 13)]
    slots, starts = 20, [1, 8, 14]
    shape = abi.make_params(n, slots, precision=precision)
    coords, acc = abi.alloc_state(shape)
    rows = abi.alloc_rows(shape)
    wmap = np.full((slots, 2), -1, np.int32)
    for k, (r, a) in enumerate(zip(reqs, starts)):
        p = r.params()
        abi.init_walkers(p, coords[a:a + r.walkers], acc[a:a + r.walkers], rows=rows[a:a + r.walkers])
        wmap[a:a + r.walkers, 0] = k
        wmap[a:a + r.walkers, 1] = np.arange(r.walkers)
    dmap = torch.from_numpy(wmap).cuda()
    t = 0
    for q in range(3):
        arr = (abi.Request * 3)()
        for k, r in enumerate(reqs):
            arr[k].params = r.params()
            arr[k].sweep0 = t
            arr[k].measure_start = 7
            arr[k].energy_every = 2
        abi.sweep_batch(arr, dmap, coords, acc, rows, 7)
        t += 7
    torch.cuda.synchronize()
    xb = coords.cpu().numpy()
    ab = abi.acc_to_numpy(acc)
    for r, a in zip(reqs, starts):
        p = r.params()
        c1, a1 = abi.alloc_state(p)
        r1 = abi.alloc_rows(p)
        abi.init_walkers(p, c1, a1, rows=r1)
        for q in range(3):
            abi.sweep(p, c1, a1, 7 * q, 7, 7, 2, rows=r1)
        torch.cuda.synchronize()
        assert np.array_equal(c1.cpu().numpy(), xb[a:a + r.walkers])
        a1 = abi.acc_to_numpy(a1)
        assert a1.tobytes() == ab[a:a + r.walkers].tobytes(), _acc_diff(a1, ab[a:a + r.walkers])
    # unused slots untouched
    assert np.all(ab["n_try"][[0, 6, 7, 11, 12, 13, 18, 19]] == 0)


def test_server_result_same_alone_and_in_mix():
    """Requests of two classes served together (sharing pools and launches)
    end with the same accumulators, bit for bit, and after the same number of
    sweeps as each served alone."""
    mk = lambda: [_req(0, 108, 64, abi.FP64, 0.0200, 2.8, 21), _req(1, 108, 96, abi.FP64, 0.0240, 3.1, 22),
                  _req(2, 256, 64, abi.FP32, 0.0219, 2.9, 23), _req(3, 108, 80, abi.FP32, 0.0210, 3.0, 24)]
    kw = dict(target_se=4e-3, equil=20, check_every=10, min_samples=2, quantum=5)
    assert serving.Server(quantum=None).quantum_for(108) == 100 and serving.Server(quantum=None).cadence(108) == 100
    mix = serving.Server(**kw).run(mk(), realtime=False)
    for r in mix:
        assert r.done is not None and r.rejected is None
    for k in range(4):
        alone = serving.Server(**kw).run([mk()[k]], realtime=False)[0]
        assert alone.sweeps == mix[k].sweeps
        assert alone.result.tobytes() == mix[k].result.tobytes()
        assert alone.se <= 4e-3


def test_server_rejects_walkers_that_do_not_fit():
    big = _req(0, 10976, 8, abi.FP64, 0.02186, 2.94, 1)    # FP64 walker of 263 KB: no workgroup can hold it
    small = _req(1, 108, 64, abi.FP64, 0.02186, 2.94, 2)
    out = serving.Server(target_se=5e-3, equil=10, check_every=10, min_samples=2, quantum=5).run(
        [big, small], realtime=False)
    assert out[0].rejected and "ENOFIT" in out[0].rejected
    assert out[1].done is not None


def test_replicated_server_alone_and_in_mix_and_energy():
    """Equilibrate-then-replicate: a request's result is the same bits alone
    and in a mix, and its energy agrees with the same request served without
    replication within their standard errors."""
    mk = lambda: [_req(0, 108, 200, abi.FP64, 0.0219, 2.94, 31), _req(1, 256, 96, abi.FP32, 0.0210, 3.0, 32)]
    kw = dict(target_se=3e-3, equil=40, check_every=20, min_samples=4, replicate=8, decorrelate=20)
    mix = serving.Server(**kw).run(mk(), realtime=False)
    for r in mix:
        assert r.done is not None and r.replicated
    alone = serving.Server(**kw).run([mk()[0]], realtime=False)[0]
    assert alone.sweeps == mix[0].sweeps and alone.result.tobytes() == mix[0].result.tobytes()
    plain = serving.Server(**{k: v for k, v in kw.items() if k not in ("replicate", "decorrelate")}).run(
        [mk()[0]], realtime=False)[0]
    assert not plain.replicated
    assert abs(alone.energy - plain.energy) < 4.0 * np.hypot(alone.se, plain.se), (alone.energy, plain.energy)



def test_freed_slots_and_admission_during_flight_keep_results():
    """Continuous batching proper: one request per class at a time, so later
    requests of a class wait for an earlier one to retire and take its freed
    slots, and the small class's requests are admitted while the large class
    has a launch in flight: the large request (N=2048 FP32, 256 walkers) comes
    first and its launches take about 10 ms each, and the first small one
    (N=108 FP64) arrives 2 ms after it.  Staggered real-time arrivals.  Every
    result equals the same request served alone, bit for bit."""
    mk = lambda: [_req(0, 2048, 256, abi.FP32, 0.0215, 3.0, 42), _req(1, 108, 64, abi.FP64, 0.0200, 2.8, 41),
                  _req(2, 108, 64, abi.FP64, 0.0230, 3.1, 43), _req(3, 2048, 192, abi.FP32, 0.0205, 2.9, 44),
                  _req(4, 108, 32, abi.FP64, 0.0219, 2.94, 45)]
    kw = dict(target_se=4e-3, equil=20, check_every=10, min_samples=2, quantum=5, max_requests_per_class=1,
              slots_per_class=256)
    reqs = mk()
    for k, r in enumerate(reqs):
        r.arrival = 0.002 * k
    mix = serving.Server(**kw).run(reqs, realtime=True)
    for r in mix:
        assert r.done is not None and r.rejected is None and r.failed is None, r.rid
    # later requests of a class reuse the slots of the one before them
    assert mix[2].slot0 == mix[1].slot0 and mix[2].admitted >= mix[1].done
    assert mix[4].slot0 == mix[2].slot0 and mix[4].admitted >= mix[2].done
    assert mix[3].slot0 == mix[0].slot0 and mix[3].admitted >= mix[0].done
    # request 1 arrives 2 ms after the large request 0 was admitted and
    # launched, into a launch of about 10 ms
    assert any(mix[k].admitted_during_flight for k in (1, 2, 4)), [(r.rid, r.admitted, r.done) for r in mix]
    for k in range(5):
        alone = serving.Server(**{**kw, "max_requests_per_class": 16, "slots_per_class": 8192}).run(
            [mk()[k]], realtime=False)[0]
        assert alone.sweeps == mix[k].sweeps, k
        assert alone.result.tobytes() == mix[k].result.tobytes(), (k, _acc_diff(alone.result, mix[k].result))


def test_replicated_request_follows_the_oracle():
    """Equilibrate-then-replicate through the oracle, in lockstep: the
    request's K seed walkers equilibrate alone (oracle: walker ids 0..K-1 from
    their fcc starts), every walker j then takes a copy of seed j mod K, its
    running totals and accumulators restart from that configuration, and it
    moves on with its own random numbers (walker id j) through the
    decorrelation and measured sweeps.  The server's final accumulators and
    configurations equal the oracle's replay of the same steps."""
    K, W, n = 4, 16, 108
    req = _req(0, n, W, abi.FP64, 0.0219, 2.94, 51)
    kw = dict(target_se=1.0, equil=20, check_every=10, min_samples=2, quantum=5, replicate=K, decorrelate=10)
    server = serving.Server(**kw)
    r = server.run([req], realtime=False)[0]
    assert r.done is not None and r.replicated
    pool = server.pools[(n, abi.FP64)]
    xg = pool.coords[r.slot0:r.slot0 + W].cpu().numpy()
    ag = r.result
    p = r.params()
    s_ = O.system(n, O.box_side(n, req.density), req.b, hbar2_over_m=configs.HBAR2_OVER_M,
                  step_sigma=p.step_sigma, seed=req.seed)
    seeds = []
    for w in range(K):
        x = O.fcc_start(s_, w)
        a = O.walker_init(s_, x)
        O.run_walker(s_, w, x, a, 0, server.equil, 0xFFFFFFFF, 0)
        seeds.append(x)
    ms = server.measure_start()
    for j in range(W):
        x = np.ascontiguousarray(seeds[j % K].copy())
        a = O.walker_init(s_, x)
        O.run_walker(s_, j, x, a, server.equil, r.sweeps - server.equil, ms, server.m)
        assert ag["n_acc"][j] == a.n_acc and ag["n_try"][j] == a.n_try, j
        assert ag["n_samples"][j] == a.n_samples == (r.sweeps - ms) // server.m, j
        assert np.max(np.abs(xg[j] - x)) < 1e-9, j
        assert ag["sum_e"][j] + ag["c_e"][j] == pytest.approx(a.sum_e + a.c_e, rel=1e-10), j
        assert ag["u_run"][j] == pytest.approx(a.u_run, rel=1e-10, abs=1e-9), j
