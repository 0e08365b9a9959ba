"""Host-side logic of the continuous-batching server (no GPU): slot free list,
launch quanta and check cadence, the stop rule, latency percentiles with
censored and failed requests, and the request-stream recipe."""
import numpy as np
import pytest

from paper_1312_1282_amd import abi, configs, serving


def test_slot_list_first_fit_and_coalescing():
    sl = serving.SlotList(100)
    assert sl.alloc(40) == 0 and sl.alloc(30) == 40 and sl.alloc(30) == 70
    assert sl.alloc(1) is None and sl.free == []
    sl.release(40, 30)
    assert sl.alloc(31) is None
    sl.release(0, 40)
    assert sl.free == [(0, 70)]
    assert sl.alloc(10) == 0
    sl.release(70, 30)
    assert sl.free == [(10, 90)]
    sl.release(0, 10)
    assert sl.free == [(0, 100)]


def test_slot_list_random_workload_never_overlaps():
    rng = np.random.default_rng(3)
    sl = serving.SlotList(1000)
    held = {}
    for step in range(3000):
        if held and rng.random() < 0.5:
            a = list(held)[rng.integers(len(held))]
            sl.release(a, held.pop(a))
        else:
            w = int(rng.integers(1, 120))
            a = sl.alloc(w)
            if a is not None:
                held[a] = w
        used = np.zeros(1000, dtype=int)
        for a, w in held.items():
            used[a:a + w] += 1
        for a, w in sl.free:
            used[a:a + w] += 1
        assert np.all(used == 1), step     # every slot is held or free, exactly once
        assert all(sl.free[k][0] + sl.free[k][1] < sl.free[k + 1][0] for k in range(len(sl.free) - 1))


@pytest.mark.parametrize("equil", [200, 20, 60, 7])
def test_quantum_divides_equilibration_and_cadence_is_a_multiple(equil):
    srv = serving.Server(equil=equil, check_every=50)
    for n in configs.SERVE_N + (10976,):
        q, c = srv.quantum_for(n), srv.cadence(n)
        assert q >= 1 and equil % q == 0
        assert c % q == 0 and c >= srv.check_every
    assert serving.Server().quantum_for(108) == 100 and serving.Server().cadence(108) == 100
    assert serving.Server().quantum_for(2048) == 10 and serving.Server().cadence(2048) == 50
    assert serving.Server(quantum=5).quantum_for(2048) == 5


def _acc(e_per_walker, n, samples):
    a = np.zeros(len(e_per_walker), dtype=abi.ACC_DTYPE)
    a["n_samples"] = samples
    a["sum_e"] = np.asarray(e_per_walker) * n * samples
    return a


def test_stop_rule_standard_error_and_min_samples():
    n = 108
    rng = np.random.default_rng(0)
    e = -5.0 + 0.01 * rng.standard_normal(200)
    req = serving.Request(rid=0, arrival=0.0, n=n, walkers=200, precision=0, density=0.02186, b=2.94, seed=1)
    srv = serving.Server(target_se=1e-3, min_samples=20)
    se, mean, ok = srv._check(req, _acc(e, n, 25))
    assert se == pytest.approx(e.std(ddof=1) / np.sqrt(200), rel=1e-12)
    assert mean == pytest.approx(e.mean(), rel=1e-12)
    assert ok == (se <= 1e-3)
    assert not srv._check(req, _acc(e, n, 19))[2]          # too few samples per walker
    assert not srv._check(req, _acc(-5.0 + 0.1 * rng.standard_normal(200), n, 25))[2]   # SE ~ 7 mK


def test_latency_summary_with_censored_failed_and_rejected():
    R = lambda rid, arr, done=None, rej=None, fail=None: serving.Request(
        rid=rid, arrival=arr, n=108, walkers=64, precision=0, density=0.02186, b=2.94, seed=rid,
        done=done, rejected=rej, failed=fail)
    reqs = [R(0, 0.0, 1.0), R(1, 0.5, 3.5), R(2, 1.0, None), R(3, 2.0, None, rej="ENOFIT"),
            R(4, 2.0, 2.5, fail="non-finite")]
    s = serving.latency_summary(reqs, censored_at=10.0)
    assert s["completed"] == 2 and s["censored"] == 1 and s["failed"] == 1
    assert s["percentiles_are_lower_bounds"]
    assert s["p50_s"] == pytest.approx(3.0) and s["max_s"] == pytest.approx(9.0)
    s2 = serving.latency_summary(reqs[:2])
    assert s2["completed"] == 2 and s2["censored"] == 0 and not s2["percentiles_are_lower_bounds"]
    assert s2["p99_s"] == pytest.approx(1.0 + 0.99 * 2.0)


def test_request_stream_recipe():
    reqs = serving.request_stream(200)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / configs.SERVE_RATE) < 0.2 / configs.SERVE_RATE
    assert {r.n for r in reqs} == set(configs.SERVE_N)
    assert all(64 <= r.walkers <= 512 for r in reqs)
    assert all(configs.SERVE_RHO[0] <= r.density <= configs.SERVE_RHO[1] for r in reqs)
    assert all(configs.SERVE_B[0] <= r.b <= configs.SERVE_B[1] for r in reqs)
    assert {r.precision for r in reqs} == {abi.FP64, abi.FP32}
    assert [r.seed for r in reqs] == list(range(1000, 1200))
    assert serving.request_stream(5)[3].arrival == serving.request_stream(5)[3].arrival


def test_class_threads_depend_on_n_only():
    srv = serving.Server()
    assert [srv.threads_for(n) for n in configs.SERVE_N] == [128, 256, 256, 256, 0, 0]
    assert serving.Server(latency_threads=False).threads_for(108) == 0
    r = serving.Request(rid=0, arrival=0.0, n=500, walkers=64, precision=0, density=0.02, b=2.9, seed=3)
    assert srv.params(r).threads == 256 and srv.params(r).n_walkers == 64


def test_replication_phases():
    srv = serving.Server(equil=200, replicate=16, decorrelate=50)
    assert srv.measure_start() == 250
    for n in configs.SERVE_N:
        q = srv.quantum_for(n)
        assert 200 % q == 0 and 250 % q == 0
    assert srv.quantum_for(108) == 50
    r = serving.Request(rid=0, arrival=0.0, n=108, walkers=100, precision=0, density=0.02, b=2.9, seed=3)
    assert srv.seeds(r) == 16
    r.replicated = True
    assert srv.seeds(r) == 100
    small = serving.Request(rid=1, arrival=0.0, n=108, walkers=10, precision=0, density=0.02, b=2.9, seed=4)
    assert srv.seeds(small) == 10
    off = serving.Server(equil=200)
    assert off.measure_start() == 200 and off.seeds(small) == 10 and off.quantum_for(108) == 100
