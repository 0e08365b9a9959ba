"""Continuous-batching server of VMC requests on one GPU.

A request asks for the energy per atom of liquid 4He at its own (N, density,
b, precision) with W walkers, run until the standard error of E/N over its
walkers is at most a target (1 mK/atom).  Requests arrive over time; the server
admits them while their footprint fits, packs the walkers of requests that
share N and precision into one device-resident slot pool per class, and
advances every class in quanta of sweeps with one batched launch
(hevmc_sweep_batch) per class on the class's own stream, so the classes'
launches overlap on the GPU.  Between quanta a class retires finished requests,
frees their slots and admits waiting requests into them.

Each request is a set of independent walkers with request-local Philox walker
ids and the request's own seed, and its sweeps are split into quanta by its own
sweep counter: its result is the same whichever slots it lands in and whatever
else runs beside it (tested bit for bit).

Stop rule (a deterministic cadence, so results do not depend on scheduling):
after equil sweeps of equilibration, measure with a local-energy sample every m
sweeps; every check_every measured sweeps compute SE = sd_w(e_w)/sqrt(W) of the
walkers' mean energies per atom e_w, and stop when SE <= target and every
walker has at least min_samples samples (the W independent chains play the
role of the paper's independent Markov chains, Eq. (10) and the text after it).
"""
import math
import time
from dataclasses import dataclass

import numpy as np

from . import abi, configs

LDS_PER_CU = 160 * 1024
CUS = 256


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    n: int
    walkers: int
    precision: int
    density: float
    b: float
    seed: int
    # filled in by the server
    admitted: float = None
    done: float = None
    sweeps: int = 0
    se: float = None
    energy: float = None
    result: np.ndarray = None
    slot0: int = None
    replicated: bool = False
    # another class had a launch in flight when this request was admitted
    admitted_during_flight: bool = False
    rejected: str = None
    failed: str = None      # set when a walker's state turns non-finite

    def params(self, threads=0, variant=abi.VARIANT_AUTO):
        return abi.make_params(self.n, self.walkers, precision=self.precision, density=self.density, b=self.b,
                               step_sigma=configs.STEP_C * self.density ** (-1.0 / 3.0), seed=self.seed,
                               walker_id_base=0, threads=threads, variant=variant)


def request_stream(count, rate=configs.SERVE_RATE, seed=0, seed_base=1000):
    """The serving workload: Poisson arrivals at `rate` per second; N uniform
    over the serving sizes; walkers uniform in [64, 512]; precision FP32/FP64
    with equal odds; density U[0.019, 0.026]; b U[1.0, 1.3] sigma; request r
    gets seed seed_base + r."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(1.0 / rate)
        out.append(Request(
            rid=r, arrival=t,
            n=int(rng.choice(configs.SERVE_N)),
            walkers=int(rng.integers(configs.SERVE_W[0], configs.SERVE_W[1] + 1)),
            precision=int(rng.integers(0, 2)),
            density=float(rng.uniform(*configs.SERVE_RHO)),
            b=float(rng.uniform(*configs.SERVE_B)),
            seed=seed_base + r,
        ))
    return out


class SlotList:
    """First-fit free list of walker slots [0, capacity): a request takes one
    contiguous range, so its walkers sit next to each other in the pool."""

    def __init__(self, capacity):
        self.capacity = capacity
        self.free = [(0, capacity)]     # (start, length), sorted, coalesced

    def alloc(self, w):
        """Start of a free range of w slots, or None."""
        for k, (a, length) in enumerate(self.free):
            if length >= w:
                if length == w:
                    self.free.pop(k)
                else:
                    self.free[k] = (a + w, length - w)
                return a
        return None

    def release(self, a, w):
        self.free.append((a, w))
        self.free.sort()
        merged = []
        for s, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((s, l))
        self.free = merged


class _Pool:
    """Device-resident walker slots of one (N, precision) class."""

    def __init__(self, n, precision, capacity, torch, threads=0):
        self.n, self.precision, self.capacity, self.threads = n, precision, capacity, threads
        shape = abi.make_params(n, capacity, precision=precision, threads=threads)
        self.coords, self.acc = abi.alloc_state(shape)
        self.rows = abi.alloc_rows(shape)
        self.map_host = np.full((capacity, 2), -1, dtype=np.int32)
        self.map = torch.full((capacity, 2), -1, dtype=torch.int32, device="cuda")
        self.stream = torch.cuda.Stream()
        # the buffers were filled on the allocating stream: order the pool's
        # own stream after that, or a walker start could land before the fill
        self.stream.wait_stream(torch.cuda.current_stream())
        self.active = []            # requests in this class
        self.event = None           # completion of the launch in flight
        self.in_flight = []         # requests advanced by that launch
        self.slots = SlotList(capacity)


class Server:
    def __init__(self, target_se=configs.SERVE_TARGET_SE, equil=200, m=5, check_every=50, min_samples=20,
                 quantum=None, lds_oversubscription=4.0, max_requests_per_class=abi.MAX_BATCH,
                 slots_per_class=8192, latency_threads=True, replicate=0, decorrelate=50):
        self.target_se = target_se
        self.equil = equil
        self.m = m
        self.check_every = check_every
        self.min_samples = min_samples
        self.quantum = quantum
        self.latency_threads = latency_threads
        # equilibrate-then-replicate: with replicate = K > 0, a request first
        # equilibrates only K seed walkers for `equil` sweeps; then every
        # walker j takes a copy of seed j mod K and decorrelates, with its own
        # random numbers, for `decorrelate` sweeps before measuring
        self.replicate = replicate
        self.decorrelate = decorrelate if replicate else 0
        self.budget = lds_oversubscription * LDS_PER_CU * CUS
        self.max_per_class = max_requests_per_class
        self.slots_per_class = slots_per_class
        self.pools = {}
        self.used_budget = 0.0
        self.launches = 0
        self.moves = 0
        self.pair_terms = 0
        self.log = None
        self.censored_at = None

    # -- launch shape ------------------------------------------------------
    def threads_for(self, n):
        """Threads per walker of a class.  A request's walkers are few next to
        the chip's compute units, and its time to the target is the length of
        its chains: small walkers get more threads than the library's
        throughput-minded choice (one wave), which shortens every move
        (N=500 FP64: 3.6 us with 64 threads, 1.7 us with 256).  A function of
        N only, so a request runs the same launches alone and in any mix."""
        if not self.latency_threads:
            return 0
        return 128 if n <= 128 else 256 if n <= 1024 else 0

    def params(self, req):
        return req.params(threads=self.threads_for(req.n))

    # -- footprint ---------------------------------------------------------
    def footprint(self, req):
        p = self.params(req)
        if abi.plan_launch(p)["slices"] > 1:
            # a walker spread over several workgroups has no batched sweep
            raise abi.HevmcError(-3, f"walker of {req.n} atoms does not fit in one workgroup's LDS")
        lds, hbm = abi.footprint(p)
        return lds * req.walkers, hbm

    def _pool(self, req, torch):
        key = (req.n, req.precision)
        if key not in self.pools:
            lds, _ = abi.footprint(self.params(req))
            cap = int(min(self.slots_per_class, self.budget // max(lds, 1)))
            self.pools[key] = _Pool(req.n, req.precision, max(cap, 1), torch, threads=self.threads_for(req.n))
        return self.pools[key]

    # -- lifecycle ---------------------------------------------------------
    def _admit(self, req, now, torch):
        pool = self._pool(req, torch)
        if len(pool.active) >= self.max_per_class:
            return False
        lds_total, _ = self.footprint(req)
        if self.used_budget + lds_total > self.budget:
            return False
        a = pool.slots.alloc(req.walkers)
        if a is None:
            return False
        req.slot0 = a
        req.admitted = now
        req.admitted_during_flight = any(q.event is not None for q in self.pools.values() if q is not pool)
        req.sweeps = 0
        self.used_budget += lds_total
        p = self.params(req)
        with torch.cuda.stream(pool.stream):
            abi.init_walkers(p, pool.coords[a:a + req.walkers], pool.acc[a:a + req.walkers], fcc_start=True,
                             stream=pool.stream, rows=pool.rows[a:a + req.walkers])
        pool.active.append(req)
        pool.map_host[a:a + req.walkers, 1] = np.arange(req.walkers, dtype=np.int32)
        return True

    def _replicate(self, pool, req):
        """Copy the equilibrated seeds to the request's other walkers (walker j
        takes seed j mod K) and restart every walker's running totals and
        accumulators from its configuration; from here on each walker moves
        with its own random numbers."""
        import torch

        K, W, a = self.seeds(req), req.walkers, req.slot0
        with torch.cuda.stream(pool.stream):
            # the index vector is made on the pool's stream too: made on another
            # stream, the gather could read it before it is written
            src = torch.arange(K, W, device="cuda") % K + a
            pool.coords[a + K:a + W] = pool.coords[src]
            pool.rows[a + K:a + W] = pool.rows[src]
            abi.init_walkers(self.params(req), pool.coords[a:a + W], pool.acc[a:a + W], fcc_start=False,
                             stream=pool.stream, rows=pool.rows[a:a + W])
        req.replicated = True

    def _retire(self, pool, req, acc_np, now):
        req.done = now
        req.result = acc_np
        pool.active.remove(req)
        pool.slots.release(req.slot0, req.walkers)
        pool.map_host[req.slot0:req.slot0 + req.walkers] = -1
        self.used_budget -= self.footprint(req)[0]

    def _check(self, req, acc_np):
        """Stop rule at a check point: (SE, mean E/N, done?)."""
        ns = acc_np["n_samples"]
        e = (acc_np["sum_e"] + acc_np["c_e"]) / np.maximum(ns, 1) / req.n
        se = float(e.std(ddof=1) / np.sqrt(len(e))) if len(e) > 1 else float("inf")
        return se, float(e.mean()), bool(ns.min() >= self.min_samples and se <= self.target_se)

    def measure_start(self):
        """Sweep index from which every request measures."""
        return self.equil + self.decorrelate

    def seeds(self, req):
        """Walkers that run during equilibration."""
        if self.replicate and not req.replicated and req.walkers > self.replicate:
            return self.replicate
        return req.walkers

    def quantum_for(self, n):
        """Sweeps per launch of a class: about the same GPU time per launch for
        every N (a small walker's sweep is short).  A function of N only, so a
        request is split into the same launches alone and in any mix; the
        equilibration length and the first measured sweep are multiples of
        it."""
        if self.quantum:
            return self.quantum
        target = 100 if n <= 128 else 50 if n <= 300 else 25 if n <= 600 else 10
        g = math.gcd(self.equil, self.measure_start()) or target
        return max(d for d in range(1, min(target, g) + 1) if g % d == 0)

    def cadence(self, n):
        """Measured sweeps between stop-rule checks: check_every, or the
        quantum if that is longer (checks fall on launch boundaries)."""
        q = self.quantum_for(n)
        c = max(self.check_every, q)
        return c if c % q == 0 else q * ((c + q - 1) // q)

    def _launch(self, pool, torch):
        reqs = list(pool.active)
        if not reqs:
            pool.event = None
            pool.in_flight = []
            return
        arr = (abi.Request * len(reqs))()
        for k, r in enumerate(reqs):
            arr[k].params = self.params(r)
            arr[k].sweep0 = r.sweeps
            arr[k].measure_start = self.measure_start()
            arr[k].energy_every = self.m
            pool.map_host[r.slot0:r.slot0 + r.walkers, 0] = -1
            pool.map_host[r.slot0:r.slot0 + self.seeds(r), 0] = k
        with torch.cuda.stream(pool.stream):
            pool.map.copy_(torch.from_numpy(pool.map_host.copy()).pin_memory(), non_blocking=True)
            abi.sweep_batch(arr, pool.map, pool.coords, pool.acc, pool.rows, self.quantum_for(pool.n),
                            stream=pool.stream)
            ev = torch.cuda.Event()
            ev.record(pool.stream)
        pool.event = ev
        pool.in_flight = reqs
        self.launches += 1
        self.moves += sum(self.seeds(r) * r.n for r in reqs) * self.quantum_for(pool.n)
        self.pair_terms += sum(self.seeds(r) * r.n * (r.n - 1) for r in reqs) * self.quantum_for(pool.n)

    def _finish_quantum(self, pool, now):
        """The launch of pool is complete: advance counters, run stop checks."""
        due = []
        q, c = self.quantum_for(pool.n), self.cadence(pool.n)
        for r in pool.in_flight:
            r.sweeps += q
            if self.seeds(r) < r.walkers and r.sweeps >= self.equil:
                self._replicate(pool, r)
            meas = r.sweeps - self.measure_start()
            if meas > 0 and meas % c == 0:
                due.append(r)
        if due:
            acc_all = abi.acc_to_numpy(pool.acc)
            for r in due:
                acc_np = acc_all[r.slot0:r.slot0 + r.walkers].copy()
                bad = ~(np.isfinite(acc_np["u_run"]) & np.isfinite(acc_np["v_run"]) & np.isfinite(acc_np["sum_e"]))
                if bad.any():
                    r.failed = f"{int(bad.sum())} walker(s) with a non-finite running state"
                    self._retire(pool, r, acc_np, now)
                    if self.log:
                        self.log(f"fail  r{r.rid}: {r.failed}")
                    continue
                r.se, r.energy, ok = self._check(r, acc_np)
                r.checks = getattr(r, "checks", 0) + 1
                if self.log and not ok and r.checks % 20 == 0:
                    self.log(f"check r{r.rid} N={r.n} after {r.sweeps} sweeps: SE {r.se * 1e3:.3f} mK at {now:.2f}s")
                if ok:
                    self._retire(pool, r, acc_np, now)
                    if self.log:
                        self.log(f"done  r{r.rid} N={r.n} W={r.walkers} prec={r.precision} after {r.sweeps} sweeps, "
                                 f"E/N = {r.energy:.4f} +- {r.se * 1e3:.3f} mK at {now:.2f}s")
        pool.event = None
        pool.in_flight = []

    def run(self, requests, realtime=True, time_limit=None, log=None):
        """Serve the requests; returns them with admitted/done times filled in.
        realtime: requests become visible at their arrival times; otherwise all
        are visible at once (used to run a request 'alone')."""
        import torch

        self.log = log
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            try:
                lds_total, _ = self.footprint(r)
            except abi.HevmcError as e:
                r.rejected = str(e)
                continue
            if lds_total > self.budget:
                r.rejected = f"footprint {lds_total} B of LDS-time exceeds the budget {self.budget:.0f} B"
        pending = [r for r in pending if r.rejected is None]
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: float("inf"))
        while pending or any(p.active for p in self.pools.values()):
            now = clock()
            if time_limit is not None and time.perf_counter() - t0 > time_limit:
                self.censored_at = time.perf_counter() - t0
                break
            progressed = False
            # finished quanta
            for pool in list(self.pools.values()):
                if pool.event is not None and pool.event.query():
                    self._finish_quantum(pool, time.perf_counter() - t0)
                    progressed = True
            # admissions, in arrival order (head-of-line per class)
            still = []
            for r in pending:
                if r.arrival <= now and self._admit(r, time.perf_counter() - t0, torch):
                    progressed = True
                    if log:
                        log(f"admit r{r.rid} N={r.n} W={r.walkers} prec={r.precision} at {r.admitted:.2f}s")
                else:
                    still.append(r)
            pending = still
            # idle classes launch their next quantum
            for pool in self.pools.values():
                if pool.event is None and pool.active:
                    self._launch(pool, torch)
                    progressed = True
            if not progressed:
                time.sleep(0.0005)
        torch.cuda.synchronize()
        return requests


def predicted_sweeps(server, req):
    """Sweeps a request needs to reach the target: its own count if it is
    done; else, from its last stop-rule check, the measured sweeps scaled by
    (SE / target)^2 (the SE of a mean over samples falls as one over the
    square root of their number); None before its first check."""
    if req.done is not None:
        return req.sweeps
    if req.se is None or not np.isfinite(req.se):
        return None
    ms = server.measure_start()
    measured = req.sweeps - ms
    if measured <= 0:
        return None
    return ms + measured * max(1.0, (req.se / server.target_se) ** 2)


def capacity_estimate(server, requests, busy_s):
    """Requests per second the GPU sustains for this request mix: pair terms
    per second while serving over the mean pair terms a request needs (from
    predicted_sweeps, over the requests that have a prediction)."""
    work = []
    for r in requests:
        sw = predicted_sweeps(server, r)
        if sw is not None:
            work.append(r.walkers * r.n * (r.n - 1) * sw)
    if not work or busy_s <= 0 or server.pair_terms == 0:
        return None, len(work)
    rate = server.pair_terms / busy_s
    return rate / float(np.mean(work)), len(work)


def latency_summary(requests, censored_at=None):
    """p50/p99 of time-to-target (completion - arrival, seconds).  Requests
    still running when the run was stopped at censored_at count with their
    elapsed time censored_at - arrival, a lower bound, so the percentiles are
    lower bounds too when any request is censored."""
    served = [r for r in requests if r.rejected is None and r.failed is None]
    lat, cens = [], 0
    for r in served:
        if r.done is not None:
            lat.append(r.done - r.arrival)
        elif censored_at is not None:
            lat.append(censored_at - r.arrival)
            cens += 1
    failed = sum(1 for r in requests if r.failed is not None)
    if not lat:
        return {"completed": 0, "censored": cens, "failed": failed}
    lat = np.array(lat)
    return {
        "completed": len(served) - cens,
        "censored": cens,
        "failed": failed,
        "percentiles_are_lower_bounds": cens > 0,
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "max_s": float(lat.max()),
        "mean_s": float(lat.mean()),
    }
