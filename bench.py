"""Throughput of the VMC hot path on one MI355X.

Workload (default): liquid 4He, N=2048 atoms per walker (fcc 8x8x8 start),
density 0.02186 / A^3, b = 1.15 sigma, 512 walkers, FP64, Gaussian moves with
~50% acceptance, local energy every 5 sweeps.  One step = one launch of the
sweep kernel: 5 sweeps of every walker (N micro-updates each, the O(N) pair loop
per micro-update) followed by one O(N^2) local-energy evaluation per walker.
Warm-up steps (the same launches) double as equilibration; accumulators restart
with the first timed step.

Prints one JSON line: moves/s, the roofline of the sweep kernel (vector ALU,
FP64) from per-launch HIP events, the CPU oracle timed on the host cores on
a bounded sample of the same workload, and a bounded serving block (the
served p50/p99 time-to-1 mK/atom half of the metric, with censoring flagged
and the offered rate against the GPU's capacity for the request mix).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work: every micro-update forms the Eq. (7) sums over its N-1 pair
# terms.  A pair term is the nominal sequence of the method at the old and the
# new position of the moved atom (per position: 3 differences, minimum image
# (mul, round, fma) x 3, r^2, cutoff compare, r^-2 and r^-5, L - r, (L-r)^-5,
# u, x, repulsive argument and scale, x^-2 and x^-6, the C6/C8/C10 series,
# damping argument and select, V, cutoff selects: 43 operations of which 12
# are fused multiply-adds = 55 FLOP) plus 4 accumulating adds:
# 2 x 55 + 4 = 114 FLOP.  Square roots, reciprocals and exponentials count
# zero, and the local-energy samples are not counted at all, so the fraction
# of peak is a lower bound.  It is the same figure for every variant: the
# row-sum sweep reaches the same sums with fewer operations, so for it this is
# an effective rate.
FLOP_PER_PAIR_TERM = 114
PEAK = {"f64": 78.6, "f32": 157.3}   # MI355X vector TFLOP/s (published)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="he4_n2048_w512_fp64")
    ap.add_argument("--sweeps-per-step", type=int, default=5)
    ap.add_argument("--threads", type=int, default=0, help="threads per walker (0 = library choice)")
    ap.add_argument("--variant", type=int, default=0, help="sweep variant: 0 auto, 1 plain, 2 row sums")
    ap.add_argument("--n", type=int, default=0, help="override the workload's atoms per walker")
    ap.add_argument("--walkers", type=int, default=0, help="override the workload's walker count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-energy", action="store_true",
                    help="sweeps only: no local-energy samples in the timed launches (the pair loop alone)")
    ap.add_argument("--cpu-sweeps", type=int, default=70,
                    help="sweeps per walker of the CPU oracle sample (about 10 s on 16 host cores at N=2048)")
    ap.add_argument("--serve", type=int, default=0, metavar="REQUESTS",
                    help="instead of the sweep throughput, serve this many requests of the Poisson request "
                         "stream (20/s) until each reaches 1 mK/atom and report p50/p99 time-to-1mK")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-time-limit", type=float, default=None,
                    help="stop serving after this many seconds; unfinished requests are reported as censored")
    ap.add_argument("--serve-block-requests", type=int, default=40,
                    help="requests of the stream served in the throughput line's bounded serving block")
    ap.add_argument("--serve-block-seconds", type=float, default=90.0,
                    help="wall-time limit of the bounded serving block (0: no serving block)")
    ap.add_argument("--precision-check", action="store_true",
                    help="instead of the throughput line, the FP32 form against FP64 at N=2048 with 1024 walkers "
                         "on identical seeds: chain energies and per-configuration local-energy error in mK/atom")
    ap.add_argument("--serve-replicate", type=int, default=0, metavar="K",
                    help="serve with equilibrate-then-replicate: K seed walkers per request")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="instead of the workload, run 5 plain device copies of MIB MiB (the reference "
                         "kernel for scaling HBM byte counters) and exit")
    ap.add_argument("--c1", action="store_true",
                    help="instead of the throughput line, the single-walker run (N=108, 200 + 1000 sweeps, a local "
                         "energy every sweep) with its error from reblocking and from the autocorrelation time")
    ap.add_argument("--tsigma", action="store_true",
                    help="instead of the throughput line, t sigma^2 (time x squared standard error of E/N, "
                         "s mK^2; Sec. 7.3) of the GPU at N=512 and N=2048 and of the oracle at N=108 and N=2048")
    ap.add_argument("--replica-decorrelation", action="store_true",
                    help="instead of the throughput line, how fast replicas of equilibrated walkers decorrelate "
                         "(equilibrate-then-replicate), against independently equilibrated walkers")
    ap.add_argument("--b-scan", action="store_true",
                    help="instead of the throughput line, one run of the workload with per-sample records and "
                         "the correlated-sampling curve E(b') around its b, with one direct run to check it")
    return ap.parse_args()


def recorded_counters(workload):
    """Per-launch figures of the sweep kernel recorded in profiles/traffic.txt
    from rocprofv3 counters, if they were taken on the kernel sources as they
    are now: {"traffic": HBM bytes (calibrated FETCH_SIZE + WRITE_SIZE),
    "executed_flop": executed vector FLOPs (the SQ_INSTS_VALU_FLOPS_* counters
    x 64 lanes), or None where not recorded}; else None."""
    import glob
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1312_1282_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 3 and not line.startswith("#") and parts[0] == workload and parts[1] == digest:
                return {"traffic": int(parts[2]),
                        "executed_flop": int(parts[3]) if len(parts) > 3 else None}
    return None


def serve(args):
    """Served time-to-1 mK/atom for the first `args.serve` requests of the
    seeded request stream, arriving in real time."""
    import numpy as np
    import torch

    from paper_1312_1282_amd import serving

    torch.cuda.set_device(0)
    reqs = serving.request_stream(args.serve, rate=args.serve_rate)
    server = serving.Server(replicate=args.serve_replicate)
    t0 = time.perf_counter()
    server.run(reqs, realtime=True, time_limit=args.serve_time_limit,
               log=lambda m: print(m, file=sys.stderr, flush=True))
    wall = time.perf_counter() - t0
    lat = serving.latency_summary(reqs, server.censored_at)
    done = [r for r in reqs if r.done is not None]
    moves = sum(r.walkers * r.n * r.sweeps for r in done)
    busy_span = max(r.done for r in done) - min(r.admitted for r in done) if done else float("nan")
    line = {
        "metric": "single-particle Metropolis moves/s at N=2048; served p50/p99 time-to-1mK",
        "value": lat.get("p99_s"),
        "unit": "s (p99 time-to-1mK)",
        "higher_is_better": False,
        "n_gpus": 1,
        "dtype": "mixed f32/f64",
        "data": "synthetic: seeded Poisson stream of liquid 4He VMC requests",
        "config": {"workload": "he4_serving_stream", "requests": args.serve, "arrival_rate_per_s": args.serve_rate,
                   "target_se_K": server.target_se, "equil_sweeps": server.equil, "energy_every": server.m,
                   "check_every": server.check_every, "quantum_sweeps": server.quantum,
                   "replicate_seeds": server.replicate, "decorrelate_sweeps": server.decorrelate},
        "serving": {
            **lat,
            "offered_rate_per_s": args.serve_rate,
            "completed_per_s": len(done) / busy_span if done else 0.0,
            "moves_per_s": moves / busy_span if done else 0.0,
            "wall_s": wall,
            "launches": server.launches,
            "rejected": [r.rid for r in reqs if r.rejected],
            "requests": [{"rid": r.rid, "n": r.n, "walkers": r.walkers, "precision": r.precision,
                          "arrival_s": round(r.arrival, 4), "admitted_s": r.admitted, "done_s": r.done,
                          "sweeps": r.sweeps, "E_per_atom_K": r.energy, "se_K": r.se} for r in reqs],
        },
    }
    print(json.dumps(line), flush=True)


def serve_block(args):
    """The serving half of the metric, bounded in time: the first
    args.serve_block_requests requests of the seeded Poisson stream (20/s)
    arrive in real time and are served until each reaches SE <= 1 mK/atom or
    the wall-time limit passes.  Requests still running then are censored
    (their elapsed time is a lower bound, and so are the percentiles).  The
    offered rate is set against the capacity the GPU sustains for this
    request mix, estimated from the work each request needs (its sweeps to
    the target, extrapolated from its last stop-rule check when unfinished)."""
    import numpy as np

    from paper_1312_1282_amd import configs, serving

    reqs = serving.request_stream(args.serve_block_requests, rate=args.serve_rate)
    server = serving.Server()
    t0 = time.perf_counter()
    server.run(reqs, realtime=True, time_limit=args.serve_block_seconds)
    wall = time.perf_counter() - t0
    lat = serving.latency_summary(reqs, server.censored_at)
    cap, n_pred = serving.capacity_estimate(server, reqs, wall)
    done = [r for r in reqs if r.done is not None]
    return {
        "workload": "he4_serving_stream",
        "requests": len(reqs),
        "offered_rate_per_s": args.serve_rate,
        "wall_limit_s": args.serve_block_seconds,
        "wall_s": wall,
        **lat,
        "completed_per_s": len(done) / wall if wall > 0 else 0.0,
        "capacity_per_s": cap,
        "capacity_basis": f"pair terms per second while serving / mean predicted pair terms per request "
                          f"({n_pred} of {len(reqs)} requests had a prediction)",
        "highest_sustainable_rate_per_s": cap,
        "offered_over_capacity": (args.serve_rate / cap) if cap else None,
        "moves_per_s": server.moves / wall if wall > 0 else 0.0,
        "pair_terms_per_s": server.pair_terms / wall if wall > 0 else 0.0,
        "launches": server.launches,
        "target_se_K": server.target_se,
        "rejected": sum(1 for r in reqs if r.rejected),
        "requests_detail": [{"rid": r.rid, "n": r.n, "walkers": r.walkers, "precision": r.precision,
                             "arrival_s": round(r.arrival, 3),
                             "done_s": None if r.done is None else round(r.done, 3), "sweeps": r.sweeps,
                             "se_mK": None if r.se is None else round(r.se * 1e3, 3),
                             "predicted_sweeps": (None if serving.predicted_sweeps(server, r) is None
                                                  else int(serving.predicted_sweeps(server, r)))}
                            for r in reqs],
    }


def c1_run(args, equil=200, measured=1000):
    """The single-walker workload (N=108, seed 1, walker id 0): E/N with the
    standard error of one correlated chain, by Flyvbjerg-Petersen reblocking
    of its E_L samples and by Eq. (10) with the autocorrelation time m_c
    summed from R(k) (Sec. 4.1)."""
    import numpy as np
    import torch

    from paper_1312_1282_amd import abi, configs, observables

    torch.cuda.set_device(0)
    wl = configs.C1_SMALL_FP64
    p = abi.params_for(wl)
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    abi.sweep(p, coords, acc, 0, equil, abi.NO_MEASURE, 0, rows=rows)
    tr = torch.zeros((1, measured // wl.m, 6), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    abi.sweep(p, coords, acc, equil, measured, equil, wl.m, rows=rows, trace=tr)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e = tr[0, :, 0].cpu().numpy() / wl.n
    a = abi.acc_to_numpy(acc)
    se_blk, level = observables.blocking_se(e)
    R, mc = observables.autocorrelation(e, kmax=100)
    se_eq10 = float(e.std() / np.sqrt(len(e)) * np.sqrt(1.0 + 2.0 * mc))
    line = {
        "metric": "single-walker E/N with its correlated-chain error",
        "value": float(e.mean()),
        "unit": "K per atom",
        "n_gpus": 1,
        "dtype": "f64",
        "data": "synthetic: fcc-started liquid 4He walker",
        "config": {"workload": wl.name, "n_atoms": wl.n, "walkers": 1, "equil_sweeps": equil,
                   "measured_sweeps": measured, "energy_every": wl.m, "seed": wl.seed},
        "se_blocking_K": se_blk,
        "blocking_level": level,
        "blocking_levels": [[n_, se_, dse_] for n_, se_, dse_ in observables.blocking(e)],
        "se_naive_K": float(e.std() / np.sqrt(len(e))),
        "autocorrelation_time_samples": mc,
        "se_eq10_K": se_eq10,
        "acceptance": float(a["n_acc"][0] / a["n_try"][0]),
        "seconds": dt,
    }
    print(json.dumps(line), flush=True)


def gpu_tsigma(n, walkers, equil, measured, m=5):
    """t sigma^2 of the GPU path: W walkers from the fcc start equilibrate
    for `equil` sweeps, then `measured` sweeps with a local energy every m
    sweeps; t is the GPU time of the measured sweeps (HIP events) and sigma
    the standard error of E/N over the walkers' means (independent chains,
    Eq. (10) with several chains)."""
    import numpy as np
    import torch

    from paper_1312_1282_amd import abi, configs

    wl = configs.C2_N2048_FP64.with_(name=f"he4_n{n}_w{walkers}_fp64", n=n, walkers=walkers, m=m)
    p = abi.params_for(wl)
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    abi.sweep(p, coords, acc, 0, equil, abi.NO_MEASURE, 0, rows=rows)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(0, measured, 50):
        abi.sweep(p, coords, acc, equil + k, min(50, measured - k), equil, m, stream=stream, rows=rows)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    a = abi.acc_to_numpy(acc)
    ew = (a["sum_e"] + a["c_e"]) / a["n_samples"] / n
    se = float(ew.std(ddof=1) / np.sqrt(len(ew)))
    return {"n": n, "walkers": walkers, "equil_sweeps": equil, "measured_sweeps": measured, "energy_every": m,
            "E_per_atom_K": float(ew.mean()), "se_mK": se * 1e3, "seconds": t, "tsigma2_s_mK2": t * (se * 1e3) ** 2}


def cpu_baseline_tsigma(n, walkers, equil, measured, m=5):
    """The oracle's t sigma^2 on the host cores (the CPU baseline of the
    same figure): one walker per thread from the fcc start, `equil` sweeps,
    then `measured` sweeps with a local energy every m; t is the wall time of
    the measured sweeps, sigma the standard error of E/N over the walkers."""
    import numpy as np

    import oracle as O
    from paper_1312_1282_amd import configs

    s_ = O.system(n, O.box_side(n, configs.RHO_EQ), configs.C2_N2048_FP64.b, hbar2_over_m=configs.HBAR2_OVER_M,
                  step_sigma=configs.C2_N2048_FP64.step_sigma, seed=1)
    xyz = np.stack([O.fcc_start(s_, w) for w in range(walkers)])
    accs = (O.Walker * walkers)(*[O.walker_init(s_, xyz[w]) for w in range(walkers)])
    O.run_walkers(s_, 0, xyz, accs, 0, equil, 0xFFFFFFFF, 0, walkers)
    t0 = time.perf_counter()
    O.run_walkers(s_, 0, xyz, accs, equil, measured, equil, m, walkers)
    t = time.perf_counter() - t0
    ew = np.array([(a.sum_e + a.c_e) / a.n_samples / n for a in accs])
    se = float(ew.std(ddof=1) / np.sqrt(len(ew)))
    return {"n": n, "walkers": walkers, "threads": walkers, "equil_sweeps": equil, "measured_sweeps": measured,
            "energy_every": m, "E_per_atom_K": float(ew.mean()), "se_mK": se * 1e3, "seconds": t,
            "tsigma2_s_mK2": t * (se * 1e3) ** 2}


def tsigma(args):
    """t sigma^2 (Sec. 7.3: time to a given error times that error squared,
    invariant in the run length) of the GPU path at N=512 (the paper's K20
    figure is 130 s mK^2 there) and N=2048, and of the oracle on the host
    cores at N=108 and N=2048."""
    import torch

    torch.cuda.set_device(0)
    cores = min(os.cpu_count() or 1, 16)
    out = {
        "metric": "t sigma^2 of E/N (time x squared standard error)",
        "unit": "s mK^2",
        "n_gpus": 1,
        "dtype": "f64",
        "data": "synthetic: fcc-started liquid 4He walkers at 0.02186 / A^3, b = 1.15 sigma",
        "gpu": [gpu_tsigma(512, 2048, 600, 2000), gpu_tsigma(2048, 512, 400, 1000)],
        "cpu_baseline": [cpu_baseline_tsigma(108, cores, 400, 2000), cpu_baseline_tsigma(2048, cores, 200, 100)],
        "cores": cores,
    }
    out["value"] = out["gpu"][0]["tsigma2_s_mK2"]
    print(json.dumps(out), flush=True)


def _corr_by_lag(a, b):
    """Correlation coefficient over pairs of a[:, t] and b[:, t], for each t."""
    import numpy as np

    a = a - a.mean(axis=0)
    b = b - b.mean(axis=0)
    return (a * b).sum(axis=0) / np.sqrt((a * a).sum(axis=0) * (b * b).sum(axis=0))


def _iat(x, cut=6.0):
    """Integrated autocorrelation time (in samples) of series x[w, t], averaged
    over w, summing the autocorrelation until the window reaches cut times it
    (Sokal's automatic window)."""
    import numpy as np

    x = x - x.mean(axis=1, keepdims=True)
    var = (x * x).mean()
    tau = 0.5
    for k in range(1, x.shape[1] // 2):
        tau += (x[:, :-k] * x[:, k:]).mean() / var
        if k >= cut * tau:
            break
    return float(tau)


def replica_decorrelation(args, n=256, seeds=64, copies=8, equil=400, sweeps=300):
    """Equilibrate-then-replicate (Sec. 4.4): `seeds` walkers equilibrate
    for `equil` sweeps; each is copied to `copies` walkers, which restart
    their running totals from the copy and move on with their own random
    numbers, a local-energy sample every sweep.  rho(t) is the correlation of
    E_L between two copies of the same seed t sweeps after the copy (1 at
    t = 0), against the same statistic for walkers equilibrated
    independently (pairs of different seeds), and beside the integrated
    autocorrelation time of E_L along one chain."""
    import numpy as np
    import torch

    from paper_1312_1282_amd import abi, configs

    torch.cuda.set_device(0)
    wl = configs.C1_SMALL_FP64.with_(name="he4_replicas", n=n, walkers=seeds * copies, m=1)
    W = wl.walkers
    p_seed = abi.params_for(wl, n_walkers=seeds)
    p_all = abi.params_for(wl)
    coords, acc = abi.alloc_state(p_all)
    rows = abi.alloc_rows(p_all)
    abi.init_walkers(p_seed, coords[:seeds], acc[:seeds], fcc_start=True, rows=rows[:seeds])
    abi.sweep(p_seed, coords[:seeds], acc[:seeds], 0, equil, abi.NO_MEASURE, 0, rows=rows[:seeds])
    # walker j (j >= seeds) takes seed j mod seeds; its Philox walker id is j
    src = torch.arange(seeds, W, device="cuda") % seeds
    coords[seeds:] = coords[src]
    rows[seeds:] = rows[src]
    abi.init_walkers(p_all, coords, acc, fcc_start=False, rows=rows)
    tr = torch.zeros((W, sweeps, 6), dtype=torch.float64, device="cuda")
    abi.sweep(p_all, coords, acc, equil, sweeps, equil, 1, rows=rows, trace=tr)
    torch.cuda.synchronize()
    e = tr[:, :, 0].cpu().numpy() / n            # E_L per atom, [walker, sample]
    fam = np.arange(W) % seeds                    # seed of each walker
    # pairs of copies of one seed: (seed + a*seeds, seed + b*seeds), a < b
    pa, pb = [], []
    for a in range(copies):
        for b in range(a + 1, copies):
            pa.append(np.arange(seeds) + a * seeds)
            pb.append(np.arange(seeds) + b * seeds)
    pa, pb = np.concatenate(pa), np.concatenate(pb)
    assert np.all(fam[pa] == fam[pb])
    rho = _corr_by_lag(e[pa], e[pb])
    # independent pairs: copies of different seeds
    qa = np.arange(seeds)
    qb = (np.arange(seeds) + 1) % seeds + seeds
    rho_ind = _corr_by_lag(e[qa], e[qb])
    below = np.nonzero(rho < np.exp(-1.0))[0]
    t_e = int(below[0]) + 1 if len(below) else None
    noise = float(np.std(rho_ind))
    below2 = np.nonzero(rho < 2.0 * noise)[0]
    t_noise = int(below2[0]) + 1 if len(below2) else None
    # integrated autocorrelation time of E_L along the chains (second half)
    iat = _iat(e[:, sweeps // 2:])
    line = {
        "metric": "replica decorrelation (equilibrate-then-replicate)",
        "value": t_e,
        "unit": "sweeps after the copy until the E_L correlation of two copies falls below 1/e",
        "n_gpus": 1,
        "dtype": "f64",
        "data": "synthetic: fcc-started liquid 4He walkers",
        "config": {"workload": wl.name, "n_atoms": n, "seeds": seeds, "copies": copies, "equil_sweeps": equil,
                   "traced_sweeps": sweeps, "density_per_A3": wl.density, "b_A": wl.b},
        "rho_by_sweep": [round(float(x), 4) for x in rho[:60]],
        "rho_independent_rms": noise,
        "sweeps_to_noise_level": t_noise,
        "el_integrated_autocorrelation_sweeps": iat,
        "samples_independent_pairs": int(len(qa)),
        "samples_copy_pairs": int(len(pa)),
    }
    print(json.dumps(line), flush=True)


def b_scan(args, equil=200, measured=2000, factors=(0.97, 0.98, 0.99, 1.0, 1.01, 1.02, 1.03), check=1.02):
    """E(b') per atom from one run at b (per-sample records + reweighting),
    and a direct run at b' = check * b for comparison.  The reweighting factor
    exp(2 (U_b' - U_b)) fluctuates like an extensive quantity, so one run
    covers a range of b' that narrows as N grows: the scan runs N=108 with
    1024 walkers (--n, --walkers override), where a few percent in b keeps an
    effective sample size in the thousands."""
    import numpy as np
    import torch

    from paper_1312_1282_amd import abi, configs, observables

    torch.cuda.set_device(0)
    wl = configs.C1_SMALL_FP64.with_(name="he4_b_scan", n=args.n or 108, walkers=args.walkers or 1024, m=5)
    m = wl.m

    def run(b, trace):
        p = abi.params_for(wl, b=b)
        coords, acc = abi.alloc_state(p)
        rows = abi.alloc_rows(p)
        abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
        abi.sweep(p, coords, acc, 0, equil, abi.NO_MEASURE, 0, rows=rows)
        cap = measured // m
        tr = torch.zeros((wl.walkers, cap, 6), dtype=torch.float64, device="cuda") if trace else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(0, measured, 25):
            abi.sweep(p, coords, acc, equil + k, 25, equil, m, rows=rows, trace=tr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        a = abi.acc_to_numpy(acc)
        e_w = (a["sum_e"] + a["c_e"]) / a["n_samples"] / wl.n
        return (None if tr is None else tr.cpu().numpy()), e_w, wl.walkers * wl.n * measured / dt

    rec, e_w, rate_trace = run(wl.b, True)
    curve = observables.reweight_b(rec, wl.b, [f * wl.b for f in factors], wl.n)
    # per-walker spread of each estimate (walkers are independent chains)
    for c in curve:
        per = [observables.reweight_b(rec[w:w + 1], wl.b, [c["b"]], wl.n)[0]["E_per_atom"]
               for w in range(wl.walkers)]
        c["se_walkers"] = float(np.std(per, ddof=1) / np.sqrt(wl.walkers))
    _, e_direct, rate_plain = run(check * wl.b, False)
    rw = [c for c in curve if abs(c["b"] - check * wl.b) < 1e-12][0]
    line = {
        "metric": "correlated-sampling E(b') per atom from one run",
        "value": rw["E_per_atom"],
        "unit": "K per atom at b' = %.3f b" % check,
        "n_gpus": 1,
        "dtype": "f64" if wl.precision == configs.FP64 else "f32",
        "data": "synthetic: fcc-started liquid 4He walkers",
        "config": {"workload": wl.name, "b_A": wl.b, "equil_sweeps": equil, "measured_sweeps": measured,
                   "energy_every": m, "samples": int(rec.shape[0] * rec.shape[1])},
        "curve": curve,
        "direct_check": {"b_A": check * wl.b, "E_per_atom": float(e_direct.mean()),
                         "se": float(e_direct.std(ddof=1) / np.sqrt(len(e_direct))),
                         "reweighted_minus_direct": rw["E_per_atom"] - float(e_direct.mean())},
        "moves_per_s_with_trace": rate_trace,
        "moves_per_s_without_trace": rate_plain,
    }
    print(json.dumps(line), flush=True)


def precision_check(args, equil=100, measured=400):
    """The precision form against FP64 on the same seeds and walker ids (the
    N=2048, 1024-walker FP32 workload): (1) the two chains' energies per atom,
    walker-paired; (2) the FP32 local energy of each FP64 chain's final
    configuration (rounded to FP32) against its FP64 local energy, in mK/atom:
    the form's own error, free of sampling noise."""
    import numpy as np
    import torch

    from paper_1312_1282_amd import abi, configs

    torch.cuda.set_device(0)
    wl = configs.C3_N2048_FP32
    out = {}
    for prec in (configs.FP64, configs.FP32):
        p = abi.params_for(wl, precision=prec)
        coords, acc = abi.alloc_state(p)
        rows = abi.alloc_rows(p)
        abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
        abi.sweep(p, coords, acc, 0, equil, abi.NO_MEASURE, 0, rows=rows)
        for k in range(0, measured, 50):
            abi.sweep(p, coords, acc, equil + k, 50, equil, wl.m, rows=rows)
        torch.cuda.synchronize()
        a = abi.acc_to_numpy(acc)
        out[prec] = ((a["sum_e"] + a["c_e"]) / a["n_samples"] / wl.n, coords)
    d = out[configs.FP32][0] - out[configs.FP64][0]
    # per-configuration error on the FP64 chains' final configurations
    x64 = out[configs.FP64][1]
    x32 = x64.to(torch.float32)
    p64 = abi.params_for(wl, precision=configs.FP64)
    p32 = abi.params_for(wl, precision=configs.FP32)
    e64 = torch.zeros((wl.walkers, 6), dtype=torch.float64, device="cuda")
    e32 = torch.zeros((wl.walkers, 6), dtype=torch.float64, device="cuda")
    abi.local_energy(p64, x32.to(torch.float64), e64)   # FP64 terms of the FP32-rounded configuration
    abi.local_energy(p32, x32, e32)
    torch.cuda.synchronize()
    err = (e32[:, 0] - e64[:, 0]).cpu().numpy() / wl.n * 1e3
    line = {
        "metric": "FP32 form against FP64 on identical seeds",
        "value": float(np.abs(err).max()),
        "unit": "mK/atom (largest per-configuration local-energy error)",
        "n_gpus": 1,
        "dtype": "f32 pair terms, f64 sums",
        "data": "synthetic: fcc-started liquid 4He walkers",
        "config": {"workload": wl.name, "equil_sweeps": equil, "measured_sweeps": measured, "energy_every": wl.m},
        "chain_difference_mK": float(d.mean() * 1e3),
        "chain_difference_se_mK": float(d.std(ddof=1) / np.sqrt(len(d)) * 1e3),
        "config_error_mK": {"mean": float(err.mean()), "rms": float(np.sqrt((err ** 2).mean())),
                            "max_abs": float(np.abs(err).max())},
    }
    print(json.dumps(line), flush=True)


def calibrate_copy(mib):
    """Plain device-to-device copies of a known size: FETCH_SIZE and WRITE_SIZE
    of these dispatches are what the counters read for mib MiB each way."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_mib": mib, "bytes_each_way": n * 8}), flush=True)


def cpu_baseline(wl, sweeps):
    """The oracle as it stands, one walker per host thread, `sweeps` sweeps of
    each with a local-energy sample every m sweeps (the step's work mix), from
    the fcc start."""
    import numpy as np

    import oracle as O
    from paper_1312_1282_amd import configs

    cores = min(os.cpu_count() or 1, 16)
    W = cores
    s_ = O.system(wl.n, O.box_side(wl.n, wl.density, wl.precision == configs.FP32), wl.b,
                  hbar2_over_m=configs.HBAR2_OVER_M, step_sigma=wl.step_sigma, seed=wl.seed)
    xyz = np.stack([O.fcc_start(s_, w) for w in range(W)])
    accs = (O.Walker * W)(*[O.walker_init(s_, xyz[w]) for w in range(W)])
    t0 = time.perf_counter()
    m = wl.m if wl.m > 0 else sweeps
    O.run_walkers(s_, 0, xyz, accs, 0, sweeps, 0, m, cores)
    dt = time.perf_counter() - t0
    moves = W * wl.n * sweeps
    # the paper's convention (one core): one walker, a few sweeps, one thread
    x1 = O.fcc_start(s_, 0)
    a1 = O.walker_init(s_, x1)
    s1 = max(1, sweeps // 10)
    t1 = time.perf_counter()
    O.run_walker(s_, 0, x1, a1, 0, s1, 0, m)
    dt1 = time.perf_counter() - t1
    return {
        "value": moves / dt,
        "unit": "moves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{W} walkers x {sweeps} sweeps of N={wl.n} with a local energy every {m} sweeps, "
                  f"one walker per thread, {dt:.1f} s wall",
        "pair_terms_per_s": moves * (wl.n - 1) / dt,
        "single_core_moves_per_s": wl.n * s1 / dt1,
        "single_core_pair_terms_per_s": wl.n * s1 * (wl.n - 1) / dt1,
        "single_core_sample": f"1 walker x {s1} sweeps, one thread, {dt1:.1f} s",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(walkers are independent chains: G GPUs would each run W/G walkers of the same kernel).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1312_1282_amd import abi, configs

    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.serve:
        serve(args)
        return
    if args.b_scan:
        b_scan(args)
        return
    if args.replica_decorrelation:
        replica_decorrelation(args)
        return
    if args.tsigma:
        tsigma(args)
        return
    if args.c1:
        c1_run(args)
        return
    if args.precision_check:
        precision_check(args)
        return
    wl = configs.ALL[args.workload]
    if args.n or args.walkers:
        wl = wl.with_(name=f"{wl.name}_n{args.n or wl.n}_w{args.walkers or wl.walkers}",
                      n=args.n or wl.n, walkers=args.walkers or wl.walkers)
    p = abi.params_for(wl, threads=args.threads, variant=args.variant)
    dtype = "f32" if wl.precision == configs.FP32 else "f64"
    torch.cuda.set_device(0)
    coords, acc = abi.alloc_state(p)
    rows = abi.alloc_rows(p)
    abi.init_walkers(p, coords, acc, fcc_start=True, rows=rows)
    S = args.sweeps_per_step
    m = 0 if args.no_energy else wl.m
    t = 0
    # warm-up launches are the same work as timed ones (equilibration with
    # local energies); the accumulators are then restarted from the current
    # configurations, so every launch of the sweep kernel costs the same
    for _ in range(args.warmup):
        abi.sweep(p, coords, acc, t, S, 0, m, rows=rows)
        t += S
    abi.init_walkers(p, coords, acc, fcc_start=False, rows=rows)
    torch.cuda.synchronize()
    mstart = t
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        abi.sweep(p, coords, acc, t, S, mstart, m, stream=stream, rows=rows)
        ev[k][1].record(stream)
        t += S
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    launch_ms = np.array([a.elapsed_time(b) for a, b in ev])

    a = abi.acc_to_numpy(acc)
    moves_per_step = wl.walkers * wl.n * S
    value = moves_per_step * args.steps / wall
    acc_rate = float(a["n_acc"].sum() / max(a["n_try"].sum(), 1))
    plan = abi.plan_launch(p)
    rows_variant = plan["variant"] == abi.VARIANT_ROWS
    pair_terms_launch = moves_per_step * (wl.n - 1)
    flop_launch = pair_terms_launch * FLOP_PER_PAIR_TERM
    avg_s = float(launch_ms.mean()) * 1e-3
    achieved = flop_launch / avg_s / 1e12

    rec = recorded_counters(wl.name) or {"traffic": None, "executed_flop": None}
    executed = rec["executed_flop"] / avg_s / 1e12 if rec["executed_flop"] else None
    spread = plan["slices"] > 1

    a = abi.acc_to_numpy(acc)
    ns = np.maximum(a["n_samples"], 1)
    e_w = (a["sum_e"] + a["c_e"]) / ns / wl.n
    physics = {
        "E_per_atom_K": float(e_w.mean()) if m > 0 else None,
        "E_se_K": float(e_w.std(ddof=1) / np.sqrt(len(e_w))) if len(e_w) > 1 and m > 0 else None,
        "acceptance": acc_rate,
        "samples_per_walker": int(a["n_samples"][0]),
    }

    line = {
        "metric": "single-particle Metropolis moves/s at N=2048; served p50/p99 time-to-1mK",
        "value": value,
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic: fcc-started liquid 4He walkers, equilibrated during warm-up",
        "config": {
            "workload": wl.name,
            "n_atoms": wl.n,
            "walkers": wl.walkers,
            "density_per_A3": wl.density,
            "b_A": wl.b,
            "step_sigma_A": wl.step_sigma,
            "sweeps_per_step": S,
            "energy_every": m,
            "threads_per_walker": plan["threads"],
            "variant": "rows" if rows_variant else "plain",
            "spatial_order": bool(plan["spatial_order"]),
            "walkers_per_cu": plan["walkers_per_cu"],
            "workgroups_per_walker": plan["slices"],
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK[dtype],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK[dtype],
            "basis": ("nominal: 114 FLOP per pair term of Eq. (7) (old and new position of the moved atom); "
                      "the row-sum variant forms fewer, so for it this is an effective rate"),
            "executed": executed,
            "executed_frac": executed / PEAK[dtype] if executed else None,
            "executed_basis": "vector FLOPs the hardware counted (SQ_INSTS_VALU_FLOPS_*), recorded per launch",
            "traffic": rec["traffic"],
            "traffic_unit": "bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
            "kernel": "k_sweep_coop (cooperative, several workgroups per walker)" if spread else "k_sweep",
            "launch_ms_avg": float(launch_ms.mean()),
            "launch_ms_median": float(np.median(launch_ms)),
            "launch_ms_min_max": [float(launch_ms.min()), float(launch_ms.max())],
            "flop_per_launch": flop_launch,
            "flop_per_pair_term": FLOP_PER_PAIR_TERM,
            "pair_terms_per_launch": pair_terms_launch,
        },
        "physics": physics,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(wl, args.cpu_sweeps)
        cb["gpu_over_cpu"] = value / cb["value"]
        cb["gpu_over_single_core"] = value / cb["single_core_moves_per_s"]
        line["cpu_baseline"] = cb
    if args.serve_block_seconds > 0 and args.serve_block_requests > 0:
        line["serving"] = serve_block(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
