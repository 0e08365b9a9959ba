"""Find the Gaussian step size that gives ~50% acceptance, using only the oracle.

The paper uses an rms displacement of 0.5 rho^(-1/3) for ~40% acceptance
(Sec. 7); the 4He workloads here ask for ~50%.  The step is parameterised as
step_sigma = c * rho^(-1/3) per Cartesian component, and c is found by bisection
on the N=108 system (b = 1.15 sigma_LJ, rho = 0.02186 / A^3) with 8 walkers,
200 equilibration + 300 measured sweeps each.  The printed c is frozen in the
workload table of the package (paper_1312_1282_amd/configs.py).

Run:  python -m oracle.tune_step
"""
import ctypes as C

import numpy as np

from . import Walker, fcc_start, run_walkers, system, walker_init

RHO = 0.02186
B = 1.15 * 2.556
N = 108


def acceptance(c, walkers=8, equil=200, meas=300):
    L = (N / RHO) ** (1.0 / 3.0)
    sys_ = system(N, L, B, step_sigma=c * RHO ** (-1.0 / 3.0), seed=7)
    xyz = np.stack([fcc_start(sys_, w) for w in range(walkers)])
    accs = (Walker * walkers)(*[walker_init(sys_, xyz[w]) for w in range(walkers)])
    run_walkers(sys_, 0, xyz, accs, 0, equil + meas, equil, 0, 8)
    return sum(a.n_acc for a in accs) / sum(a.n_try for a in accs)


def main():
    lo, hi = 0.05, 0.6
    for _ in range(14):
        mid = 0.5 * (lo + hi)
        a = acceptance(mid)
        print(f"c = {mid:.6f}  acceptance = {a:.4f}", flush=True)
        if a > 0.5:
            lo = mid
        else:
            hi = mid
    c = round(0.5 * (lo + hi), 4)
    print(f"c = {c}  (step_sigma = {c * RHO ** (-1/3):.5f} A at rho = {RHO})  acceptance = {acceptance(c):.4f}")


if __name__ == "__main__":
    main()
