"""Synthetic liquid-4He workloads (Sec. 7 of the paper: 4He at its equilibrium
density, Jastrow wavefunction of Eqs. (6), (8), (9), HFD-B(HE) potential, cubic
periodic box cut at L/2, Gaussian single-particle moves).

All runs start from an fcc lattice with a small deterministic jitter.  The box
side is L = (N / rho)^(1/3).

STEP_C: the Gaussian step is step_sigma = STEP_C * rho^(-1/3) per Cartesian
component.  STEP_C = 0.1764 gives 50.0% acceptance for N=108 at rho = 0.02186
and b = 1.15 sigma (found by bisection with the CPU oracle, oracle/tune_step.py).
The paper's own choice, an rms step of 0.5 rho^(-1/3) at b = 3.07 A, gave ~40%.
"""
from dataclasses import dataclass, replace

SIGMA_LJ = 2.556          # length unit for b (Angstrom)
RHO_EQ = 0.02186          # equilibrium density of liquid 4He (1 / Angstrom^3)
HBAR2_OVER_M = 12.1194    # hbar^2 / m(4He) (K Angstrom^2)
STEP_C = 0.1764

FP64 = 0
FP32 = 1


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    walkers: int
    precision: int = FP64
    density: float = RHO_EQ
    b: float = 1.15 * SIGMA_LJ
    equil: int = 200
    measured: int = 1000
    m: int = 1
    seed: int = 1

    @property
    def L(self) -> float:
        return (self.n / self.density) ** (1.0 / 3.0)

    @property
    def step_sigma(self) -> float:
        return STEP_C * self.density ** (-1.0 / 3.0)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The five workloads of this implementation.
C1_SMALL_FP64 = Workload("he4_n108_w1_fp64", 108, 1, FP64, equil=200, measured=1000, m=1)
C2_N2048_FP64 = Workload("he4_n2048_w512_fp64", 2048, 512, FP64, equil=500, measured=2000, m=5)
C3_N2048_FP32 = Workload("he4_n2048_w1024_fp32mixed", 2048, 1024, FP32, equil=500, measured=2000, m=5)
C5_N10976_FP32 = Workload("he4_n10976_w256_fp32mixed", 10976, 256, FP32, equil=200, measured=500, m=5)
# Walkers beyond one workgroup's LDS, spread over several workgroups (Sec. 3's
# cooperative kernel across compute units; the paper shows 40960 atoms, Sec. 7).
SPREAD_N8000_FP64 = Workload("he4_n8000_w128_fp64_spread", 8000, 128, FP64, equil=100, measured=200, m=5)
SPREAD_N40960_FP32 = Workload("he4_n40960_w64_fp32_spread", 40960, 64, FP32, equil=50, measured=100, m=5)

# Serving stream: N from this set, density U[0.019, 0.026], b U[1.0, 1.3] sigma,
# 64..512 walkers, run until the standard error of E/N is <= 1 mK.
SERVE_N = (108, 256, 500, 864, 2048, 4000)
SERVE_RHO = (0.019, 0.026)
SERVE_B = (1.0 * SIGMA_LJ, 1.3 * SIGMA_LJ)
SERVE_W = (64, 512)
SERVE_RATE = 20.0          # requests per second (Poisson)
SERVE_TARGET_SE = 1.0e-3   # K per atom

ALL = {w.name: w for w in (C1_SMALL_FP64, C2_N2048_FP64, C3_N2048_FP32, C5_N10976_FP32, SPREAD_N8000_FP64,
                            SPREAD_N40960_FP32)}
