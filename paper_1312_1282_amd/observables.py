"""Host-side analysis of what the sweep accumulates (no GPU work here)."""
import numpy as np


def pair_distribution(counts, n, L, samples):
    """g(r) from summed pair histograms (the g(r) of the paper's analysis of
    sampled configurations, Sec. 5.4).

    counts: [..., nb] pair counts over nb equal bins of [0, L/2] (from
    hevmc_sweep_gr or hevmc_pair_histogram), summed over `samples`
    configurations of n atoms in a box of side L.  Returns (r, g): the bin
    centres and counts divided by what an ideal gas of the same n and L puts in
    each shell, n(n-1)/2 * shell volume / L^3 per configuration.
    """
    counts = np.asarray(counts, dtype=np.float64)
    nb = counts.shape[-1]
    w = 0.5 * L / nb
    edges = np.arange(nb + 1) * w
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    ideal = samples * 0.5 * n * (n - 1) * shell / L ** 3
    return 0.5 * (edges[1:] + edges[:-1]), counts / ideal


TRACE_FIELDS = ("E_L", "V", "T_PB", "T_JF", "T_F", "U")


def energy_at_b(records, lam):
    """E_L and ln psi^2 ratio of sampled configurations at b' = b lam^(1/5).

    records: [..., 6] per-sample (E_L, V, T_PB, T_JF, T_F, U) at parameter b
    (hevmc_sweep_trace).  f of Eq. (9) scales as b^5, so u, ln psi, its
    gradient and its Laplacian at b' are lam times those at b: with
    T_JF = -(hbar^2/4m) sum lap ln psi and T_F = (hbar^2/2m) sum |grad ln psi|^2,
    E_L(b') = V + 2 lam T_JF - lam^2 T_F, and the sampling weight of b' over b
    is exp(2 (lam - 1) U).  Returns (E_L(b'), log weight)."""
    r = np.asarray(records, dtype=np.float64)
    V, tjf, tf, U = r[..., 1], r[..., 3], r[..., 4], r[..., 5]
    return V + 2.0 * lam * tjf - lam * lam * tf, 2.0 * (lam - 1.0) * U


def reweight_b(records, b, b_primes, n_atoms):
    """Correlated-sampling estimates of the energy per atom at other Jastrow
    parameters b' from one run at b (the paper's variational optimisation of
    b, Sec. 2 and Sec. 7, done from a single set of samples).

    records: [W, S, 6] per-sample records of W walkers (all samples pooled;
    each walker's chain samples |psi_b|^2).  Returns a list of dicts with b',
    E/N, and the effective number of samples (sum w)^2 / sum w^2 that says
    how far from b the estimate can be trusted."""
    r = np.asarray(records, dtype=np.float64).reshape(-1, 6)
    out = []
    for bp in b_primes:
        lam = (bp / b) ** 5
        e, lw = energy_at_b(r, lam)
        lw = lw - lw.max()
        w = np.exp(lw)
        out.append({"b": float(bp), "E_per_atom": float((w * e).sum() / w.sum() / n_atoms),
                    "ess": float(w.sum() ** 2 / (w * w).sum())})
    return out

