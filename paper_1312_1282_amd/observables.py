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



def autocorrelation(x, kmax=None):
    """R(k) of a stationary sequence and its autocorrelation time m_c (the
    definitions of Sec. 4.1): R(k) = sum_i (A_i - <A>)(A_{i+k} - <A>) /
    sum_i (A_i - <A>)^2, and m_c = sum_{k >= 1} R(k), the sum cut where R first
    falls to zero or below (beyond that the estimate is noise).  Returns
    (R[0..kmax], m_c)."""
    a = np.asarray(x, dtype=np.float64)
    a = a - a.mean()
    n = len(a)
    kmax = n // 4 if kmax is None else min(kmax, n - 1)
    den = (a * a).sum()
    R = np.array([(a[: n - k] * a[k:]).sum() / den for k in range(kmax + 1)])
    mc = 0.0
    for k in range(1, kmax + 1):
        if R[k] <= 0.0:
            break
        mc += R[k]
    return R, mc


def blocking(x):
    """Flyvbjerg-Petersen reblocking of a correlated sequence (the reblocking
    the paper names as an alternative to summing R(k), Sec. 4.1): at level l
    the sequence is averaged in consecutive pairs l times, and the standard
    error of the mean is estimated as if the blocks were independent,
    se_l = sqrt(var_l / (n_l - 1)), with its own uncertainty
    se_l / sqrt(2 (n_l - 1)).  Levels run while n_l >= 4.  Returns a list of
    (n_l, se_l, dse_l)."""
    a = np.asarray(x, dtype=np.float64).copy()
    out = []
    while len(a) >= 4:
        n = len(a)
        var = a.var()                      # population variance of the blocks
        se = np.sqrt(var / (n - 1))
        out.append((n, float(se), float(se / np.sqrt(2.0 * (n - 1)))))
        if n % 2:
            a = a[:-1]
        a = 0.5 * (a[0::2] + a[1::2])
    return out


def blocking_se(x):
    """Standard error of the mean of a correlated sequence from reblocking:
    the estimate at the first level after which reblocking stops raising it,
    i.e. the next two levels exceed it by no more than its own uncertainty
    (once and twice over); if no level qualifies, the largest estimate.
    Returns (se, level)."""
    lv = blocking(x)
    if not lv:
        return float("nan"), -1
    for l in range(len(lv)):
        se, dse = lv[l][1], lv[l][2]
        nxt = [lv[m][1] for m in (l + 1, l + 2) if m < len(lv)]
        if len(nxt) >= 1 and nxt[0] - se <= dse and (len(nxt) < 2 or nxt[1] - se <= 2.0 * dse):
            return se, l
    k = int(np.argmax([se for _, se, _ in lv]))
    return lv[k][1], k
