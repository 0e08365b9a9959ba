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
