"""Velocity statistics of oracle states -- TEST INFRASTRUCTURE ONLY.

Test 7, Fig. 8: probability densities of the velocity components, normalised
by their empirical standard deviation, and the moments behind them.  From
FP64 populations by the plain definitions: u = sum_i c_i f_i / sum_i f_i
(eq. macro), central moments about the mean over all sites, and a histogram
of x = (u_a - mean_a) / sigma_a with an underflow bin (x < -xmax), nbins
equal bins on [-xmax, xmax) and an overflow bin (x >= xmax).
"""
from __future__ import annotations

import numpy as np

from . import lattice


def velocity(q, f):
    """(3, N) velocity of populations f ((q, N) FP64)."""
    c, _ = lattice(q)
    return (c.T.astype(float) @ f) / f.sum(axis=0)


def velocity_moments(u):
    """(3, 4): mean, variance (1/N), skewness and kurtosis of each row."""
    out = np.zeros((3, 4))
    for a in range(3):
        mean = u[a].mean()
        d = u[a] - mean
        var = (d * d).mean()
        out[a, 0], out[a, 1] = mean, var
        if var > 0:
            out[a, 2] = (d ** 3).mean() / var ** 1.5
            out[a, 3] = (d ** 4).mean() / var ** 2
    return out


def velocity_histogram(u, dims, nbins, xmax):
    """(3, nbins + 2) integer counts of the normalised components (rows
    beyond dims are zero), and the normalised values themselves."""
    mom = velocity_moments(u)
    counts = np.zeros((3, nbins + 2), dtype=np.int64)
    xs = []
    width = 2.0 * xmax / nbins
    for a in range(dims):
        x = (u[a] - mom[a, 0]) / np.sqrt(mom[a, 1])
        xs.append(x)
        for v in x:
            if not v >= -xmax:
                counts[a, 0] += 1
            elif v >= xmax:
                counts[a, nbins + 1] += 1
            else:
                counts[a, 1 + min(int(np.floor((v + xmax) / width)), nbins - 1)] += 1
    return counts, xs
