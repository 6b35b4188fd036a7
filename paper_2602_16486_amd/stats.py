"""Host-side diagnostics of a statistics series (rows of cmf_stats, columns
``STAT_COLUMNS``), as the paper defines them (Sec. 3):

* theta_a = (kT/rho0 - <u_a^2>) / (kT/rho0) x 100 (Test 3),
* bias = mean over the window of <u_a^2>(t) - kT/rho0 and
  RMS = sqrt(mean of (<u_a^2>(t) - kT/rho0)^2) (Test 3, Table 2),
* e = (1/d) sum_a <u_a^2> with its bias and RMS, and the anisotropy
  max_a |bias_a - bias_e| (Test 7, Table 3),
* psi = |kT/rho0 - (1/d) sum_a <u_a^2>| / (kT/rho0) x 100 (Test 6),
where <.> is the spatial mean at one step and the window is a range of
recorded steps.
"""
from __future__ import annotations

import numpy as np


def spatial_means(series, n_sites, dims):
    """(T, dims) array of <u_a^2>(t)."""
    s = np.asarray(series)
    return s[:, 8:8 + dims] / n_sites


def equipartition(series, n_sites, kT, rho0, dims, start=0, stop=None):
    """Diagnostics of the window series[start:stop]."""
    u2 = spatial_means(series, n_sites, dims)[start:stop]
    target = kT / rho0
    dev = u2 - target
    e = u2.mean(axis=1)
    bias = dev.mean(axis=0)
    bias_e = float((e - target).mean())
    out = {
        "steps": int(len(u2)),
        "u2_over_target": (u2.mean(axis=0) / target).tolist(),
        "theta_percent": ((target - u2.mean(axis=0)) / target * 100).tolist(),
        "bias": bias.tolist(),
        "rms": np.sqrt((dev ** 2).mean(axis=0)).tolist(),
        "bias_e": bias_e,
        "rms_e": float(np.sqrt(((e - target) ** 2).mean())),
        "anisotropy": float(np.abs(bias - bias_e).max()),
        "psi_percent": float(abs(target - e.mean()) / target * 100),
        # white-noise size of the per-step RMS (independent sites)
        "rms_white": float(np.sqrt(2.0 / n_sites) * target),
    }
    return out


def conservation(series):
    """Largest change of total mass and momentum over the series."""
    s = np.asarray(series)
    return {"mass_drift": float(np.ptp(s[:, 1])), "momentum_drift": float(np.abs(s[:, 2:5] - s[0, 2:5]).max())}
