"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
harness.  This module holds none of the method's arithmetic: it only draws
macroscopic fields, population perturbations, site samples and ensemble
manifests from fixed seeds (numpy PCG64), so that the HIP path and the CPU
oracle can be fed identical inputs.

Shapes follow the paper's setups: periodic boxes at rest with uniform density
(Sec. 3), the Taylor-Green initial field of Test 2, the anisotropic boxes of
Test 7, and the batched ensemble of mixed D2Q9/D3Q27 replicas.
"""
from __future__ import annotations

import math

import numpy as np


def n_sites(shape):
    n = 1
    for s in shape:
        n *= int(s)
    return n


def shape3(shape):
    """(nx, ny, nz) with nz = 1 for a 2-D shape."""
    s = tuple(int(v) for v in shape)
    return (s + (1, 1))[:3]


def random_macro(shape, seed, rho0=1.0, drho=0.02, umax=0.05, dims=None):
    """Per-site density rho0*(1 + U(-drho, drho)) and velocity U(-umax, umax)
    per component ((3, N), zero beyond ``dims``)."""
    rng = np.random.default_rng(seed)
    n = n_sites(shape)
    dims = dims if dims is not None else len(shape)
    rho = rho0 * (1.0 + rng.uniform(-drho, drho, n))
    u = np.zeros((3, n))
    u[:dims] = rng.uniform(-umax, umax, (dims, n))
    return rho, u


def perturbation(q, n, seed, amp=1e-3):
    """A (q, N) non-equilibrium perturbation, uniform in [-amp, amp]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, (q, n))


def taylor_green(shape, u0):
    """Test 2 initial velocity u_x = -u0 cos(k x) sin(k y),
    u_y = u0 sin(k x) cos(k y) with k = 2 pi / N_y, as (3, N)."""
    nx, ny, nz = shape3(shape)
    k = 2.0 * math.pi / ny
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    ux = -u0 * np.cos(k * x) * np.sin(k * y) * np.ones((nz, 1, 1))
    uy = u0 * np.sin(k * x) * np.cos(k * y) * np.ones((nz, 1, 1))
    u = np.zeros((3, nx * ny * nz))
    u[0] = ux.ravel()
    u[1] = uy.ravel()
    return u


def sample_sites(shape, count, seed, include_corners=True):
    """Distinct site indices (x fastest) drawn uniformly, plus the eight box
    corners and edge midpoints (the periodic-wrap cases) when requested."""
    nx, ny, nz = shape3(shape)
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    picks = set(rng.choice(n, size=min(count, n), replace=False).tolist())
    if include_corners:
        for x in (0, nx // 2, nx - 1):
            for y in (0, ny // 2, ny - 1):
                for z in (0, nz // 2, nz - 1):
                    picks.add(x + nx * (y + ny * z))
    return np.array(sorted(picks), dtype=np.int64)


def ensemble_manifest(seed=2026, n2d=256, n3d=64, edge2d=(32, 512), edge3d=(32, 96),
                      kT_range=(1e-6, 1e-3), tau_range=(0.502, 2.0), seed_base=1000):
    """Replica list of the batched ensemble: D2Q9 replicas with every edge
    drawn independently and uniformly in ``edge2d`` and D3Q27 replicas in
    ``edge3d``; per replica seed = seed_base + r, kT log-uniform in
    ``kT_range``, tau uniform in ``tau_range``, rho0 = 1."""
    rng = np.random.default_rng(seed)
    out = []
    r = 0
    for q, count, (lo, hi), dims in ((9, n2d, edge2d, 2), (27, n3d, edge3d, 3)):
        for _ in range(count):
            edges = rng.integers(lo, hi + 1, dims).tolist()
            shape = tuple(edges) + ((1,) if dims == 2 else ())
            kT = float(math.exp(rng.uniform(math.log(kT_range[0]), math.log(kT_range[1]))))
            tau = float(rng.uniform(*tau_range))
            out.append({"q": q, "shape": shape, "kT": kT, "tau": tau, "rho0": 1.0,
                        "seed": seed_base + r, "replica": r})
            r += 1
    return out
