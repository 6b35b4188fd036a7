"""FP64 CPU oracle of the fluctuating central-moment LBM (De Rosis & Zhou,
arXiv 2602.16486) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``cmflb_oracle.c`` (plain C,
FP64, OpenMP over lattice rows) through ctypes and shares no code with the HIP
library.  See the header of ``cmflb_oracle.c`` for what each routine follows in
the paper and for the readings taken where the paper is ambiguous.

Array conventions: populations are ``(q, N)`` float64 arrays in the paper's
velocity order, site ``s = x + nx*(y + ny*z)``; velocities are ``(3, N)``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import build as _build, library_path

NSTAT = 12
# column names of one statistics row
STAT_COLUMNS = ("step", "sum_rho", "sum_jx", "sum_jy", "sum_jz",
                "sum_ux", "sum_uy", "sum_uz", "sum_ux2", "sum_uy2", "sum_uz2",
                "nonfinite")

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_up = ctypes.POINTER(ctypes.c_uint32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        _build()
    lib = ctypes.CDLL(path)
    c_int, c_double, c_u32, c_u64, c_i64 = (ctypes.c_int, ctypes.c_double, ctypes.c_uint32,
                                            ctypes.c_uint64, ctypes.c_int64)
    lib.orc_lattice.argtypes = [c_int, _ip, _dp]
    lib.orc_transform.argtypes = [c_int, c_int, _dp, _dp]
    lib.orc_norms.argtypes = [c_int, c_int, _dp]
    lib.orc_equilibrium.argtypes = [c_int, c_double, _dp, _dp]
    lib.orc_paper_lambda.argtypes = [c_int, c_double, _dp]
    lib.orc_normals.argtypes = [c_int, c_u64, c_u32, c_u64, c_u32, _dp]
    lib.orc_philox4x32_10.argtypes = [_up, _up, _up]
    lib.orc_philox4x32_10.restype = None
    lib.orc_collide_site.argtypes = [c_int, c_int, c_int, c_double, _dp, _dp, _dp,
                                     _dp, _dp, _dp, _dp]
    lib.orc_run.argtypes = [c_int, c_int, c_int, c_int, c_int, c_int, c_double, _dp,
                            c_u64, c_u32, _dp, c_i64, c_i64, _dp, c_int]
    lib.orc_init_equilibrium.argtypes = [c_int, c_i64, c_double, _dp, _dp, _dp]
    lib.orc_hermite.argtypes = [_dp, _ip, c_int]
    lib.orc_hermite.restype = c_double
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def _vec3(u):
    out = np.zeros(3)
    if u is not None:
        u = np.asarray(u, dtype=np.float64).ravel()
        out[: u.size] = u
    return out


def lattice(q):
    """Velocities ``c`` (q, 3) int and weights ``w`` (q,) in the paper's order."""
    lib = _load()
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    _check(lib.orc_lattice(q, c.ctypes.data_as(_ip), _d(w)), "lattice")
    return c, w


def transform(q, u=None, basis=0):
    """T(u) (row v, column i); ``u=None`` gives the raw-moment matrix M."""
    lib = _load()
    T = np.zeros((q, q))
    uu = _vec3(u)
    _check(lib.orc_transform(q, basis, _d(uu) if u is not None else None, _d(T)), "transform")
    return T


def norms(q, basis=0):
    lib = _load()
    b = np.zeros(q)
    _check(lib.orc_norms(q, basis, _d(b)), "norms")
    return b


def equilibrium(q, rho, u):
    lib = _load()
    f = np.zeros(q)
    uu = _vec3(u)
    _check(lib.orc_equilibrium(q, float(rho), _d(uu), _d(f)), "equilibrium")
    return f


def hermite(c, idx):
    """Hermite tensor component H^(n)_idx(c) (idx: axis indices 0/1/2)."""
    lib = _load()
    cc = _vec3(c)
    ii = np.ascontiguousarray(idx, dtype=np.int32)
    return lib.orc_hermite(_d(cc), ii.ctypes.data_as(_ip), len(ii))


def paper_lambda(q, omega):
    lib = _load()
    lam = np.zeros(q)
    _check(lib.orc_paper_lambda(q, float(omega), _d(lam)), "paper_lambda")
    return lam


def normals(q, seed, replica, step, site):
    """eta[v] for one site and step (zero on the conserved modes)."""
    lib = _load()
    eta = np.zeros(q)
    _check(lib.orc_normals(q, seed, replica, step, site, _d(eta)), "normals")
    return eta


def philox4x32_10(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(c.ctypes.data_as(_up), k.ctypes.data_as(_up), out.ctypes.data_as(_up))
    return out


def collide_site(q, f, eta, kT, lam, basis=0, method=0):
    """One collision at one site; returns a dict with macro (rho, ux, uy, uz),
    kpre, kstar and fstar."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    mac, kpre, kstar, fstar = np.zeros(4), np.zeros(q), np.zeros(q), np.zeros(q)
    _check(lib.orc_collide_site(q, basis, method, float(kT), _d(lam), _d(f), _d(eta), _d(mac),
                                _d(kpre), _d(kstar), _d(fstar)), "collide_site")
    return {"macro": mac, "kpre": kpre, "kstar": kstar, "fstar": fstar}


def init_equilibrium(q, n_sites, rho0=1.0, rho=None, u=None):
    """(q, N) equilibrium populations of per-site rho (N,) and u (3, N)."""
    lib = _load()
    f = np.zeros((q, n_sites))
    r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    _check(lib.orc_init_equilibrium(q, n_sites, float(rho0), None if r is None else _d(r),
                                    None if uu is None else _d(uu), _d(f)), "init_equilibrium")
    return f


def run(q, shape, f, kT, lam, seed, replica=0, step0=0, nsteps=1, basis=0, method=0,
        nthreads=0):
    """Advance ``f`` ((q, N) float64, modified in place) by ``nsteps`` and return
    the (nsteps, 12) statistics rows (columns ``STAT_COLUMNS``)."""
    lib = _load()
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    if not (f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (q, nx * ny * nz)):
        raise ValueError("f must be a C-contiguous float64 array of shape (q, N)")
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    stats = np.zeros((nsteps, NSTAT))
    rc = lib.orc_run(q, basis, method, nx, ny, nz, float(kT), _d(lam), seed, replica, _d(f),
                     step0, nsteps, _d(stats), nthreads)
    _check(rc, "run")
    return stats
