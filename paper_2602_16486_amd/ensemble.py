"""Python-side handle of a batched ensemble of libcmflb (a thin wrapper of
the C ABI; every computation runs in the HIP kernels)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib


class Ensemble:
    """Many independent D2Q9/D3Q27 replicas advanced by one fused launch per
    step.  ``replicas`` is a list of dicts with the keyword arguments of
    :class:`Lattice` (q, shape, rho0, tau, kT, lam, seed, replica); ``storage``,
    ``flags`` and ``series_capacity`` are common to all."""

    def __init__(self, replicas, storage="f32", flags=0, stream=None, series_capacity=0):
        self._lib = _lib.load()
        descs = (_lib.Desc * len(replicas))()
        self._keep = []
        self.q, self.shapes, self.sizes = [], [], []
        for k, r in enumerate(replicas):
            d, keep = _lib.make_desc(r["q"], r["shape"], storage=storage, rho0=r.get("rho0", 1.0),
                                     tau=r.get("tau", 0.8), kT=r.get("kT", 0.0), lam=r.get("lam"),
                                     seed=r.get("seed", 1), replica=r.get("replica", k), flags=flags,
                                     series_capacity=series_capacity)
            descs[k] = d
            self._keep.append(keep)
            self.q.append(int(r["q"]))
            self.shapes.append((d.nx, d.ny, d.nz))
            self.sizes.append(d.nx * d.ny * d.nz)
        handle = ctypes.c_void_p()
        _lib.check(self._lib.cmf_ensemble_create(descs, len(replicas), ctypes.c_void_p(stream or 0),
                                                 ctypes.byref(handle)))
        self._h = handle
        self.n = len(replicas)
        # steps each replica's statistics ring holds (the library's default
        # when 0); no call can return more rows
        self._ring = int(series_capacity) if int(series_capacity) > 0 else 4096

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cmf_ensemble_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def info(self):
        n, sites, tiles = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _lib.check(self._lib.cmf_ensemble_info(self._h, ctypes.byref(n), ctypes.byref(sites),
                                               ctypes.byref(tiles)))
        return {"replicas": n.value, "sites": sites.value, "tiles": tiles.value}

    def init_equilibrium(self, index, rho=None, u=None):
        n = self.sizes[index]
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(n)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(3, n)
        _lib.check(self._lib.cmf_ensemble_init_equilibrium(
            self._h, index, None if r is None else _lib._d(r), None if uu is None else _lib._d(uu)))

    def set_populations(self, index, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (self.q[index], self.sizes[index]):
            raise ValueError("populations have the wrong shape")
        _lib.check(self._lib.cmf_ensemble_set_populations(self._h, index, _lib._d(f)))

    def get_populations(self, index):
        f = np.zeros((self.q[index], self.sizes[index]))
        _lib.check(self._lib.cmf_ensemble_get_populations(self._h, index, _lib._d(f)))
        return f

    def step(self, n=1):
        _lib.check(self._lib.cmf_ensemble_step(self._h, int(n)))

    # -- tile shape ---------------------------------------------------------
    @property
    def tiles(self):
        """(spt9, spt3d): sites per thread of the D2Q9 and of the 3-D tiles."""
        out = _lib.EnsembleTiles()
        _lib.check(self._lib.cmf_ensemble_get_tiles(self._h, ctypes.byref(out)))
        return out.spt9, out.spt3d

    def set_tiles(self, spt9, spt3d):
        _lib.check(self._lib.cmf_ensemble_set_tiles(self._h, int(spt9), int(spt3d)))

    def autotune(self, steps_per_trial=5):
        """Time the candidate tile shapes (state restored afterwards), keep
        the fastest; returns a list of (spt9, spt3d, ms_per_step)."""
        cap = 64
        buf = (_lib.EnsembleTiles * cap)()
        n = ctypes.c_int32()
        _lib.check(self._lib.cmf_ensemble_autotune(self._h, int(steps_per_trial), buf, cap,
                                                   ctypes.byref(n)))
        return [(buf[k].spt9, buf[k].spt3d, buf[k].ms_per_step) for k in range(min(n.value, cap))]

    def profile_steps(self, n):
        ms = ctypes.c_double()
        _lib.check(self._lib.cmf_ensemble_profile_steps(self._h, int(n), ctypes.byref(ms)))
        return ms.value

    def synchronize(self):
        _lib.check(self._lib.cmf_ensemble_synchronize(self._h))

    @property
    def step_index(self):
        v = ctypes.c_int64()
        _lib.check(self._lib.cmf_ensemble_get_step(self._h, ctypes.byref(v)))
        return v.value

    @step_index.setter
    def step_index(self, step):
        """Set the index of the next step (resuming a saved run continues its
        noise sequence)."""
        _lib.check(self._lib.cmf_ensemble_set_step(self._h, int(step)))

    def stats(self, index, cap=1 << 16, raise_nonfinite=True):
        """Statistics rows of replica ``index`` since the previous call, as
        :meth:`Lattice.stats`."""
        cap = max(0, min(int(cap), self._ring))
        buf = (_lib.Moments * cap)()
        n = ctypes.c_int64()
        rc = self._lib.cmf_ensemble_stats(self._h, index, buf, cap, ctypes.byref(n))
        out = np.frombuffer(buf, dtype=np.float64, count=12 * n.value).reshape(n.value, 12).copy()
        if rc == _lib.CMF_ENONFINITE and not raise_nonfinite:
            return out
        _lib.check(rc)
        return out
