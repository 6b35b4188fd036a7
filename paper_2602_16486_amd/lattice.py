"""Python-side handle of one lattice of libcmflb (a thin wrapper of the C ABI;
every computation runs in the HIP kernels)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib


def rate_vector(q, tau, kind="paper"):
    """Per-mode relaxation rates Lambda_v, in the mode order of the paper's
    bases (Sec. 2.2 for D2Q9, Sec. 2.3 for D3Q27, Sec. 2.4 for D3Q19),
    omega = 1 / tau.

    * ``paper``: the printed rates -- D2Q9 Lambda_4 = Lambda_5 = omega, D3Q27
      and D3Q19 Lambda_7..9 = omega, every other mode 1.  On the 3-D lattices
      the diagonal second-order modes (4..6) then relax at 1, so
      normal-stress differences diffuse with nu = c_s^2 (1 - 1/2) = 1/6
      whatever tau is, and only the off-diagonal shear follows
      c_s^2 (tau - 1/2).
    * ``isotropic``: 3-D lattices with Lambda_4..9 = omega (one viscosity
      for every second-order mode, bulk included); on D2Q9 the paper's rates,
      which are already isotropic.
    * ``single``: Lambda_v = omega for every mode (single-rate comparator of
      Test 6).
    """
    omega = 1.0 / float(tau)
    lam = np.ones(int(q))
    if kind == "single":
        lam[:] = omega
    elif kind == "paper" or (kind == "isotropic" and q == 9):
        lam[[4, 5] if q == 9 else [7, 8, 9]] = omega
    elif kind == "isotropic":
        lam[4:10] = omega
    else:
        raise ValueError(f"unknown rate kind {kind!r}")
    return lam


def external_bytes(q, shape, storage="f32", in_place=False):
    """Device bytes a lattice needs for its population buffers (two, or one
    with ``in_place``) when they are provided by the caller
    (``Lattice(..., external=(ptr, nbytes))``)."""
    lib = _lib.load()
    d, _ = _lib.make_desc(q, shape, storage=storage, flags=_lib.FLAG_IN_PLACE if in_place else 0)
    n = lib.cmf_external_bytes(ctypes.byref(d))
    if n == 0:
        raise ValueError("invalid lattice description")
    return int(n)


class Lattice:
    """A periodic D2Q9, D3Q19 or D3Q27 box stepped by the fused CM-FLBM kernel.

    ``shape`` is (nx, ny) or (nx, ny, nz); ``storage`` one of f64, f32, f16,
    bf16; ``lam`` optional per-mode relaxation rates (default: the paper's);
    ``stream`` an optional hipStream_t handle (int), e.g.
    ``torch.cuda.current_stream().cuda_stream``; ``external`` an optional
    (device pointer, bytes) pair of caller-owned memory for the population
    buffers (see :func:`external_bytes`), e.g. from a torch tensor;
    ``in_place`` in-place (AA) streaming on one population buffer (half the
    population memory, the same results bit for bit).
    """

    def __init__(self, q, shape, storage="f32", rho0=1.0, tau=0.8, kT=0.0, lam=None, seed=1,
                 replica=0, flags=0, stream=None, series_capacity=0, external=None,
                 in_place=False):
        self._lib = _lib.load()
        nx, ny, nz = (tuple(int(s) for s in shape) + (1, 1))[:3]
        self.q = int(q)
        self.shape = (nx, ny, nz)
        self.n = nx * ny * nz
        self.storage = storage
        d = _lib.Desc()
        d.q, d.nx, d.ny, d.nz = self.q, nx, ny, nz
        d.storage = _lib.STORAGE[storage]
        d.flags = flags | (_lib.FLAG_IN_PLACE if in_place else 0)
        d.rho0, d.tau, d.kT = float(rho0), float(tau), float(kT)
        self._lam = None
        if lam is not None:
            self._lam = np.ascontiguousarray(lam, dtype=np.float64)
            if self._lam.shape != (self.q,):
                raise ValueError(f"lam must have {self.q} entries")
            d.lam = self._lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.seed = int(seed)
        d.replica = int(replica)
        d.series_capacity = int(series_capacity)
        # the statistics ring holds this many steps (the library's default
        # when 0); no call can return more rows
        self._ring = int(series_capacity) if int(series_capacity) > 0 else 4096
        self.rho0, self.tau, self.kT = float(rho0), float(tau), float(kT)
        handle = ctypes.c_void_p()
        if external is None:
            _lib.check(self._lib.cmf_create(ctypes.byref(d), ctypes.c_void_p(stream or 0),
                                            ctypes.byref(handle)))
        else:
            ptr, nbytes = external
            _lib.check(self._lib.cmf_create_external(ctypes.byref(d), ctypes.c_void_p(int(ptr)),
                                                     int(nbytes), ctypes.c_void_p(stream or 0),
                                                     ctypes.byref(handle)))
        self._h = handle

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.cmf_destroy(self._h)
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

    # -- state --------------------------------------------------------------
    def init_equilibrium(self, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(self.n)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(3, self.n)
        _lib.check(self._lib.cmf_init_equilibrium(
            self._h, None if r is None else _lib._d(r), None if uu is None else _lib._d(uu)))

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (self.q, self.n):
            raise ValueError(f"populations must have shape {(self.q, self.n)}")
        _lib.check(self._lib.cmf_set_populations(self._h, _lib._d(f)))

    def get_populations(self):
        f = np.zeros((self.q, self.n))
        _lib.check(self._lib.cmf_get_populations(self._h, _lib._d(f)))
        return f

    def macroscopic(self):
        """(rho, u) of the current pre-collision state, FP64 from the device:
        rho shape (N,), u shape (3, N)."""
        rho = np.zeros(self.n)
        u = np.zeros((3, self.n))
        _lib.check(self._lib.cmf_get_macro(self._h, _lib._d(rho), _lib._d(u)))
        return rho, u

    def velocity_pdf(self, nbins=64, xmax=5.0):
        """Velocity statistics of the current state (device): returns
        (moments, counts) with moments shape (3, 4) = mean, variance,
        skewness, kurtosis per component and counts shape (3, nbins + 2) of
        x = (u_a - mean_a) / sigma_a (first / last column: below -xmax /
        at or above xmax)."""
        mom = np.zeros(12)
        counts = np.zeros(3 * (nbins + 2), dtype=np.int64)
        _lib.check(self._lib.cmf_velocity_pdf(self._h, int(nbins), float(xmax), _lib._d(mom),
                                              counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return mom.reshape(3, 4), counts.reshape(3, nbins + 2)

    def gather_sites(self, sites):
        s = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.zeros((s.size, self.q))
        _lib.check(self._lib.cmf_gather_sites(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                              s.size, _lib._d(out)))
        return out

    # -- stepping -----------------------------------------------------------
    def step(self, n=1):
        _lib.check(self._lib.cmf_step(self._h, int(n)))

    def profile_steps(self, n):
        """Run n direct-launch steps with HIP events around each fused-step
        kernel; returns the summed kernel time in milliseconds."""
        ms = ctypes.c_double()
        _lib.check(self._lib.cmf_profile_steps(self._h, int(n), ctypes.byref(ms)))
        return ms.value

    # -- structure factor --------------------------------------------------
    def sk_reset(self, nbins=64):
        self._sk_nbins = int(nbins)
        _lib.check(self._lib.cmf_sk_reset(self._h, int(nbins)))

    def sk_accumulate(self):
        _lib.check(self._lib.cmf_sk_accumulate(self._h))

    def sk_shells(self):
        """(nbins, 6) array: mean |k|, modes, S_rho, S_ux, S_uy, S_uz; and
        the number of samples."""
        out = np.zeros((self._sk_nbins, 6))
        ns = ctypes.c_int64()
        _lib.check(self._lib.cmf_sk_shells(self._h, _lib._d(out), ctypes.byref(ns)))
        return out, ns.value

    # -- launch shape -------------------------------------------------------
    @property
    def launch(self):
        """(block, grid) of the fused-step kernel."""
        out = _lib.Launch()
        _lib.check(self._lib.cmf_get_launch(self._h, ctypes.byref(out)))
        return out.block, out.grid

    def set_launch(self, block, grid):
        _lib.check(self._lib.cmf_set_launch(self._h, int(block), int(grid)))

    def autotune(self, steps_per_trial=10):
        """Time the candidate launch shapes (state restored afterwards), keep
        the fastest; returns a list of (block, grid, ms_per_step)."""
        cap = 64
        buf = (_lib.Launch * cap)()
        n = ctypes.c_int32()
        _lib.check(self._lib.cmf_autotune(self._h, int(steps_per_trial), buf, cap, ctypes.byref(n)))
        return [(buf[k].block, buf[k].grid, buf[k].ms_per_step) for k in range(min(n.value, cap))]

    def synchronize(self):
        _lib.check(self._lib.cmf_synchronize(self._h))

    @property
    def step_index(self):
        v = ctypes.c_int64()
        _lib.check(self._lib.cmf_get_step(self._h, ctypes.byref(v)))
        return v.value

    @step_index.setter
    def step_index(self, step):
        """Set the index of the next step (resuming a saved run continues its
        noise sequence)."""
        _lib.check(self._lib.cmf_set_step(self._h, int(step)))

    def stats(self, cap=1 << 20, raise_nonfinite=True):
        """(n, 12) array of the per-step statistics rows recorded since the
        previous call (columns ``_lib.STAT_COLUMNS``), at most the last
        min(cap, series capacity) of them."""
        cap = max(0, min(int(cap), self._ring))
        buf = (_lib.Moments * cap)()
        n = ctypes.c_int64()
        rc = self._lib.cmf_stats(self._h, buf, cap, ctypes.byref(n))
        out = np.frombuffer(buf, dtype=np.float64, count=12 * n.value).reshape(n.value, 12).copy()
        if rc == _lib.CMF_ENONFINITE and not raise_nonfinite:
            return out
        _lib.check(rc)
        return out

    def sample_macro(self, rho_ptr, u_ptr):
        """Write rho (N floats) and u (3N floats) into device buffers given as
        raw device pointers (ints), e.g. ``tensor.data_ptr()``."""
        _lib.check(self._lib.cmf_sample_macro(self._h, ctypes.c_void_p(rho_ptr or 0),
                                              ctypes.c_void_p(u_ptr or 0)))
