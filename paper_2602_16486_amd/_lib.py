"""ctypes binding of libcmflb (include/cmflb.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts numpy
arrays to pointers and status codes to exceptions.  It raises at load time
when the built library is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "cmflb.h")

CMF_OK = 0
CMF_EINVAL = -1
CMF_ENOMEM = -2
CMF_EHIP = -3
CMF_ENONFINITE = -4
CMF_EUNSUPPORTED = -5

STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
FLAG_NO_GRAPH = 1
FLAG_NO_STATS = 2
FLAG_IN_PLACE = 4

# columns of one statistics row (same order as cmf_moments)
STAT_COLUMNS = ("step", "sum_rho", "sum_jx", "sum_jy", "sum_jz", "sum_ux", "sum_uy", "sum_uz",
                "sum_ux2", "sum_uy2", "sum_uz2", "nonfinite")


class CmfError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"libcmflb status {code}: {message}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("rho0", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("lam", ctypes.POINTER(ctypes.c_double)),
        ("seed", ctypes.c_uint64),
        ("replica", ctypes.c_uint32),
        ("series_capacity", ctypes.c_int32),
    ]


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("grid", ctypes.c_int32), ("ms_per_step", ctypes.c_double)]


class EnsembleTiles(ctypes.Structure):
    _fields_ = [("spt9", ctypes.c_int32), ("spt3d", ctypes.c_int32), ("ms_per_step", ctypes.c_double)]


class Moments(ctypes.Structure):
    _fields_ = [("v", ctypes.c_double * 12)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def library_path():
    """The in-tree build (the only library the binding loads)."""
    return os.path.join(HERE, "libcmflb.so")


def load():
    """Load the built HIP library; raises if it has not been built.

    When PyTorch shares the process (device buffers, streams), import torch
    before the first call: the torch wheel carries its own HIP runtime, and
    the library must bind to that one (a HIP runtime loaded after another one
    sees no device)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2602_16486_amd.build` "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                              ctypes.c_uint64)
    lib.cmf_version.restype = ctypes.c_char_p
    lib.cmf_version.argtypes = []
    lib.cmf_last_error.restype = ctypes.c_char_p
    lib.cmf_last_error.argtypes = []
    lib.cmf_device_count.argtypes = []
    lib.cmf_create.argtypes = [ctypes.POINTER(Desc), vp, ctypes.POINTER(vp)]
    lib.cmf_destroy.argtypes = [vp]
    lib.cmf_init_equilibrium.argtypes = [vp, _dp, _dp]
    lib.cmf_set_populations.argtypes = [vp, _dp]
    lib.cmf_get_populations.argtypes = [vp, _dp]
    lib.cmf_gather_sites.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), i64, _dp]
    lib.cmf_step.argtypes = [vp, i64]
    lib.cmf_synchronize.argtypes = [vp]
    lib.cmf_profile_steps.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
    lib.cmf_get_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.cmf_set_step.argtypes = [vp, i64]
    lib.cmf_stats.argtypes = [vp, ctypes.POINTER(Moments), i64, ctypes.POINTER(ctypes.c_int64)]
    lib.cmf_sample_macro.argtypes = [vp, vp, vp]
    lib.cmf_get_macro.argtypes = [vp, _dp, _dp]
    lib.cmf_create_external.argtypes = [ctypes.POINTER(Desc), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.cmf_create_external.restype = ctypes.c_int
    lib.cmf_external_bytes.argtypes = [ctypes.POINTER(Desc)]
    lib.cmf_external_bytes.restype = ctypes.c_size_t
    lib.cmf_velocity_pdf.argtypes = [vp, i32, ctypes.c_double, _dp, ctypes.POINTER(ctypes.c_int64)]
    lib.cmf_noise_sample.argtypes = [i32, u64, u32, i64, i64, i64, i32, _dp]
    lib.cmf_philox_words.argtypes = [ctypes.POINTER(ctypes.c_uint32), i64, u32, u32,
                                     ctypes.POINTER(ctypes.c_uint32)]
    lib.cmf_stream_copy.argtypes = [ctypes.c_size_t, i32, ctypes.POINTER(ctypes.c_double)]
    lib.cmf_step_noalloc.argtypes = [ctypes.POINTER(Desc), vp, vp, i64, i32, i32, vp, vp]
    lib.cmf_step_noalloc.restype = ctypes.c_int
    lib.cmf_get_launch.argtypes = [vp, ctypes.POINTER(Launch)]
    lib.cmf_set_launch.argtypes = [vp, i32, i32]
    lib.cmf_autotune.argtypes = [vp, i32, ctypes.POINTER(Launch), i32, ctypes.POINTER(ctypes.c_int32)]
    lib.cmf_ensemble_create.argtypes = [ctypes.POINTER(Desc), i32, vp, ctypes.POINTER(vp)]
    lib.cmf_ensemble_destroy.argtypes = [vp]
    lib.cmf_ensemble_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.cmf_ensemble_init_equilibrium.argtypes = [vp, i32, _dp, _dp]
    lib.cmf_ensemble_set_populations.argtypes = [vp, i32, _dp]
    lib.cmf_ensemble_get_populations.argtypes = [vp, i32, _dp]
    lib.cmf_ensemble_step.argtypes = [vp, i64]
    lib.cmf_ensemble_profile_steps.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
    lib.cmf_ensemble_synchronize.argtypes = [vp]
    lib.cmf_ensemble_get_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.cmf_ensemble_set_step.argtypes = [vp, i64]
    lib.cmf_ensemble_stats.argtypes = [vp, i32, ctypes.POINTER(Moments), i64, ctypes.POINTER(ctypes.c_int64)]
    lib.cmf_ensemble_get_tiles.argtypes = [vp, ctypes.POINTER(EnsembleTiles)]
    lib.cmf_ensemble_set_tiles.argtypes = [vp, i32, i32]
    lib.cmf_ensemble_autotune.argtypes = [vp, i32, ctypes.POINTER(EnsembleTiles), i32,
                                          ctypes.POINTER(ctypes.c_int32)]
    lib.cmf_sk_reset.argtypes = [vp, i32]
    lib.cmf_sk_accumulate.argtypes = [vp]
    lib.cmf_sk_shells.argtypes = [vp, _dp, ctypes.POINTER(ctypes.c_int64)]
    for name in ("cmf_sk_reset", "cmf_sk_accumulate", "cmf_sk_shells"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("cmf_ensemble_create", "cmf_ensemble_destroy", "cmf_ensemble_info",
                 "cmf_ensemble_init_equilibrium", "cmf_ensemble_set_populations",
                 "cmf_ensemble_get_populations", "cmf_ensemble_step", "cmf_ensemble_profile_steps",
                 "cmf_ensemble_synchronize", "cmf_ensemble_get_step", "cmf_ensemble_set_step",
                 "cmf_ensemble_stats",
                 "cmf_ensemble_get_tiles", "cmf_ensemble_set_tiles", "cmf_ensemble_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("cmf_get_launch", "cmf_set_launch", "cmf_autotune", "cmf_stream_copy", "cmf_create", "cmf_destroy", "cmf_init_equilibrium", "cmf_set_populations",
                 "cmf_get_populations", "cmf_gather_sites", "cmf_step", "cmf_synchronize",
                 "cmf_get_step", "cmf_set_step", "cmf_stats", "cmf_sample_macro", "cmf_get_macro", "cmf_velocity_pdf",
                 "cmf_noise_sample",
                 "cmf_philox_words", "cmf_device_count", "cmf_profile_steps"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc):
    if rc != CMF_OK:
        raise CmfError(rc, load().cmf_last_error().decode())
    return rc


def declared_functions(header=HEADER):
    """Names of the functions declared in include/cmflb.h."""
    text = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(cmf_\w+)\s*\(", text, re.M)))


def make_desc(q, shape, storage="f32", rho0=1.0, tau=0.8, kT=0.0, lam=None, seed=1, replica=0,
              flags=0, series_capacity=0):
    """A Desc plus the numpy array that keeps its rate vector alive."""
    nx, ny, nz = (tuple(int(s) for s in shape) + (1, 1))[:3]
    d = Desc()
    d.q, d.nx, d.ny, d.nz = int(q), nx, ny, nz
    d.storage = STORAGE[storage]
    d.flags = flags
    d.rho0, d.tau, d.kT = float(rho0), float(tau), float(kT)
    keep = None
    if lam is not None:
        keep = np.ascontiguousarray(lam, dtype=np.float64)
        if keep.shape != (int(q),):
            raise ValueError(f"lam must have {q} entries")
        d.lam = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.seed = int(seed)
    d.replica = int(replica)
    d.series_capacity = int(series_capacity)
    return d, keep


def _d(a):
    return a.ctypes.data_as(_dp)


def version():
    return load().cmf_version().decode()


def device_count():
    return load().cmf_device_count()


def noise_sample(q, seed, replica, step, site0, n, fp64=False):
    """(n, q) normals the step kernels draw (zeros on conserved modes)."""
    lib = load()
    out = np.zeros((n, q))
    check(lib.cmf_noise_sample(q, seed, replica, step, site0, n, 1 if fp64 else 0, _d(out)))
    return out


def philox_words(ctr, key0, key1):
    """Philox4x32-10 on the device for counters ctr (n, 4) uint32."""
    lib = load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    up = ctypes.POINTER(ctypes.c_uint32)
    check(lib.cmf_philox_words(c.ctypes.data_as(up), c.shape[0], key0, key1, out.ctypes.data_as(up)))
    return out


def stream_copy(nbytes, reps=5):
    """Fastest plain device copy of nbytes (ms): read nbytes + write nbytes."""
    ms = ctypes.c_double()
    check(load().cmf_stream_copy(int(nbytes), int(reps), ctypes.byref(ms)))
    return ms.value
