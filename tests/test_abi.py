"""Host-side checks of the C-ABI library: it loads, exports every function
declared in include/cmflb.h, and rejects invalid descriptors before touching
a device.  CPU only (no compute calls)."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2602_16486_amd import _lib


def test_library_exports_every_declared_function():
    lib = _lib.load()
    names = _lib.declared_functions()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported


def test_version_and_error_string():
    assert _lib.version().startswith("cmflb")
    lib = _lib.load()
    assert isinstance(lib.cmf_last_error(), bytes)


def _create(**kw):
    d = _lib.Desc()
    d.q, d.nx, d.ny, d.nz = kw.get("q", 9), kw.get("nx", 8), kw.get("ny", 8), kw.get("nz", 1)
    d.storage = kw.get("storage", 1)
    d.rho0, d.tau, d.kT = kw.get("rho0", 1.0), kw.get("tau", 0.8), kw.get("kT", 1e-4)
    lam = kw.get("lam")
    if lam is not None:
        arr = (ctypes.c_double * len(lam))(*lam)
        d.lam = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
    d.series_capacity = kw.get("series_capacity", 0)
    h = ctypes.c_void_p()
    rc = _lib.load().cmf_create(ctypes.byref(d), None, ctypes.byref(h))
    return rc, _lib.load().cmf_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    ({"q": 10}, "q must be 9, 19 or 27"),
    ({"q": 9, "nz": 2}, "D2Q9 needs nz = 1"),
    ({"nx": 0}, "box edges"),
    ({"q": 27, "nx": 2048, "ny": 1024, "nz": 1024}, "exceeds 2^31"),
    ({"storage": 7}, "unknown storage"),
    ({"rho0": 0.0}, "rho0"),
    ({"tau": 0.49}, "tau"),
    ({"kT": -1e-4}, "kT"),
    ({"lam": [1.0] * 8 + [2.5]}, "outside [0, 2]"),
    ({"series_capacity": -1}, "series_capacity"),
])
def test_create_rejects_invalid_descriptors(kw, msg):
    rc, err = _create(**kw)
    assert rc == _lib.CMF_EINVAL
    assert msg in err


def test_null_arguments_are_rejected():
    lib = _lib.load()
    assert lib.cmf_create(None, None, None) == _lib.CMF_EINVAL
    assert lib.cmf_step(None, 1) == _lib.CMF_EINVAL
    assert lib.cmf_destroy(None) == _lib.CMF_EINVAL
    assert lib.cmf_noise_sample(10, 1, 0, 0, 0, 4, 0, None) == _lib.CMF_EINVAL
    assert lib.cmf_ensemble_get_tiles(None, None) == _lib.CMF_EINVAL
    assert lib.cmf_ensemble_set_tiles(None, 3, 1) == _lib.CMF_EINVAL
    assert lib.cmf_ensemble_autotune(None, 2, None, 0, None) == _lib.CMF_EINVAL
    ms = ctypes.c_double()
    assert lib.cmf_stream_copy(0, 1, ctypes.byref(ms)) == _lib.CMF_EINVAL
    assert lib.cmf_stream_copy(1 << 20, 0, ctypes.byref(ms)) == _lib.CMF_EINVAL
    assert lib.cmf_stream_copy(1 << 20, 1, None) == _lib.CMF_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    """The binding never falls back to a CPU path: without the built library,
    creating a lattice raises."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2602_16486_amd._lib as L\n"
        "L.library_path = lambda: %r\n"
        "import paper_2602_16486_amd as P\n"
        "try:\n"
        "    P.Lattice(9, (8, 8))\n"
        "except ImportError as e:\n"
        "    print('raised', e)\n" % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                      str(tmp_path / "absent.so")))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert "raised" in out.stdout and "no CPU fallback" in out.stdout


def test_external_buffer_validation_before_any_device_call():
    """cmf_external_bytes and the argument checks of cmf_create_external run
    on the host: NULL, misaligned and too small buffers are rejected before
    the pointer is looked at."""
    lib = _lib.load()
    d, _ = _lib.make_desc(27, (10, 6, 4), storage="f32")
    need = lib.cmf_external_bytes(ctypes.byref(d))
    assert need == 2 * ((27 * 240 * 4 + 255) // 256 * 256)
    bad, _ = _lib.make_desc(27, (10, 6, 4), storage="f32")
    bad.q = 11
    assert lib.cmf_external_bytes(ctypes.byref(bad)) == 0
    h = ctypes.c_void_p()
    for ptr, nbytes, msg in ((0, need, b"dev_ptr is NULL"), (4096 + 64, need, b"256-byte aligned"),
                             (4096, need - 256, b"needs")):
        rc = lib.cmf_create_external(ctypes.byref(d), ctypes.c_void_p(ptr), nbytes, None, ctypes.byref(h))
        assert rc == _lib.CMF_EINVAL
        assert msg in lib.cmf_last_error()
        assert not h.value


@pytest.mark.parametrize("q", [9, 19, 27])
def test_rate_presets(q):
    from paper_2602_16486_amd import rate_vector
    tau = 0.7
    w = 1 / tau
    paper = rate_vector(q, tau)
    omega_modes = [4, 5] if q == 9 else [7, 8, 9]
    assert np.array_equal(paper, np.where(np.isin(np.arange(q), omega_modes), w, 1.0))
    iso = rate_vector(q, tau, "isotropic")
    if q == 9:
        assert np.array_equal(iso, paper)
    else:
        assert np.array_equal(iso, np.where((np.arange(q) >= 4) & (np.arange(q) <= 9), w, 1.0))
    assert np.array_equal(rate_vector(q, tau, "single"), np.full(q, w))
    with pytest.raises(ValueError):
        rate_vector(q, tau, "bgk")


def test_header_is_plain_c(tmp_path):
    """include/cmflb.h compiles as strict C99 (no C++ in the interface) and a
    C program links against libcmflb and reaches its error path without a
    device."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "t.c"
    src.write_text(
        "#include <stdio.h>\n#include <string.h>\n#include \"cmflb.h\"\n"
        "int main(void) {\n"
        "  cmf_desc d;\n  memset(&d, 0, sizeof d);\n"
        "  int rc = cmf_step(NULL, 1);\n"
        "  printf(\"%s|%d|%s\\n\", cmf_version(), rc, cmf_last_error());\n"
        "  return rc == CMF_EINVAL ? 0 : 1;\n}\n")
    lib = os.path.dirname(_lib.library_path())
    exe = tmp_path / "t"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(root, "include"), str(src), "-L", lib, "-lcmflb",
                    f"-Wl,-rpath,{lib}", "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    version, rc, err = out.strip().split("|")
    assert version.startswith("cmflb") and int(rc) == _lib.CMF_EINVAL and "NULL" in err


def test_ensemble_create_rejects_before_any_device_call():
    """Host-side checks of cmf_ensemble_create: mixed storage, mixed flags,
    a replica of 4 GiB or more (tiles address a replica with 32-bit byte
    offsets) and an invalid member descriptor all fail with CMF_EINVAL."""
    lib = _lib.load()
    cases = [
        ([(9, (16, 16), "f32", 0), (9, (16, 16), "f16", 0)], "storage differs"),
        ([(9, (16, 16), "f32", 0), (9, (16, 16), "f32", _lib.FLAG_NO_GRAPH)], "flags differ"),
        ([(27, (1024, 256, 160), "f32", 0)], "below 4 GiB"),
        ([(9, (16, 16), "f32", 0), (10, (16, 16), "f32", 0)], "q must be"),
    ]
    for members, msg in cases:
        descs = (_lib.Desc * len(members))()
        keep = []
        for k, (q, shape, storage, flags) in enumerate(members):
            d, kp = _lib.make_desc(q, shape, storage=storage, kT=1e-4, flags=flags, replica=k)
            descs[k] = d
            keep.append(kp)
        h = ctypes.c_void_p()
        rc = lib.cmf_ensemble_create(descs, len(members), None, ctypes.byref(h))
        assert rc == _lib.CMF_EINVAL, msg
        assert msg in lib.cmf_last_error().decode()
        assert not h.value


def test_in_place_checks_before_any_device_call():
    """CMF_FLAG_IN_PLACE: cmf_external_bytes counts one population buffer;
    a z plane of 4 GiB or more (in-place steps address a plane with 32-bit
    byte offsets), an ensemble member and cmf_step_noalloc (a two-buffer
    step) are refused with CMF_EUNSUPPORTED before any device call."""
    lib = _lib.load()
    d, _ = _lib.make_desc(27, (10, 6, 4), storage="f32", flags=_lib.FLAG_IN_PLACE)
    assert lib.cmf_external_bytes(ctypes.byref(d)) == (27 * 240 * 4 + 255) // 256 * 256
    big, _ = _lib.make_desc(27, (8192, 8192, 1), storage="f64", flags=_lib.FLAG_IN_PLACE)
    assert lib.cmf_external_bytes(ctypes.byref(big)) == 0
    h = ctypes.c_void_p()
    assert lib.cmf_create(ctypes.byref(big), None, ctypes.byref(h)) == _lib.CMF_EUNSUPPORTED
    assert b"4 GiB" in lib.cmf_last_error() and not h.value
    descs = (_lib.Desc * 1)()
    descs[0] = d
    assert lib.cmf_ensemble_create(descs, 1, None, ctypes.byref(h)) == _lib.CMF_EUNSUPPORTED
    assert b"single lattices" in lib.cmf_last_error() and not h.value
    rc = lib.cmf_step_noalloc(ctypes.byref(d), ctypes.c_void_p(4096), ctypes.c_void_p(8192), 0, 256, 1,
                              None, None)
    assert rc == _lib.CMF_EUNSUPPORTED and b"IN_PLACE" in lib.cmf_last_error()
