"""cmf_step_noalloc, the allocation-free step (statistics scratch in a static
device array): two calls in a row, the second on a smaller lattice, each
equal to cmf_step of a lattice on the same state in the same launch shape --
the stored state bit for bit and the statistics row exactly (same kernels,
same summation order).  Needs an MI355X."""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import Lattice, _lib, external_bytes
from paper_2602_16486_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


def _state(q, shape, seed):
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, seed, umax=0.04, dims=2 if q == 9 else 3)
    return O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, seed + 1, 5e-4)


def _buffers(torch, q, shape, storage):
    """A zeroed device tensor holding the two population buffers at a
    256-byte aligned address: (tensor, offset of that address, bytes)."""
    nbytes = external_bytes(q, shape, storage)
    t = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-t.data_ptr()) % 256
    return t, off, nbytes


# (q, shape, storage, launch shape, step index): the second lattice is
# smaller than the first, so the second call finds the first one's partial
# sums in the scratch beyond its own
CALLS = [
    (27, (40, 12, 10), "f32", (64, 120), 7),        # one workgroup per tile
    (27, (20, 9, 7), "f16", (64, 16), (1 << 32) + 3),  # persistent grid, step beyond 2^32
    (9, (64, 20), "f64", (64, 20), 11),             # D2Q9 one-tile workgroups
    (19, (20, 9, 7), "bf16", (128, 40), 2),
]


def test_noalloc_step_equals_cmf_step():
    import torch
    lib = _lib.load()
    kw = dict(tau=0.7, kT=2e-4, seed=9, replica=3)
    for k, (q, shape, storage, (block, grid), step0) in enumerate(CALLS):
        f0 = _state(q, shape, 40 + k)
        ebytes = q * W.n_sites(shape) * {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[storage]
        # the existing entry point: a lattice on caller-owned buffers
        t1, o1, nb = _buffers(torch, q, shape, storage)
        half = nb // 2
        torch.cuda.synchronize()
        with Lattice(q, shape, storage=storage, external=(t1.data_ptr() + o1, nb), **kw) as a:
            a.set_launch(block, grid)
            a.set_populations(f0)
            a.step_index = step0
            a.step(1)
            ref_st = a.stats()
            a.synchronize()
        ref = t1[o1 + half: o1 + half + ebytes].cpu()
        # the same state written by a lattice into buffer 0 of another tensor,
        # then the allocation-free step into its buffer 1
        t2, o2, _ = _buffers(torch, q, shape, storage)
        base = t2.data_ptr() + o2
        torch.cuda.synchronize()
        with Lattice(q, shape, storage=storage, external=(base, nb), **kw) as b:
            b.set_populations(f0)
            b.synchronize()
        stats = torch.full((12,), -1.0, dtype=torch.float64, device="cuda")
        d, keep = _lib.make_desc(q, shape, storage=storage, **kw)
        torch.cuda.synchronize()
        rc = lib.cmf_step_noalloc(ctypes.byref(d), ctypes.c_void_p(base), ctypes.c_void_p(base + half),
                                  step0, block, grid, ctypes.c_void_p(stats.data_ptr()), None)
        assert rc == _lib.CMF_OK, lib.cmf_last_error().decode()
        torch.cuda.synchronize()
        got = t2[o2 + half: o2 + half + ebytes].cpu()
        assert torch.equal(got, ref), f"call {k}: state differs from cmf_step"
        st = stats.cpu().numpy()
        assert st[0] == step0
        assert np.array_equal(st, ref_st[0]), f"call {k}: statistics differ from cmf_step"


def test_noalloc_rejects_bad_arguments():
    import torch
    lib = _lib.load()
    q, shape, storage = 27, (32, 6, 5), "f32"
    t, off, nb = _buffers(torch, q, shape, storage)
    base = t.data_ptr() + off
    d, keep = _lib.make_desc(q, shape, storage=storage, kT=1e-4)
    half = nb // 2
    cases = [
        ((base, base + half, 0, 64, 65537), b"scratch holds"),        # grid beyond the scratch
        ((base, base + half, 0, 100, 10), b"block must be"),
        ((base, base, 0, 64, 10), b"two different buffers"),
        ((base + 64, base + half, 0, 64, 10), b"256-byte aligned"),
        ((base, base + half, 1 << 56, 64, 10), b"outside [0, 2^56)"),
        ((base, base + half, -1, 64, 10), b"outside [0, 2^56)"),
    ]
    # host memory (256-byte aligned, so that only the memory check refuses it)
    host = np.zeros(nb + 256, dtype=np.uint8)
    hbase = host.ctypes.data + (-host.ctypes.data) % 256
    cases += [
        ((hbase, base + half, 0, 64, 10), b"src is not device memory"),
        ((base, hbase, 0, 64, 10), b"dst is not device memory"),
    ]
    # a destination too close to the end of its allocation (torch's segment
    # holding the tensor, one hipMalloc): 256 bytes short of the state
    state = q * W.n_sites(shape) * 4
    seg = [g for g in torch.cuda.memory_snapshot()
           if g["address"] <= base < g["address"] + g["total_size"]]
    assert len(seg) == 1, "the tensor's segment is not in torch's memory snapshot"
    end = seg[0]["address"] + seg[0]["total_size"]
    short = (end - state + 255) // 256 * 256 + 256
    assert base + half <= short < end and end - short < state
    cases.append(((base, short, 0, 64, 10), b"dst: "))
    for (src, dst, step, block, grid), msg in cases:
        rc = lib.cmf_step_noalloc(ctypes.byref(d), ctypes.c_void_p(src), ctypes.c_void_p(dst), step,
                                  block, grid, None, None)
        assert rc == _lib.CMF_EINVAL and msg in lib.cmf_last_error(), (msg, lib.cmf_last_error())
    rc = lib.cmf_step_noalloc(ctypes.byref(d), ctypes.c_void_p(base), ctypes.c_void_p(base + half), 0,
                              64, 10, ctypes.c_void_p(hbase), None)
    assert rc == _lib.CMF_EINVAL and b"stats_dev is not device memory" in lib.cmf_last_error()
    torch.cuda.synchronize()
    assert not t.any().item()  # nothing was launched
