"""In-place (AA) streaming against the two-buffer pull step: the same
arithmetic in another storage order, so every population, every statistics
row and every derived quantity must agree bit for bit, on every lattice,
storage type and rate set, after even and odd step counts (the state sits in
the natural or in the swapped slot order), through direct launches and
captured graphs.  One run is also compared with the FP64 oracle directly.
Streaming, eq. (streaming); the step is the fused collide-and-stream of the
paper's algorithm.  Needs an MI355X."""
import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import Lattice, _lib, rate_vector
from paper_2602_16486_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


def _state(q, shape, seed, rho0=1.0):
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, seed, rho0=rho0, umax=0.04, dims=2 if q == 9 else 3)
    return O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, seed + 1, 1e-3)


# ragged rows (plain accesses) and rows of whole cache lines in every
# storage type (the non-temporal accesses)
SHAPES = {9: [(37, 29), (128, 24)], 19: [(20, 18, 16), (64, 10, 6)], 27: [(20, 18, 16), (64, 10, 6)]}
CASES = [(q, shape, storage, rates)
         for q in (9, 19, 27) for shape in SHAPES[q]
         for storage in ("f64", "f32", "f16", "bf16") for rates in ("paper", "single")]


def _pair(q, shape, storage, rates, steps, flags=0, seed=11):
    f = _state(q, shape, seed)
    lam = None if rates == "paper" else rate_vector(q, 0.62, "single")
    out = []
    for in_place in (False, True):
        with Lattice(q, shape, storage=storage, tau=0.62, kT=2e-5, lam=lam, seed=seed, flags=flags,
                     in_place=in_place) as lat:
            lat.set_populations(f)
            lat.step(steps)
            out.append((lat.get_populations(), lat.stats()))
    return out


@pytest.mark.parametrize("q,shape,storage,rates", CASES)
def test_in_place_equals_pull_bit_for_bit(q, shape, storage, rates):
    # 7 steps: direct launches, the state ends in the swapped order; 40: one
    # captured 32-step graph plus 8 direct steps, natural order
    for steps in (7, 40):
        (f_ab, st_ab), (f_aa, st_aa) = _pair(q, shape, storage, rates, steps)
        assert np.array_equal(f_ab, f_aa), f"{steps} steps: populations differ"
        assert np.array_equal(st_ab, st_aa), f"{steps} steps: statistics differ"


@pytest.mark.parametrize("q,shape", [(9, (37, 29)), (27, (20, 18, 16))])
def test_in_place_direct_launches_equal_graphs(q, shape):
    (f_ab, st_ab), _ = _pair(q, shape, "f32", "paper", 33)
    _, (f_aa, st_aa) = _pair(q, shape, "f32", "paper", 33, flags=_lib.FLAG_NO_GRAPH)
    assert np.array_equal(f_ab, f_aa)
    assert np.array_equal(st_ab, st_aa)


@pytest.mark.parametrize("q,shape", [(9, (37, 29)), (19, (20, 18, 16)), (27, (20, 18, 16))])
def test_in_place_state_access_in_both_slot_orders(q, shape):
    """Set and read the state, the macroscopic fields, sampled sites and the
    velocity statistics after an odd and an even number of steps: the
    in-place lattice reports what the pull lattice reports."""
    f0, f1 = _state(q, shape, 21), _state(q, shape, 23)
    sites = np.array([0, 1, W.n_sites(shape) // 2, W.n_sites(shape) - 1])
    for steps in (3, 4):
        res = []
        for in_place in (False, True):
            with Lattice(q, shape, storage="f32", tau=0.7, kT=1e-5, seed=5, in_place=in_place) as lat:
                lat.set_populations(f0)
                lat.step(steps)
                a = lat.get_populations()
                lat.set_populations(f1)  # written in the current slot order
                b = lat.get_populations()
                rho, u = lat.macroscopic()
                g = lat.gather_sites(sites)
                mom, counts = lat.velocity_pdf(nbins=16, xmax=4.0)
                lat.step(5)
                c = lat.get_populations()
                res.append((a, b, rho, u, g, mom, counts, c, lat.stats()))
        for x, y in zip(*res):
            assert np.array_equal(x, y)


def test_in_place_run_matches_oracle():
    q, shape, steps = 27, (12, 10, 8), 9
    f = _state(q, shape, 31)
    with Lattice(q, shape, storage="f64", tau=0.7, kT=1e-4, seed=7, replica=3, in_place=True) as lat:
        lat.set_populations(f)
        lat.step(steps)
        got = lat.get_populations()
    ref = f.copy()
    O.run(q, shape, ref, 1e-4, O.paper_lambda(q, 1 / 0.7), 7, 3, 0, steps)
    _, w = O.lattice(q)
    assert np.abs(got - ref).max() / np.abs(ref - w[:, None]).max() < 1e-12


def test_in_place_at_benchmark_size_sampled():
    """D3Q27 256^3 FP32 in the benchmark's launch shape (one workgroup of
    256 per row tile): 3 steps in place and pulled agree bit for bit on
    sampled sites."""
    q, shape = 27, (256, 256, 256)
    rng = np.random.default_rng(3)
    sites = np.sort(rng.choice(W.n_sites(shape), 4096, replace=False))
    sites[:2] = [0, W.n_sites(shape) - 1]
    got = []
    for in_place in (False, True):
        with Lattice(q, shape, storage="f32", tau=0.8, kT=1e-4, seed=1, in_place=in_place) as lat:
            lat.set_launch(256, 65536)
            lat.step(3)
            got.append((lat.gather_sites(sites), lat.stats()))
    assert np.array_equal(got[0][0], got[1][0])
    assert np.array_equal(got[0][1], got[1][1])
    assert np.abs(got[0][0] - O.lattice(q)[1][None, :]).max() > 0  # noise moved the state


def test_in_place_external_buffer_is_half_the_size():
    import torch
    from paper_2602_16486_amd import external_bytes
    q, shape = 19, (24, 20, 18)
    n = W.n_sites(shape)
    one = (q * n * 4 + 255) // 256 * 256
    assert external_bytes(q, shape, "f32") == 2 * one
    assert external_bytes(q, shape, "f32", in_place=True) == one
    f = _state(q, shape, 41)
    t = torch.zeros(one + 256, dtype=torch.uint8, device="cuda")
    base = (t.data_ptr() + 255) // 256 * 256
    torch.cuda.synchronize()
    out = []
    for kw in ({}, {"in_place": True, "external": (base, one)}):
        with Lattice(q, shape, storage="f32", tau=0.7, kT=1e-4, seed=43, **kw) as lat:
            lat.set_populations(f)
            lat.step(37)
            out.append((lat.get_populations(), lat.stats()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    with pytest.raises(_lib.CmfError):
        Lattice(q, shape, storage="f32", in_place=True, external=(base, one - 256))


def test_in_place_autotune_and_resume_keep_the_trajectory():
    """Autotuning from the swapped slot order restores that state, and a run
    saved and resumed (populations, step index) continues it: the
    populations equal the pull lattice's bit for bit (they do not depend on
    the launch shape)."""
    q, shape = 27, (24, 20, 18)
    f0 = _state(q, shape, 61)
    res = []
    for in_place in (False, True):
        kw = dict(storage="f32", tau=0.7, kT=1e-4, seed=9, in_place=in_place)
        with Lattice(q, shape, **kw) as lat:
            lat.set_populations(f0)
            lat.step(3)
            lat.autotune(steps_per_trial=3)
            assert lat.step_index == 3
            lat.step(6)
            saved, at = lat.get_populations(), lat.step_index
        with Lattice(q, shape, **kw) as lat:
            lat.set_populations(saved)
            lat.step_index = at
            lat.step(35)
            res.append((saved, lat.get_populations()))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("q,shape", [(9, (70, 40)), (19, (40, 12, 10)), (27, (40, 12, 10))])
@pytest.mark.parametrize("block,grid", [(64, 4), (128, 1 << 20), (256, 33)])
def test_in_place_equals_pull_in_every_launch_shape(q, shape, block, grid):
    """Persistent grids (workgroups striding over the row tiles) and one
    workgroup per tile, with row tiles shorter than and as long as a row."""
    f = _state(q, shape, 71)
    out = []
    for in_place in (False, True):
        with Lattice(q, shape, storage="f32", tau=0.66, kT=5e-5, seed=4, in_place=in_place) as lat:
            lat.set_launch(block, grid)
            lat.set_populations(f)
            lat.step(9)
            out.append((lat.get_populations(), lat.stats()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
