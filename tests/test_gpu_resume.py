"""Resuming a run and steps beyond 2^32.  A run saved as (populations, step
index) and restored into a new lattice or ensemble continues exactly as the
uninterrupted run; the noise of steps of 2^32 and beyond (whose Philox
counters carry the high step bits next to the block index) matches the
oracle's, and a run that crosses step 2^32 matches the oracle step by step.
Needs an MI355X."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import Ensemble, Lattice, _lib
from paper_2602_16486_amd import workloads as W

pytestmark = pytest.mark.gpu

BIG = [(1 << 32) - 1, 1 << 32, (1 << 32) + 7, (1 << 44) + 5, (1 << 56) - 1]


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


def _state(q, shape, seed):
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, seed, umax=0.04, dims=2 if q == 9 else 3)
    return O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, seed + 1, 5e-4)


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("step", BIG)
def test_normals_beyond_2_32_match_oracle(q, fp64, step):
    n, site0, seed, replica = 500, 1000, (1 << 36) + 3, 2
    got = _lib.noise_sample(q, seed, replica, step, site0, n, fp64=fp64)
    ref = np.array([O.normals(q, seed, replica, step, site0 + k) for k in range(n)])
    assert np.abs(got - ref).max() < (1e-13 if fp64 else 4e-6)


def test_step_outside_range_is_rejected():
    with Lattice(9, (16, 8), storage="f32", kT=1e-4) as lat:
        for bad in (-1, 1 << 56):
            with pytest.raises(_lib.CmfError) as exc:
                lat.step_index = bad
            assert exc.value.code == _lib.CMF_EINVAL
        assert lat.step_index == 0
    with pytest.raises(_lib.CmfError):
        _lib.noise_sample(9, 1, 0, 1 << 56, 0, 4)


@pytest.mark.parametrize("q,shape", [(9, (40, 24)), (19, (20, 9, 7)), (27, (20, 9, 7))])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_resume_equals_uninterrupted_run(q, shape, storage):
    """Save (populations, step) after 21 steps, restore into a new lattice
    (FP64 round trip of the stored values is exact for these storages) and
    step 45 more: populations and statistics rows equal those of the run
    that was never interrupted."""
    kw = dict(storage=storage, tau=0.7, kT=1e-4, seed=9, replica=1)
    with Lattice(q, shape, **kw) as a:
        a.step(21)
        saved, t = a.get_populations(), a.step_index
        a.stats()
        a.step(45)
        ref, ref_st = a.get_populations(), a.stats()
    with Lattice(q, shape, **kw) as b:
        b.set_populations(saved)
        b.step_index = t
        assert b.step_index == 21 and b.stats().shape == (0, 12)
        b.step(45)
        got, st = b.get_populations(), b.stats()
    assert np.array_equal(got, ref)
    assert np.array_equal(st[:, 0], np.arange(21, 66))
    assert np.allclose(st, ref_st, rtol=1e-13, atol=1e-18)


@pytest.mark.parametrize("q,shape", [(9, (40, 24)), (19, (20, 9, 7)), (27, (20, 9, 7))])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_run_across_step_2_32_matches_oracle(q, shape, storage):
    """Steps 2^32 - 3 ... 2^32 + 2 (direct launches) and 2^32 + 3 ... +34
    (one captured 32-step graph) against the oracle from the same state."""
    t0, steps = (1 << 32) - 3, 38
    f0 = _state(q, shape, 71)
    kT, tau, seed = 2e-4, 0.7, 5
    with Lattice(q, shape, storage=storage, tau=tau, kT=kT, seed=seed) as lat:
        lat.set_populations(f0)
        lat.step_index = t0
        lat.step(6)
        lat.step(32)
        got = lat.get_populations()
        st = lat.stats()
        assert lat.step_index == t0 + steps
    f = f0.copy()
    st_ref = O.run(q, shape, f, kT, O.paper_lambda(q, 1 / tau), seed, 0, t0, steps)
    _, w = O.lattice(q)
    err = np.abs(got - f).max() / np.abs(f - w[:, None]).max()
    tol = 1e-12 if storage == "f64" else 3e-6 * (1 + math.sqrt(steps))
    assert err < tol
    assert np.array_equal(st[:, 0], t0 + np.arange(steps))
    assert np.array_equal(st_ref[:, 0], t0 + np.arange(steps))


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_ensemble_across_step_2_32_matches_standalone(storage):
    reps = [{"q": 9, "shape": (37, 23), "kT": 1e-4, "tau": 0.7, "seed": 11, "replica": 0},
            {"q": 27, "shape": (13, 9, 7), "kT": 3e-4, "tau": 0.55, "seed": 12, "replica": 1},
            {"q": 19, "shape": (11, 10, 9), "kT": 2e-4, "tau": 0.65, "seed": 16, "replica": 5}]
    t0 = (1 << 32) - 2
    states = [_state(r["q"], r["shape"], 80 + k) for k, r in enumerate(reps)]
    with Ensemble(reps, storage=storage) as ens:
        for k, f in enumerate(states):
            ens.set_populations(k, f)
        ens.step_index = t0
        ens.step(36)
        got = [ens.get_populations(k) for k in range(len(reps))]
        st = [ens.stats(k) for k in range(len(reps))]
    for k, r in enumerate(reps):
        kw = {key: r[key] for key in ("kT", "tau", "seed", "replica")}
        with Lattice(r["q"], r["shape"], storage=storage, **kw) as lat:
            lat.set_populations(states[k])
            lat.step_index = t0
            lat.step(36)
            assert np.array_equal(got[k], lat.get_populations()), f"replica {k}"
        assert np.array_equal(st[k][:, 0], t0 + np.arange(36))
