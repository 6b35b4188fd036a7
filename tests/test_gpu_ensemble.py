"""Batched ensembles on the GPU: every replica of one fused launch evolves as
a standalone lattice with the same descriptor, and one replica is checked
against the FP64 oracle.  Needs an MI355X."""
import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import Ensemble, Lattice, _lib
from paper_2602_16486_amd import workloads as W

pytestmark = pytest.mark.gpu

REPLICAS = [
    {"q": 9, "shape": (37, 23), "kT": 1e-4, "tau": 0.7, "seed": 11, "replica": 0},
    {"q": 27, "shape": (13, 9, 7), "kT": 3e-4, "tau": 0.55, "seed": 12, "replica": 1},
    {"q": 9, "shape": (300, 5), "kT": 1e-5, "tau": 1.9, "seed": 13, "replica": 2, "rho0": 1.3},
    {"q": 27, "shape": (20, 18, 16), "kT": 1e-3, "tau": 0.9, "seed": 14, "replica": 3},
    {"q": 9, "shape": (64, 64), "kT": 0.0, "tau": 0.8, "seed": 15, "replica": 4},
    {"q": 19, "shape": (11, 10, 9), "kT": 2e-4, "tau": 0.65, "seed": 16, "replica": 5},
]


def _state(r, seed):
    q, shape = r["q"], r["shape"]
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, seed, rho0=r.get("rho0", 1.0), umax=0.04, dims=2 if q == 9 else 3)
    return O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, seed + 1, 5e-4)


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16"])
def test_replicas_match_standalone_lattices(storage):
    steps = 40  # one captured 32-step graph + 8 direct steps
    states = [_state(r, 100 + k) for k, r in enumerate(REPLICAS)]
    with Ensemble(REPLICAS, storage=storage) as ens:
        info = ens.info
        assert info["replicas"] == len(REPLICAS)
        assert info["sites"] == sum(W.n_sites(r["shape"]) for r in REPLICAS)
        for k, f in enumerate(states):
            ens.set_populations(k, f)
        ens.step(steps)
        assert ens.step_index == steps
        got = [ens.get_populations(k) for k in range(len(REPLICAS))]
        st = [ens.stats(k) for k in range(len(REPLICAS))]
    for k, r in enumerate(REPLICAS):
        kw = {key: r[key] for key in ("kT", "tau", "seed", "replica") if key in r}
        with Lattice(r["q"], r["shape"], storage=storage, rho0=r.get("rho0", 1.0), **kw) as lat:
            lat.set_populations(states[k])
            lat.step(steps)
            ref = lat.get_populations()
            ref_st = lat.stats()
        assert np.array_equal(got[k], ref), f"replica {k}"
        assert st[k].shape == ref_st.shape
        assert np.array_equal(st[k][:, 0], ref_st[:, 0])
        # FP64 sums of identical per-site values in a different grouping
        assert np.allclose(st[k], ref_st, rtol=1e-12, atol=1e-18), f"replica {k} statistics"


@pytest.mark.parametrize("spt9,spt27", [("1", "3"), ("7", "2")])
def test_tile_lengths_do_not_change_results(monkeypatch, spt9, spt27):
    """Sites per thread of the ensemble tiles (a launch-shape choice) leave
    every population bit-identical."""
    states = [_state(r, 400 + k) for k, r in enumerate(REPLICAS)]
    out = []
    for env in ({}, {"CMF_ENSEMBLE_SPT9": spt9, "CMF_ENSEMBLE_SPT27": spt27}):
        for key in ("CMF_ENSEMBLE_SPT9", "CMF_ENSEMBLE_SPT27"):
            monkeypatch.delenv(key, raising=False)
        for key, val in env.items():
            monkeypatch.setenv(key, val)
        with Ensemble(REPLICAS, storage="f32") as ens:
            for k, f in enumerate(states):
                ens.set_populations(k, f)
            ens.step(9)
            out.append(([ens.get_populations(k) for k in range(len(REPLICAS))],
                        [ens.stats(k) for k in range(len(REPLICAS))], ens.info["tiles"]))
    assert out[0][2] != out[1][2]
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(out[0][1], out[1][1]):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-18)


def test_replica_matches_oracle():
    r = REPLICAS[3]
    f0 = _state(r, 7)
    with Ensemble(REPLICAS, storage="f64") as ens:
        ens.set_populations(3, f0)
        ens.step(6)
        got = ens.get_populations(3)
    f = f0.copy()
    O.run(27, r["shape"], f, r["kT"], O.paper_lambda(27, 1 / r["tau"]), r["seed"], r["replica"], 0, 6)
    _, w = O.lattice(27)
    assert np.abs(got - f).max() / np.abs(f - w[:, None]).max() < 1e-12


def test_graph_replay_equals_direct_launches():
    states = [_state(r, 200 + k) for k, r in enumerate(REPLICAS)]
    out = []
    for flags in (0, _lib.FLAG_NO_GRAPH):
        with Ensemble(REPLICAS, storage="f32", flags=flags) as ens:
            for k, f in enumerate(states):
                ens.set_populations(k, f)
            ens.step(70)
            out.append([ens.get_populations(k) for k in range(len(REPLICAS))] +
                       [ens.stats(k) for k in range(len(REPLICAS))])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_profiled_steps_are_real_steps():
    """cmf_ensemble_profile_steps (statistics reduced after batches of
    steps) advances every replica, its statistics rows and the step counter
    exactly like cmf_ensemble_step."""
    states = [_state(r, 250 + k) for k, r in enumerate(REPLICAS)]
    out = []
    for profiled in (True, False):
        with Ensemble(REPLICAS, storage="f32", flags=0 if profiled else _lib.FLAG_NO_GRAPH) as ens:
            for k, f in enumerate(states):
                ens.set_populations(k, f)
            if profiled:
                ens.step(3)
                assert ens.profile_steps(11) > 0.0
                ens.step(2)
                assert ens.profile_steps(19) > 0.0
            else:
                ens.step(35)
            assert ens.step_index == 35
            out.append([ens.get_populations(k) for k in range(len(REPLICAS))] +
                       [ens.stats(k) for k in range(len(REPLICAS))])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_general_rates_replica_and_rest_replicas():
    """A replica with a non-paper rate vector switches the ensemble to the
    general kernel; the other replicas are unaffected (the general kernel with
    the paper's rates gives the same result up to rounding)."""
    reps = [dict(REPLICAS[1]), dict(REPLICAS[0])]
    reps[0]["lam"] = np.linspace(0.5, 1.9, 27)
    states = [_state(r, 300 + k) for k, r in enumerate(reps)]
    with Ensemble(reps, storage="f64") as ens:
        for k, f in enumerate(states):
            ens.set_populations(k, f)
        ens.step(5)
        got = [ens.get_populations(k) for k in range(2)]
    _, w27 = O.lattice(27)
    f = states[0].copy()
    O.run(27, reps[0]["shape"], f, reps[0]["kT"], reps[0]["lam"], reps[0]["seed"], reps[0]["replica"], 0, 5)
    assert np.abs(got[0] - f).max() / np.abs(f - w27[:, None]).max() < 1e-12
    _, w9 = O.lattice(9)
    g = states[1].copy()
    O.run(9, reps[1]["shape"], g, reps[1]["kT"], O.paper_lambda(9, 1 / reps[1]["tau"]), reps[1]["seed"],
          reps[1]["replica"], 0, 5)
    assert np.abs(got[1] - g).max() / np.abs(g - w9[:, None]).max() < 1e-12


def test_invalid_ensembles_are_rejected():
    with pytest.raises(_lib.CmfError):
        Ensemble([])
    with pytest.raises(_lib.CmfError):
        Ensemble([{"q": 9, "shape": (8, 8, 2)}])


def test_set_tiles_mid_run_keeps_results():
    """Changing the tile shape between steps (cmf_ensemble_set_tiles) leaves
    every population bit-identical to an untouched ensemble."""
    states = [_state(r, 500 + k) for k, r in enumerate(REPLICAS)]
    out = []
    for retile in (False, True):
        with Ensemble(REPLICAS, storage="f32") as ens:
            for k, f in enumerate(states):
                ens.set_populations(k, f)
            ens.step(5)
            if retile:
                tiles0 = ens.info["tiles"]
                ens.set_tiles(5, 3)
                assert ens.tiles == (5, 3)
                assert ens.info["tiles"] != tiles0
            ens.step(37)  # one captured graph, re-captured for the new tiles
            out.append([ens.get_populations(k) for k in range(len(REPLICAS))])
    for k in range(len(REPLICAS)):
        assert np.array_equal(out[0][k], out[1][k]), f"replica {k}"


def test_autotune_restores_state_and_keeps_results():
    states = [_state(r, 600 + k) for k, r in enumerate(REPLICAS)]
    with Ensemble(REPLICAS, storage="f32") as ens:
        for k, f in enumerate(states):
            ens.set_populations(k, f)
        ens.step(3)
        before = [ens.get_populations(k) for k in range(len(REPLICAS))]
        trials = ens.autotune(steps_per_trial=2)
        # D2Q9 and 3-D replicas present: 6 x 6 shapes
        assert len(trials) == 36 and all(t[2] > 0 for t in trials)
        best = min(trials, key=lambda t: t[2])
        assert ens.tiles == best[:2]
        assert ens.step_index == 3
        for k in range(len(REPLICAS)):
            assert np.array_equal(ens.get_populations(k), before[k])
        ens.step(6)
        got = [ens.get_populations(k) for k in range(len(REPLICAS))]
        st = [ens.stats(k) for k in range(len(REPLICAS))]
    with Ensemble(REPLICAS, storage="f32", flags=_lib.FLAG_NO_GRAPH) as ref:
        for k, f in enumerate(states):
            ref.set_populations(k, f)
        ref.step(9)
        for k in range(len(REPLICAS)):
            assert np.array_equal(got[k], ref.get_populations(k)), f"replica {k}"
            ref_st = ref.stats(k)
            assert np.array_equal(st[k][:, 0], np.arange(9))
            assert np.allclose(st[k], ref_st, rtol=1e-12, atol=1e-18), f"replica {k} statistics"


def test_set_tiles_rejects_bad_shapes():
    with Ensemble(REPLICAS[:2], storage="f32") as ens:
        for bad in ((0, 1), (1, 0), (17, 1), (1, 17)):
            with pytest.raises(Exception):
                ens.set_tiles(*bad)
        assert ens.tiles == (3, 1)


def test_autotune_without_statistics():
    """CMF_FLAG_NO_STATS ensembles tune too and keep their state."""
    states = [_state(r, 700 + k) for k, r in enumerate(REPLICAS)]
    with Ensemble(REPLICAS, storage="f32", flags=_lib.FLAG_NO_STATS) as ens:
        for k, f in enumerate(states):
            ens.set_populations(k, f)
        ens.step(2)
        before = [ens.get_populations(k) for k in range(len(REPLICAS))]
        trials = ens.autotune(steps_per_trial=1)
        assert len(trials) == 36
        assert ens.step_index == 2
        for k in range(len(REPLICAS)):
            assert np.array_equal(ens.get_populations(k), before[k])


ALIGNED = [  # every population row a whole number of 128-byte lines in FP32 and FP16
    {"q": 9, "shape": (64, 40), "kT": 1e-4, "tau": 0.7, "seed": 21, "replica": 0},
    {"q": 27, "shape": (64, 9, 7), "kT": 3e-4, "tau": 0.55, "seed": 22, "replica": 1},
    {"q": 19, "shape": (128, 5, 6), "kT": 2e-4, "tau": 0.65, "seed": 23, "replica": 2},
    {"q": 9, "shape": (192, 3), "kT": 0.0, "tau": 0.8, "seed": 24, "replica": 3},
]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_aligned_replicas_match_standalone_lattices(storage):
    """Ensembles whose rows are all whole cache lines take the non-temporal
    store and c_x = 0 load path; replicas still equal standalone lattices."""
    states = [_state(r, 800 + k) for k, r in enumerate(ALIGNED)]
    with Ensemble(ALIGNED, storage=storage) as ens:
        for k, f in enumerate(states):
            ens.set_populations(k, f)
        ens.step(35)
        got = [ens.get_populations(k) for k in range(len(ALIGNED))]
    for k, r in enumerate(ALIGNED):
        kw = {key: r[key] for key in ("kT", "tau", "seed", "replica")}
        with Lattice(r["q"], r["shape"], storage=storage, **kw) as lat:
            lat.set_populations(states[k])
            lat.step(35)
            assert np.array_equal(got[k], lat.get_populations()), f"replica {k}"


def test_invalid_fields_and_cap_leave_the_ensemble_unchanged():
    """cmf_ensemble_init_equilibrium applies cmf_init_equilibrium's checks and
    cmf_ensemble_stats rejects a negative cap; neither changes any replica."""
    import ctypes
    with Ensemble(REPLICAS[:2], storage="f32") as ens:
        ens.step(2)
        before = [ens.get_populations(k) for k in range(2)]
        n = ens.sizes[1]
        u = np.zeros((3, n))
        u[2, n - 1] = np.inf
        with pytest.raises(_lib.CmfError) as exc:
            ens.init_equilibrium(1, u=u)
        assert exc.value.code == _lib.CMF_EINVAL and "not finite" in str(exc.value)
        with pytest.raises(_lib.CmfError) as exc:
            ens.init_equilibrium(0, rho=np.zeros(ens.sizes[0]))
        assert exc.value.code == _lib.CMF_EINVAL
        cnt = ctypes.c_int64(7)
        assert ens._lib.cmf_ensemble_stats(ens._h, 0, None, -1, ctypes.byref(cnt)) == _lib.CMF_EINVAL
        for k in range(2):
            assert np.array_equal(ens.get_populations(k), before[k])
            assert np.array_equal(ens.stats(k)[:, 0], np.arange(2))


def test_degenerate_replicas_match_standalone_lattices():
    """Replicas with edges of 1 and 2 sites (exact divisions by 1 and 2 in the
    tile-to-site mapping, rows shorter than a wave) and one row longer than a
    tile, next to ordinary ones: bit-identical to standalone lattices."""
    reps = [
        {"q": 9, "shape": (1, 7), "kT": 1e-4, "tau": 0.8, "seed": 21},
        {"q": 9, "shape": (5, 1), "kT": 1e-4, "tau": 0.6, "seed": 22},
        {"q": 9, "shape": (1, 1), "kT": 1e-4, "tau": 0.9, "seed": 23},
        {"q": 27, "shape": (1, 3, 2), "kT": 2e-4, "tau": 0.7, "seed": 24},
        {"q": 27, "shape": (2, 1, 1), "kT": 2e-4, "tau": 0.7, "seed": 25},
        {"q": 19, "shape": (1, 1, 4), "kT": 2e-4, "tau": 0.7, "seed": 26},
        {"q": 9, "shape": (1100, 3), "kT": 1e-5, "tau": 1.5, "seed": 27},
        {"q": 27, "shape": (9, 7, 5), "kT": 1e-4, "tau": 0.8, "seed": 28},
    ]
    for k, r in enumerate(reps):
        r["replica"] = k
    steps = 36
    states = [_state(r, 300 + k) for k, r in enumerate(reps)]
    with Ensemble(reps, storage="f32") as ens:
        for k, f in enumerate(states):
            ens.set_populations(k, f)
        ens.step(steps)
        got = [ens.get_populations(k) for k in range(len(reps))]
    for k, r in enumerate(reps):
        kw = {key: r[key] for key in ("kT", "tau", "seed", "replica")}
        with Lattice(r["q"], r["shape"], storage="f32", **kw) as lat:
            lat.set_populations(states[k])
            lat.step(steps)
            assert np.array_equal(got[k], lat.get_populations()), f"replica {k} {r['shape']}"
