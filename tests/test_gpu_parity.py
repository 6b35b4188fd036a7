"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle on
identical seeded inputs.  Needs an MI355X.

Tolerances (derivation in the design notes):
  * Philox words: bit-exact.
  * FP64 path (F64 storage): populations within 1e-12 of the oracle, relative
    to the largest deviation |f - w rho0| -- both sides are FP64 and differ
    only in rounding order and libm ulps.
  * FP32 path: normals within 4e-6 absolute; populations within
    F32_TOL(steps) = 3e-6 * (1 + sqrt(steps)) relative to the largest
    deviation: FP32 rounds each deviation to ~6e-8 of itself per operation
    and the conserved modes keep (do not damp) what rounding adds, so the
    error grows like a random walk in the number of steps.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import Lattice, _lib
from paper_2602_16486_amd import workloads as W

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def F32_TOL(steps):
    return 3e-6 * (1.0 + math.sqrt(steps))


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


def _rel_err(f_gpu, f_ref, q):
    _, w = O.lattice(q)
    scale = np.abs(f_ref - w[:, None] * 1.0).max()
    return np.abs(f_gpu - f_ref).max() / max(scale, 1e-300)


def _random_state(q, shape, seed, rho0=1.0, umax=0.05, amp=1e-3):
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, seed, rho0=rho0, umax=umax, dims=2 if q == 9 else 3)
    return O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, seed + 1, amp)


# ---- noise ----------------------------------------------------------------

def test_philox_words_bit_exact():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 1 << 32, (4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 2, 3, 4], [7, 0, 0, 5]]
    for key in [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (12345, 678)]:
        got = _lib.philox_words(ctr, *key)
        ref = np.array([O.philox4x32_10(c, key) for c in ctr])
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("fp64", [False, True])
def test_normals_match_oracle(q, fp64):
    n, site0, step, seed, replica = 3000, 123456, 77, (1 << 40) + 5, 3
    got = _lib.noise_sample(q, seed, replica, step, site0, n, fp64=fp64)
    ref = np.array([O.normals(q, seed, replica, step, site0 + k) for k in range(n)])
    tol = 1e-13 if fp64 else 4e-6
    assert np.abs(got - ref).max() < tol


# ---- state conversion -----------------------------------------------------

@pytest.mark.parametrize("q,shape", [(9, (37, 23)), (19, (11, 9, 7)), (27, (13, 9, 7))])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_init_equilibrium_matches_oracle(q, shape, storage):
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, 5, rho0=1.1, umax=0.1, dims=2 if q == 9 else 3)
    with Lattice(q, shape, storage=storage, rho0=1.1, kT=1e-4) as lat:
        lat.init_equilibrium(rho, u)
        got = lat.get_populations()
        assert lat.step_index == 0
    ref = O.init_equilibrium(q, n, rho=rho, u=u)
    _, w = O.lattice(q)
    err = np.abs(got - ref).max()
    if storage == "f64":
        # two FP64 evaluations of f_eq (Hermite sum; tensor-product inverse
        # transform of the deviation, then w rho0 added back), each of about
        # 30 operations on values no larger than max |f|: within 64 ulps of
        # the largest population
        assert err <= 64 * 2.0 ** -53 * np.abs(ref).max()
    else:
        # one FP32 rounding of each stored deviation f - w rho0
        assert err <= 2.0 ** -24 * np.abs(ref - 1.1 * w[:, None]).max() * (1 + 2 ** -20)


@pytest.mark.parametrize("q,shape", [(9, (300, 5)), (19, (70, 6, 5)), (27, (70, 6, 5))])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_set_get_roundtrip(q, shape, storage):
    f = _random_state(q, shape, 9)
    with Lattice(q, shape, storage=storage, kT=1e-4) as lat:
        lat.set_populations(f)
        got = lat.get_populations()
        sites = W.sample_sites(shape, 50, 3)
        g = lat.gather_sites(sites)
    _, w = O.lattice(q)
    dev = f - w[:, None]
    if storage == "f64":
        assert np.array_equal(got, f)
    else:
        rel = {"f32": 2 ** -24, "f16": 2 ** -11, "bf16": 2 ** -8}[storage]
        # rounding is relative to the deviation, not to f: FP32 then the
        # 16-bit format (at most rel (1 + 2^-13)), plus the FP16 subnormal
        # spacing 2^-24 s_i (s_i <= 2^-6 here)
        assert np.all(np.abs(got - f) <= rel * np.abs(dev) * (1 + 2 ** -12) + 2 ** -30)
    assert np.array_equal(g, got[:, sites].T)


# ---- one step and many steps ---------------------------------------------

@pytest.mark.parametrize("q,shape", [(9, (300, 7)), (19, (300, 4, 3)), (19, (37, 5, 6)), (27, (300, 4, 3)),
                                     (27, (37, 5, 6))])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("general", [False, True])
def test_one_step_matches_oracle(q, shape, storage, general):
    f = _random_state(q, shape, 21)
    kT, tau, seed, replica = 2e-4, 0.7, 99, 4
    lam = None
    if general:
        lam = np.linspace(0.4, 1.9, q)
        lam_o = lam
    else:
        lam_o = O.paper_lambda(q, 1 / tau)
    with Lattice(q, shape, storage=storage, tau=tau, kT=kT, lam=lam, seed=seed,
                 replica=replica) as lat:
        lat.set_populations(f)
        lat.step(1)
        got = lat.get_populations()
        st = lat.stats()
    g = f.copy()
    ref_st = O.run(q, shape, g, kT, lam_o, seed, replica, step0=0, nsteps=1)
    tol = F64_TOL if storage == "f64" else F32_TOL(1)
    assert _rel_err(got, g, q) < tol
    assert st.shape == (1, 12)
    assert st[0, 0] == 0
    n = W.n_sites(shape)
    # statistics of the pre-collision state: exact up to summation order
    assert st[0, 1] == pytest.approx(ref_st[0, 1], rel=1e-13 if storage == "f64" else 1e-9)
    assert np.allclose(st[0, 2:11], ref_st[0, 2:11], rtol=1e-5 if storage == "f32" else 1e-10,
                       atol=1e-12 * n)


@pytest.mark.parametrize("q,shape", [(9, (300, 7)), (19, (37, 5, 6)), (27, (37, 5, 6))])
@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("general", [False, True])
def test_one_step_16bit_matches_oracle(q, shape, storage, general):
    """16-bit storage, one step from the stored (already rounded) state: each
    population is the oracle's within one rounding of its deviation to the
    storage format (relative 2^-11 FP16, 2^-8 BF16) plus the FP32 collision
    error (F32_TOL(1) of the largest deviation)."""
    f = _random_state(q, shape, 23)
    kT, tau, seed = 2e-4, 0.7, 5
    lam = np.linspace(0.4, 1.9, q) if general else None
    lam_o = lam if general else O.paper_lambda(q, 1 / tau)
    with Lattice(q, shape, storage=storage, tau=tau, kT=kT, lam=lam, seed=seed) as lat:
        lat.set_populations(f)
        f0 = lat.get_populations()
        lat.step(1)
        got = lat.get_populations()
    ref = f0.copy()
    O.run(q, shape, ref, kT, lam_o, seed, 0, 0, 1)
    _, w = O.lattice(q)
    dev = np.abs(ref - w[:, None])
    rel = {"f16": 2 ** -11, "bf16": 2 ** -8}[storage]
    bound = rel * (dev + F32_TOL(1) * dev.max()) * (1 + 2 ** -8) + F32_TOL(1) * dev.max()
    excess = (np.abs(got - ref) / bound).max()
    print(f"16-bit one step q={q} {storage} general={general}: worst |err| / bound {excess:.3f}")
    assert excess <= 1.0


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_d2q9_64_prefix_matches_oracle(storage):
    """D2Q9 64x64, rho0 = 1, tau = 0.8, kT = 1e-4, Philox seed 1, from rest:
    the first 200 steps against the oracle, fields and statistics."""
    q, shape, kT, steps = 9, (64, 64), 1e-4, 200
    with Lattice(q, shape, storage=storage, tau=0.8, kT=kT, seed=1) as lat:
        lat.step(steps)
        got = lat.get_populations()
        st = lat.stats()
    f = O.init_equilibrium(q, 4096, rho0=1.0)
    ref = O.run(q, shape, f, kT, O.paper_lambda(q, 1 / 0.8), 1, 0, 0, steps)
    tol = F64_TOL if storage == "f64" else F32_TOL(steps)
    err = _rel_err(got, f, q)
    print(f"D2Q9 64^2 prefix {storage}: rel err {err:.3e} (tol {tol:.1e})")
    assert err < tol
    assert np.array_equal(st[:, 0], np.arange(steps))
    rtol = 1e-10 if storage == "f64" else 50 * F32_TOL(steps)
    assert np.allclose(st[:, 8:10], ref[:, 8:10], rtol=rtol, atol=1e-14)
    # mass: FP64 exact to rounding; FP32 rounds each stored deviation (of
    # size ~sigma = sqrt(rho0 kT w_0 / c_s^2)) to 2^-24 of itself every step,
    # a random walk over N sites, q populations and the steps: bound 6 sigma
    sigma = math.sqrt(kT * (4 / 9) * 3)
    f32_mass = 6 * math.sqrt(4096 * steps * q) * 2 ** -24 * sigma
    assert np.abs(st[:, 1] - ref[:, 1]).max() < (1e-9 if storage == "f64" else f32_mass)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("general", [False, True])
def test_3d_multistep_matches_oracle(q, storage, general):
    shape, kT, steps = (20, 18, 16), 1e-4, 12
    f0 = _random_state(q, shape, 31, umax=0.04)
    lam = np.full(q, 1 / 0.55) if general else None
    lam_o = lam if general else O.paper_lambda(q, 1 / 0.55)
    with Lattice(q, shape, storage=storage, tau=0.55, kT=kT, seed=7, lam=lam) as lat:
        lat.set_populations(f0)
        lat.step(steps)
        got = lat.get_populations()
    f = f0.copy()
    O.run(q, shape, f, kT, lam_o, 7, 0, 0, steps)
    tol = F64_TOL if storage == "f64" else F32_TOL(steps)
    err = _rel_err(got, f, q)
    print(f"d3q{q} {storage} general={general}: rel err {err:.3e} (tol {tol:.1e})")
    assert err < tol


# ---- invariants of the implementation -------------------------------------

@pytest.mark.parametrize("q,shape", [(9, (40, 30)), (19, (12, 10, 8)), (27, (12, 10, 8))])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_zero_noise_rest_state_is_exact(q, shape, storage):
    """Test 1: kT = 0 from rest stays exactly at rest (deviations stay 0)."""
    _, w = O.lattice(q)
    with Lattice(q, shape, storage=storage, kT=0.0) as lat:
        lat.step(40)
        got = lat.get_populations()
        st = lat.stats()
    assert np.array_equal(got, np.repeat(w[:, None], W.n_sites(shape), axis=1))
    assert np.all(st[:, 5:] == 0.0)


def test_graph_replay_equals_direct_launches():
    q, shape = 27, (40, 12, 10)
    f0 = _random_state(q, shape, 41)
    res = []
    for flags in (0, _lib.FLAG_NO_GRAPH):
        with Lattice(q, shape, storage="f32", kT=1e-4, seed=3, flags=flags) as lat:
            lat.set_populations(f0)
            lat.step(70)  # two graph replays + 6 direct steps
            res.append((lat.get_populations(), lat.stats()))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("q", [27, 19, 9])
@pytest.mark.parametrize("block,grid", [(64, 1), (128, 7), (192, 3), (256, 100000)])
def test_results_do_not_depend_on_launch_shape(q, block, grid):
    """Persistent grids and one workgroup per tile (grid >= tiles; for D2Q9
    the variant with per-site statistics) give the same populations, and
    statistics equal up to the FP64 summation order."""
    shape = (150, 7) if q == 9 else (150, 7, 5)
    f0 = _random_state(q, shape, 43)
    with Lattice(q, shape, storage="f32", kT=1e-4, seed=3) as lat:
        lat.set_populations(f0)
        lat.step(5)
        ref = lat.get_populations()
        ref_st = lat.stats()
    with Lattice(q, shape, storage="f32", kT=1e-4, seed=3) as lat:
        lat.set_launch(block, grid)
        assert lat.launch[0] == block
        lat.set_populations(f0)
        lat.step(5)
        got = lat.get_populations()
        st = lat.stats()
    assert np.array_equal(got, ref)
    # statistics agree up to the FP64 summation order
    assert np.allclose(st, ref_st, rtol=1e-12, atol=1e-18)


def test_autotune_restores_state_and_keeps_results():
    q, shape = 27, (200, 16, 12)
    f0 = _random_state(q, shape, 45)
    with Lattice(q, shape, storage="f32", kT=1e-4, seed=3) as lat:
        lat.set_populations(f0)
        lat.step(3)
        ref = lat.get_populations()
        trials = lat.autotune(steps_per_trial=2)
        assert len(trials) >= 4 and all(t[2] > 0 for t in trials)
        best = min(trials, key=lambda t: t[2])
        assert lat.launch == best[:2]
        assert lat.step_index == 3
        assert np.array_equal(lat.get_populations(), ref)
        lat.step(4)
        got = lat.get_populations()
        st = lat.stats()
    with Lattice(q, shape, storage="f32", kT=1e-4, seed=3, flags=_lib.FLAG_NO_GRAPH) as lat:
        lat.set_populations(f0)
        lat.step(7)
        assert np.array_equal(lat.get_populations(), got)
        st2 = lat.stats()
    assert np.array_equal(st[:, 0], np.arange(7))
    assert np.allclose(st, st2, rtol=1e-12, atol=1e-18)


def test_nonfinite_is_reported():
    """A thermal energy far beyond the low-Mach regime drives rho negative;
    the statistics report non-finite sites and cmf_stats returns
    CMF_ENONFINITE."""
    with Lattice(9, (16, 16), storage="f32", kT=50.0, seed=2) as lat:
        lat.step(20)
        with pytest.raises(_lib.CmfError) as exc:
            lat.stats()
        assert exc.value.code == _lib.CMF_ENONFINITE


def test_tune_cache_file_round_trip(tmp_path):
    """CMFLB_TUNE_CACHE: an autotuned launch shape is appended to the file
    and a later process creating the same lattice starts with it; a file
    with malformed lines is read up to the first bad line, lines with a
    launch shape outside the supported ones (block 64/128/192/256, grid >= 1)
    are skipped, and neither fails a creation."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    code = ("import sys, json; sys.path.insert(0, %r)\n"
            "from paper_2602_16486_amd import Lattice\n"
            "with Lattice(27, (40, 12, 10), storage='f32', kT=1e-4) as lat:\n"
            "    first = list(lat.launch)\n"
            "    if sys.argv[1] == 'tune':\n"
            "        lat.autotune(steps_per_trial=2)\n"
            "    print(json.dumps([first, list(lat.launch)]))\n" % root)
    env = dict(os.environ, CMFLB_TUNE_CACHE=str(cache))

    def run(mode):
        out = subprocess.run([sys.executable, "-c", code, mode], env=env, capture_output=True,
                             text=True, timeout=120)
        assert out.returncode == 0, out.stderr[-2000:]
        return json.loads(out.stdout.strip().splitlines()[-1])

    _, tuned = run("tune")
    lines = cache.read_text().split("\n")
    assert any(line.startswith("dev") and line.split()[1:3] == [str(v) for v in tuned] for line in lines)
    first, _ = run("plain")
    assert first == tuned
    key = next(line.split()[0] for line in lines if line.startswith("dev"))
    cache.write_text("")
    default, _ = run("plain")
    cache.write_text("this is not a cache line\n")
    first, _ = run("plain")
    assert first == default
    # parseable lines with shapes cmf_set_launch rejects are skipped
    cache.write_text(f"{key} 100 7 0.5\n{key} 256 0 0.5\n{key} 512 4 0.5\n")
    first, _ = run("plain")
    assert first == default


@pytest.mark.parametrize("q,shape,in_place", [(27, (40, 12, 10), False), (27, (40, 12, 10), True),
                                              (9, (70, 40), False)])
def test_profiled_steps_are_real_steps(q, shape, in_place):
    """cmf_profile_steps times direct launches with their statistics
    reduced after batches of steps: the state, every statistics row and the
    step counter advance exactly as with cmf_step (runs that end inside a
    batch included)."""
    f0 = _random_state(q, shape, 61)
    kw = dict(storage="f32", kT=1e-4, seed=8, in_place=in_place)
    with Lattice(q, shape, **kw) as lat, Lattice(q, shape, flags=_lib.FLAG_NO_GRAPH, **kw) as ref:
        lat.set_populations(f0)
        ref.set_populations(f0)
        lat.step(3)
        assert lat.profile_steps(11) > 0.0
        lat.step(2)
        assert lat.profile_steps(19) > 0.0
        ref.step(35)
        assert lat.step_index == ref.step_index == 35
        assert np.array_equal(lat.get_populations(), ref.get_populations())
        st, st_ref = lat.stats(), ref.stats()
        assert np.array_equal(st[:, 0], np.arange(35))
        assert np.array_equal(st, st_ref)


@pytest.mark.parametrize("cap", [1, 3, 7])
def test_short_statistics_ring_keeps_the_latest_steps(cap):
    """A statistics ring shorter than the batch of steps whose statistics
    are reduced together keeps the most recent rows, as one reduction per
    step would: direct calls (batches of 8, 8, 4 steps), graph replays and
    profiled steps, read after each call."""
    q, shape = 27, (30, 10, 8)
    f0 = _random_state(q, shape, 91)
    kw = dict(storage="f32", kT=1e-4, seed=4)
    with Lattice(q, shape, series_capacity=cap, **kw) as lat, Lattice(q, shape, **kw) as ref:
        lat.set_populations(f0)
        ref.set_populations(f0)
        for call in ("step 20", "step 37", "profile 11", "step 5"):
            kind, n = call.split()
            for x in (lat, ref):
                if kind == "step":
                    x.step(int(n))
                else:
                    x.profile_steps(int(n))
            got, want = lat.stats(), ref.stats()
            assert len(want) == int(n) and len(got) == min(cap, int(n)), call
            assert np.array_equal(got, want[-cap:]), call


def test_empty_calls_are_no_ops():
    """Zero steps, an empty site list, a statistics read with no new step and
    a zero-step profile change nothing; the next real step is step 0's
    successor as if they had not happened."""
    import ctypes
    shape = (20, 9, 7)
    with Lattice(27, shape, storage="f32", kT=1e-4, seed=6) as lat, \
            Lattice(27, shape, storage="f32", kT=1e-4, seed=6) as ref:
        lat.step(0)
        assert lat.step_index == 0
        assert lat.gather_sites(np.zeros(0, dtype=np.int64)).shape == (0, 27)
        assert lat.stats().shape == (0, 12)
        ms = ctypes.c_double(1.0)
        assert lat._lib.cmf_profile_steps(lat._h, 0, ctypes.byref(ms)) == _lib.CMF_OK and ms.value == 0.0
        lat.step(5)
        ref.step(5)
        assert lat.step_index == 5
        assert np.array_equal(lat.get_populations(), ref.get_populations())
        assert np.array_equal(lat.stats(), ref.stats())


def test_invalid_fields_and_cap_leave_the_lattice_unchanged():
    """cmf_init_equilibrium rejects a non-positive density and a non-finite
    velocity, and cmf_stats a negative cap, with CMF_EINVAL before touching
    the state: populations, step counter and unread statistics survive."""
    import ctypes
    shape = (16, 12)
    n = W.n_sites(shape)
    with Lattice(9, shape, storage="f32", kT=1e-4, seed=4) as lat:
        lat.step(3)
        f = lat.get_populations()
        rho = np.ones(n)
        rho[5] = -1.0
        u = np.zeros((3, n))
        u[1, 7] = np.nan
        for kw, msg in (({"rho": rho}, "positive density"), ({"u": u}, "not finite")):
            with pytest.raises(_lib.CmfError) as exc:
                lat.init_equilibrium(**kw)
            assert exc.value.code == _lib.CMF_EINVAL and msg in str(exc.value)
        cnt = ctypes.c_int64(7)
        assert lat._lib.cmf_stats(lat._h, None, -1, ctypes.byref(cnt)) == _lib.CMF_EINVAL
        assert b"cap < 0" in lat._lib.cmf_last_error()
        assert lat.step_index == 3
        assert np.array_equal(lat.get_populations(), f)
        assert np.array_equal(lat.stats()[:, 0], np.arange(3))


def test_mass_and_momentum_conserved_fp64():
    q, shape = 27, (24, 20, 16)
    f0 = _random_state(q, shape, 47)
    with Lattice(q, shape, storage="f64", kT=1e-3, seed=5) as lat:
        lat.set_populations(f0)
        lat.step(100)
        st = lat.stats()
    assert np.ptp(st[:, 1]) / st[0, 1] < 1e-13
    assert np.abs(st[:, 2:5] - st[0, 2:5]).max() / st[0, 1] < 1e-14


# ---- full size: the bench workload, sampled --------------------------------

@pytest.mark.parametrize("q,shape,storage,grid", [
    (27, (256, 256, 256), "f32", None),    # the benchmark: one workgroup per tile
    (27, (256, 256, 256), "f16", 8192),    # 16-bit variant, persistent grid
    (19, (256, 256, 256), "f32", None),
    (9, (1024, 1024), "f32", None),
    (27, (1024, 1024, 1024), "f32", None),  # largest cube whose two buffers fit (232 GB)
    # z planes of 4 GiB or more: the step's 64-bit-addressed form
    (9, (12288, 10240), "f32", None),       # one 4.5 GB plane
    (27, (6400, 6272, 2), "f32", None),     # 4.3 GB planes
    (27, (9216, 8704, 2), "f16", 8192),
    (19, (8192, 7680, 2), "f32", None),     # 4.8 GB planes
])
def test_full_size_sampled_one_step(q, shape, storage, grid):
    """Full-size lattices in the launch shapes the benchmark times, the
    largest D3Q27 cube that fits (2^30 sites, 116 GB per buffer, element
    offsets beyond 2^32), and boxes whose z planes (Q ny nx values) span
    4 GiB or more, which the step addresses with 64-bit pointers instead of
    32-bit buffer offsets: after 20 steps from rest, one more step is checked
    at sampled sites (random plus every box corner/edge midpoint) against the
    oracle's single-site collision of the gathered pre-collision populations.
    16-bit storage adds one rounding of each deviation to the storage
    format."""
    n_all = int(np.prod(shape))
    need = 2 * q * n_all * {"f32": 4, "f16": 2}[storage]
    if need > 64 << 30:
        import torch
        free, _ = torch.cuda.mem_get_info()
        if free < need + (4 << 30):
            pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")
    kT, tau, seed = 1e-4, 0.8, 1
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) == 3 else 1
    c, _ = O.lattice(q)
    cz = c[:, 2] if q != 9 else np.zeros(q, dtype=int)
    sites = W.sample_sites(shape, 1500, 11)
    n = W.n_sites(shape)
    with Lattice(q, shape, storage=storage, tau=tau, kT=kT, seed=seed) as lat:
        lat.set_launch(256, grid if grid else (nx + 255) // 256 * ny * nz)
        lat.step(20)
        t = lat.step_index
        pre = lat.gather_sites(sites)
        lat.step(1)
        x, y, z = sites % nx, (sites // nx) % ny, sites // (nx * ny)
        dest = np.stack([((x + c[i, 0]) % nx) + nx * (((y + c[i, 1]) % ny) + ny * ((z + cz[i]) % nz))
                         for i in range(q)], axis=1)
        post = lat.gather_sites(dest.ravel()).reshape(len(sites), q, q)
    assert n == nx * ny * nz
    lam = O.paper_lambda(q, 1 / tau)
    _, w = O.lattice(q)
    rel = {"f32": 0.0, "f16": 2 ** -11}[storage]
    worst = 0.0
    for k, s in enumerate(sites):
        eta = O.normals(q, seed, 0, t, int(s))
        fs = O.collide_site(q, pre[k], eta, kT, lam)["fstar"]
        got = np.array([post[k, i, i] for i in range(q)])
        dev = np.abs(fs - w)
        e32 = F32_TOL(1) * dev.max()
        bound = rel * (dev + e32) * (1 + 2 ** -8) + e32
        worst = max(worst, (np.abs(got - fs) / bound).max())
    print(f"{shape} q={q} {storage} sampled one step: worst |err| / bound {worst:.3f}")
    assert worst <= 1.0


@pytest.mark.parametrize("q,shape,storage,grid", [
    (27, (256, 256, 256), "f32", None),    # the benchmark: one workgroup per tile
    (27, (256, 256, 256), "f16", 8192),    # 16-bit variant, persistent grid
    (27, (256, 256, 256), "bf16", 8192),
    (19, (256, 256, 256), "f32", None),
    (19, (256, 256, 256), "f16", 4096),
    (9, (1024, 1024), "f32", None),
])
def test_full_size_rest_state_and_conservation(q, shape, storage, grid):
    """Whole-box properties at full size, in the benchmark's launch shapes,
    over 40 steps (one captured 32-step graph and 8 direct steps): from rest
    with kT = 0 every site stays exactly at rest (the FP64 sums of rho - rho0,
    rho u, u and u^2 are exactly zero); with kT = 1e-4 total mass and momentum
    stay within the random walk of the storage rounding, 6 sqrt(N T q) eps
    sigma with sigma = sqrt(rho0 kT w_0 / c_s^2) and eps = 2^-24 (FP32),
    2^-11 (FP16) or 2^-8 (BF16; relative to the scaled value), since the
    collision conserves both exactly and streaming permutes the populations.
    A systematic error (a drift linear in the steps) exceeds it at once."""
    n = W.n_sites(shape)
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) == 3 else 1
    steps = 40
    launch = (256, grid if grid else (nx + 255) // 256 * ny * nz)
    with Lattice(q, shape, storage=storage, tau=0.8, kT=0.0, seed=1) as lat:
        lat.set_launch(*launch)
        lat.step(steps)
        st = lat.stats()
    assert np.array_equal(st[:, 0], np.arange(steps))
    assert np.all(st[:, 1] == n * 1.0)
    assert not np.any(st[:, 2:])
    kT = 1e-4
    _, w = O.lattice(q)
    sigma = math.sqrt(kT * w[0] * 3)
    eps = {"f32": 2 ** -24, "f16": 2 ** -11, "bf16": 2 ** -8}[storage]
    bound = 6 * math.sqrt(n * steps * q) * eps * sigma
    with Lattice(q, shape, storage=storage, tau=0.8, kT=kT, seed=1) as lat:
        lat.set_launch(*launch)
        lat.step(steps)
        st = lat.stats()
    assert np.array_equal(st[:, 0], np.arange(steps))
    assert not np.any(st[:, 11])
    drift = np.abs(st[:, 1] - n).max()
    mom = np.abs(st[:, 2:5]).max()
    print(f"{shape} q={q} {storage}: mass drift {drift:.2e}, momentum {mom:.2e}, bound {bound:.2e}")
    assert drift < bound and mom < bound
    # and the noise is on: <u^2> has grown to a sizeable part of kT / rho0
    assert st[-1, 8:11].sum() / (3 * n) > 0.1 * kT


@pytest.mark.parametrize("q,shape,storage", [(9, (19, 7), "f64"), (27, (9, 6, 5), "f64"), (27, (9, 6, 5), "f32")])
def test_get_macro_matches_populations(q, shape, storage):
    """cmf_get_macro: rho = sum f and u = sum c f / rho of the pre-collision
    state (eq. macro), in FP64 on the device."""
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, 21, umax=0.04, dims=2 if q == 9 else 3)
    f = O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, 22, 5e-4)
    with Lattice(q, shape, storage=storage, kT=1e-4) as lat:
        lat.set_populations(f)
        lat.step(3)
        g = lat.get_populations()
        r, uu = lat.macroscopic()
    c, _ = O.lattice(q)
    rho_ref = g.sum(axis=0)
    u_ref = (c.T @ g) / rho_ref
    assert np.allclose(r, rho_ref, rtol=1e-14, atol=0)
    assert np.abs(uu - u_ref).max() <= 1e-14


@pytest.mark.parametrize("q,shape,storage,steps", [(9, (40, 30), "f64", 0), (27, (12, 10, 9), "f64", 0),
                                                   (27, (12, 10, 9), "f64", 4), (19, (12, 10, 9), "f64", 4),
                                                   (9, (64, 48), "f32", 0)])
def test_velocity_pdf_matches_oracle(q, shape, storage, steps):
    """cmf_velocity_pdf (Test 7, Fig. 8) against the oracle's plain
    definitions on the same state: moments to FP64 (FP32 storage: to the
    rounding of the stored deviations) and integer counts equal except for
    values within rounding of a bin edge."""
    from oracle import pdf as P
    n = W.n_sites(shape)
    dims = 2 if q == 9 else 3
    rho, u = W.random_macro(shape, 31, umax=0.03, dims=dims)
    f = O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, 32, 5e-4)
    nbins, xmax = 24, 3.0
    with Lattice(q, shape, storage=storage, tau=0.7, kT=1e-4, seed=33) as lat:
        lat.set_populations(f)
        lat.step(steps)
        mom, counts = lat.velocity_pdf(nbins, xmax)
    if steps:
        O.run(q, shape, f, 1e-4, O.paper_lambda(q, 1 / 0.7), 33, 0, 0, steps)
    uref = P.velocity(q, f)
    mref = P.velocity_moments(uref)
    cref, xs = P.velocity_histogram(uref, dims, nbins, xmax)
    tol = 1e-12 if storage == "f64" else 1e-5
    for a in range(dims):
        assert abs(mom[a, 0] - mref[a, 0]) <= tol * np.sqrt(mref[a, 1])
        assert np.allclose(mom[a, 1:], mref[a, 1:], rtol=tol * 10, atol=0)
        edges = np.linspace(-xmax, xmax, nbins + 1)
        near = int(np.sum(np.min(np.abs(xs[a][:, None] - edges[None, :]), axis=1) < 1e3 * tol))
        assert np.abs(counts[a] - cref[a]).sum() <= 2 * near, (a, near)
        assert counts[a].sum() == n
    if dims == 2:
        assert not counts[2].any() and not mom[2].any()


def test_external_buffers_from_torch():
    """cmf_create_external: population buffers in a torch tensor give the
    same populations and statistics as library-owned buffers; bad buffers
    are rejected."""
    import torch
    from paper_2602_16486_amd import external_bytes
    q, shape = 27, (24, 20, 18)
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, 41, umax=0.03)
    f = O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, 42, 5e-4)
    nbytes = external_bytes(q, shape, "f32")
    assert nbytes == 2 * ((q * n * 4 + 255) // 256 * 256)
    t = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = (t.data_ptr() + 255) // 256 * 256
    torch.cuda.synchronize()
    out = []
    for ext in (None, (base, nbytes)):
        with Lattice(q, shape, storage="f32", tau=0.7, kT=1e-4, seed=43, external=ext) as lat:
            lat.set_populations(f)
            lat.step(37)
            out.append((lat.get_populations(), lat.stats()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert t.count_nonzero().item() > 0  # the lattice wrote into the tensor
    for bad in ((base + 64, nbytes), (base, nbytes - 256)):
        with pytest.raises(_lib.CmfError):
            Lattice(q, shape, storage="f32", external=bad)
    host = np.zeros(nbytes, dtype=np.uint8)
    with pytest.raises(_lib.CmfError):
        Lattice(q, shape, storage="f32", external=(host.ctypes.data, nbytes))
    # a claimed size beyond the end of the allocation (torch's segment, one
    # hipMalloc) is refused before the lattice writes its rest state
    end = _segment_end(torch, base)
    near = (end - nbytes + 255) // 256 * 256 + 256
    with pytest.raises(_lib.CmfError, match="to the end of its allocation"):
        Lattice(q, shape, storage="f32", external=(near, nbytes))


def _segment_end(torch, ptr):
    """End address of the torch allocator segment (one hipMalloc) holding ptr."""
    seg = [g for g in torch.cuda.memory_snapshot()
           if g["address"] <= ptr < g["address"] + g["total_size"]]
    assert len(seg) == 1, "the pointer's segment is not in torch's memory snapshot"
    return seg[0]["address"] + seg[0]["total_size"]


@pytest.mark.parametrize("q,shape", [(9, (33, 17)), (19, (20, 12, 9)), (27, (20, 12, 9))])
def test_sample_macro_into_torch_buffers(q, shape):
    """cmf_sample_macro writes rho (N floats) and u (3 N floats, u_x block
    first) of the current state into caller device buffers (torch tensors):
    the FP64 values of cmf_get_macro rounded to FP32, exactly; either buffer
    may be NULL, and nothing beyond the N and 3 N floats is written."""
    import torch
    n = W.n_sites(shape)
    dims = 2 if q == 9 else 3
    rho, u = W.random_macro(shape, 51, umax=0.03, dims=dims)
    f = O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, 52, 5e-4)
    r_t = torch.full((n + 64,), -7.0, dtype=torch.float32, device="cuda")
    u_t = torch.full((3 * n + 64,), -7.0, dtype=torch.float32, device="cuda")
    r2_t = torch.full((n,), -7.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with Lattice(q, shape, storage="f32", tau=0.7, kT=1e-4, seed=53) as lat:
        lat.set_populations(f)
        lat.step(5)
        rho64, u64 = lat.macroscopic()
        lat.sample_macro(r_t.data_ptr(), u_t.data_ptr())
        lat.sample_macro(r2_t.data_ptr(), 0)
        lat.synchronize()
    got_r, got_u = r_t.cpu().numpy(), u_t.cpu().numpy()
    assert np.array_equal(got_r[:n], rho64.astype(np.float32))
    assert np.array_equal(got_u[:3 * n].reshape(3, n), u64.astype(np.float32))
    assert np.all(got_r[n:] == -7.0) and np.all(got_u[3 * n:] == -7.0)
    assert np.array_equal(r2_t.cpu().numpy(), got_r[:n])
    # host memory, or a buffer shorter than N floats before the end of its
    # allocation, is refused before any launch
    host = np.zeros(3 * n, dtype=np.float32)
    short = _segment_end(torch, r2_t.data_ptr()) - 4 * (n - 1)
    with Lattice(q, shape, storage="f32") as lat:
        with pytest.raises(_lib.CmfError, match="rho_dev is not device memory"):
            lat.sample_macro(host.ctypes.data, 0)
        with pytest.raises(_lib.CmfError, match="u_dev is not device memory"):
            lat.sample_macro(0, host.ctypes.data)
        with pytest.raises(_lib.CmfError, match="to the end of its allocation"):
            lat.sample_macro(short, 0)


def test_stream_copy_diagnostic():
    """cmf_stream_copy times a plain copy of the given size and returns the
    fastest of `reps` runs."""
    ms = _lib.stream_copy(64 << 20, reps=3)
    assert 0.0 < ms < 100.0


@pytest.mark.parametrize("q,shape", [(9, (1, 1)), (9, (1, 5)), (9, (7, 1)), (9, (2, 2)),
                                     (27, (1, 1, 1)), (27, (2, 1, 3)), (27, (1, 4, 1)),
                                     (19, (1, 1, 1)), (19, (3, 1, 2))])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_degenerate_boxes_match_oracle(q, shape, storage):
    """Boxes with edges of 1 or 2 sites (every periodic wrap lands on the
    site itself or its single neighbour), 9 steps against the oracle."""
    f0 = _random_state(q, shape, 51)
    kT, tau, seed, steps = 3e-4, 0.7, 13, 9
    with Lattice(q, shape, storage=storage, tau=tau, kT=kT, seed=seed) as lat:
        lat.set_populations(f0)
        lat.step(steps)
        got = lat.get_populations()
        st = lat.stats()
    f = f0.copy()
    ref_st = O.run(q, shape, f, kT, O.paper_lambda(q, 1 / tau), seed, 0, 0, steps)
    tol = F64_TOL if storage == "f64" else F32_TOL(steps)
    assert _rel_err(got, f, q) < tol
    assert np.allclose(st[:, 1], ref_st[:, 1], rtol=1e-12 if storage == "f64" else 1e-7)
