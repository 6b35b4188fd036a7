"""Parity of the HIP path with the FP64 oracle at the parameters of the
paper's density and relaxation-time scans, where the step's arithmetic takes
other branches than at rho0 = 1, tau = 0.8:

* reference density rho0 != 1 (Sec. 3, Test 5, rho0 in {0.5, 1, 2, 4}): the
  step uses rho0 in rho = rho0 + sum d, in both rest-moment shifts of the
  deviation form and, with 16-bit storage, in the storage scales
  s_i = 2^ceil(log2 sqrt(rho0 kT w_i / c_s^2));
* relaxation times at and next to the stability limit (Sec. 3, Test 6,
  tau in {0.5, 0.5001, 0.5005}; tau = 0.5 is omega = 2, where the modes
  relaxed at omega get no noise and flip sign), with the paper's rates and
  with one rate for every mode (Lambda = omega I, the single-rate operator of
  the special cases closing Sec. 2.3).

Fields are compared element by element from random non-equilibrium states,
after one step and after twelve.  Tolerances as in the other parity tests:
FP64 1e-12 of the largest deviation |f - w rho0|; FP32 3e-6 (1 + sqrt(steps))
of it (each stored deviation rounded to 2^-24 of itself per step, kept by the
conserved modes); 16-bit storage is checked step by step, each step within
one rounding of every deviation to the storage format of the oracle's step
from the same stored state.  Needs an MI355X."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import Lattice, _lib, rate_vector
from paper_2602_16486_amd import workloads as W

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def F32_TOL(steps):
    return 3e-6 * (1.0 + math.sqrt(steps))


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


def _state(q, shape, seed, rho0):
    """Random non-equilibrium state around rho0: equilibrium of random
    rho = rho0 (1 + U(-0.02, 0.02)), u = U(-0.04, 0.04), plus population
    perturbations of a tenth of the smallest rest population rho0 w_i."""
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, seed, rho0=rho0, umax=0.04, dims=2 if q == 9 else 3)
    _, w = O.lattice(q)
    return O.init_equilibrium(q, n, rho=rho, u=u) + W.perturbation(q, n, seed + 1, 0.1 * rho0 * w.min())


def _rel_err(got, ref, q, rho0):
    _, w = O.lattice(q)
    return np.abs(got - ref).max() / np.abs(ref - rho0 * w[:, None]).max()


def _rates(q, tau, kind):
    """(rates passed to the library or None for its paper default, rates the
    oracle steps with)."""
    if kind == "paper":
        return None, O.paper_lambda(q, 1.0 / tau)
    if kind == "general":
        lam = np.linspace(0.4, 1.9, q)
        return lam, lam
    lam = rate_vector(q, tau, kind)
    return lam, lam


SHAPES_1 = {9: (300, 7), 19: (37, 5, 6), 27: (37, 5, 6)}   # rows not whole cache lines
SHAPES_12 = {9: (64, 9), 19: (32, 6, 5), 27: (32, 6, 5)}   # rows of whole cache lines


def _gpu_vs_oracle(q, shape, storage, rho0, tau, kT, kind, steps, seed):
    f0 = _state(q, shape, 100 + seed, rho0)
    lam, lam_o = _rates(q, tau, kind)
    with Lattice(q, shape, storage=storage, rho0=rho0, tau=tau, kT=kT, lam=lam, seed=seed,
                 replica=2) as lat:
        lat.set_populations(f0)
        lat.step(steps)
        got = lat.get_populations()
        st = lat.stats()
    f = f0.copy()
    st_ref = O.run(q, shape, f, kT, lam_o, seed, 2, 0, steps)
    return got, f, st, st_ref


# ---- reference density (Test 5) ------------------------------------------

@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("rho0", [0.5, 2.0])
@pytest.mark.parametrize("kind", ["paper", "general"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("steps", [1, 12])
def test_rho0_step_matches_oracle(q, rho0, kind, storage, steps):
    shape = SHAPES_1[q] if steps == 1 else SHAPES_12[q]
    kT = 2e-4
    got, ref, st, st_ref = _gpu_vs_oracle(q, shape, storage, rho0, 0.7, kT, kind, steps, 17)
    tol = F64_TOL if storage == "f64" else F32_TOL(steps)
    err = _rel_err(got, ref, q, rho0)
    print(f"q={q} rho0={rho0} {kind} {storage} {steps} steps: rel err {err:.3e} (tol {tol:.1e})")
    assert err < tol
    # statistics of the pre-collision states: mass to summation order (FP32:
    # the stored deviations' rounding, a random walk over N q T roundings),
    # momentum and velocity moments
    n = W.n_sites(shape)
    assert np.array_equal(st[:, 0], np.arange(steps))
    dev = np.abs(ref - O.lattice(q)[1][:, None] * rho0).max()
    mass_tol = 1e-12 * n * rho0 if storage == "f64" else 6 * math.sqrt(n * q * steps) * 2 ** -24 * dev
    assert np.abs(st[:, 1] - st_ref[:, 1]).max() < mass_tol
    rtol = 1e-10 if storage == "f64" else 30 * F32_TOL(steps)
    assert np.allclose(st[:, 2:11], st_ref[:, 2:11], rtol=rtol, atol=1e-12 * n)


def _raw_storage(q, shape, f, storage, **kw):
    """Set the populations of a lattice whose buffers live in a torch tensor
    and return the 16-bit words of the buffer holding them (uint16, the
    q N elements of that buffer in its own layout)."""
    import torch
    from paper_2602_16486_amd import external_bytes
    nbytes = external_bytes(q, shape, storage)
    t = torch.zeros(nbytes // 2 + 128, dtype=torch.int16, device="cuda")
    base = (t.data_ptr() + 255) // 256 * 256
    torch.cuda.synchronize()
    with Lattice(q, shape, storage=storage, external=(base, nbytes), **kw) as lat:
        lat.set_populations(f)
        lat.synchronize()
        off = (base - t.data_ptr()) // 2
        # a new lattice holds its state in buffer 0, at the start of the memory
        words = t[off: off + q * W.n_sites(shape)].cpu().numpy().view(np.uint16)
    return words


@pytest.mark.parametrize("q,shape", [(9, (64, 6)), (27, (32, 4, 3)), (19, (32, 4, 3))])
@pytest.mark.parametrize("rho0", [0.5, 1.0, 2.0])
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_16bit_storage_scale_follows_rho0(q, shape, rho0, storage):
    """The stored 16-bit word of population i is the deviation f_i - w_i rho0
    divided by s_i = 2^ceil(log2 sigma_i), sigma_i = sqrt(rho0 kT w_i / c_s^2)
    (the documented storage scale), rounded to nearest even.  Read from
    caller-owned buffers in the row-interleaved layout: element
    ((y + ny z) q + slot_i) nx + x, slot_i the rank of population i in the
    order of its velocity (c_z, c_y, c_x) on the 3-D lattices and i on D2Q9,
    holding the value pulled by site x + c_i."""
    import torch
    kT = 1e-4
    n = W.n_sites(shape)
    nx, ny, nz = W.shape3(shape)
    f = _state(q, shape, 61, rho0)
    words = _raw_storage(q, shape, f, storage, rho0=rho0, tau=0.8, kT=kT)
    c, w = O.lattice(q)
    s = 2.0 ** np.ceil(np.log2(np.sqrt(rho0 * kT * w * 3.0)))
    dt = torch.float16 if storage == "f16" else torch.bfloat16
    vals = torch.from_numpy(words.view(np.int16).copy()).view(dt).float().numpy()
    vals = vals.astype(np.float64).reshape(ny * nz, q, nx)  # [row][slot][x]
    pos = (c[:, 0] + 1) + 3 * (c[:, 1] + 1) + 9 * (c[:, 2] + 1)
    slot = np.argsort(np.argsort(pos)) if q != 9 else np.arange(q)
    site = np.arange(n)
    x, y, z = site % nx, (site // nx) % ny, site // (nx * ny)
    got = np.zeros((q, n))
    for i in range(q):
        # the slot read by site s for population i sits at s - c_i
        xs, ys, zs = (x - c[i, 0]) % nx, (y - c[i, 1]) % ny, (z - c[i, 2]) % nz
        got[i] = vals[ys + ny * zs, slot[i], xs] * s[i]
    dev = f - rho0 * w[:, None]
    # FP64 -> FP32 -> 16-bit, both rounding to nearest: within one 16-bit
    # rounding of the scaled deviation (plus FP16 subnormal spacing)
    rel = {"f16": 2 ** -11, "bf16": 2 ** -8}[storage]
    sub = {"f16": 2.0 ** -24, "bf16": 0.0}[storage]
    # (words decoded with another scale miss by a factor of two or more)
    assert np.all(np.abs(got - dev) <= rel * np.abs(dev) * (1 + 2 ** -12) + sub * s[:, None])


def _stepwise_16bit(q, shape, storage, rho0, tau, kT, kind, steps, seed):
    """Step a 16-bit lattice one step at a time; after each step compare with
    the oracle's step from the same stored state.  Returns the worst
    |err| / bound over all steps."""
    f0 = _state(q, shape, 200 + seed, rho0)
    lam, lam_o = _rates(q, tau, kind)
    _, w = O.lattice(q)
    rel = {"f16": 2 ** -11, "bf16": 2 ** -8}[storage]
    worst = 0.0
    with Lattice(q, shape, storage=storage, rho0=rho0, tau=tau, kT=kT, lam=lam, seed=seed) as lat:
        lat.set_populations(f0)
        for t in range(steps):
            pre = lat.get_populations()
            lat.step(1)
            got = lat.get_populations()
            ref = pre.copy()
            O.run(q, shape, ref, kT, lam_o, seed, 0, t, 1)
            dev = np.abs(ref - rho0 * w[:, None])
            e32 = F32_TOL(1) * dev.max()
            bound = rel * (dev + e32) * (1 + 2 ** -8) + e32
            worst = max(worst, float((np.abs(got - ref) / bound).max()))
        assert lat.step_index == steps
    return worst


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("rho0", [0.5, 2.0])
@pytest.mark.parametrize("kind", ["paper", "general"])
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_rho0_16bit_steps_match_oracle(q, rho0, kind, storage):
    worst = _stepwise_16bit(q, SHAPES_12[q], storage, rho0, 0.7, 2e-4, kind, 12, 19)
    print(f"q={q} rho0={rho0} {kind} {storage}: worst |err| / bound over 12 steps {worst:.3f}")
    assert worst <= 1.0


# ---- relaxation times at the stability limit (Test 6) ----------------------

@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("tau", [0.5, 0.5001, 0.5005])
@pytest.mark.parametrize("kind", ["paper", "single"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("steps", [1, 12])
def test_tau_limit_noisy_step_matches_oracle(q, tau, kind, storage, steps):
    shape = SHAPES_1[q] if steps == 1 else SHAPES_12[q]
    got, ref, st, st_ref = _gpu_vs_oracle(q, shape, storage, 1.0, tau, 1.0 / 3000, kind, steps, 23)
    tol = F64_TOL if storage == "f64" else F32_TOL(steps)
    err = _rel_err(got, ref, q, 1.0)
    print(f"q={q} tau={tau} {kind} {storage} {steps} steps: rel err {err:.3e} (tol {tol:.1e})")
    assert err < tol
    assert not np.any(st[:, 11]) and not np.any(st_ref[:, 11])
    rtol = 1e-10 if storage == "f64" else 30 * F32_TOL(steps)
    assert np.allclose(st[:, 5:11], st_ref[:, 5:11], rtol=rtol, atol=1e-12 * W.n_sites(shape))


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("tau", [0.5, 0.501])
@pytest.mark.parametrize("kind", ["paper", "single"])
def test_tau_limit_16bit_steps_match_oracle(q, tau, kind):
    worst = _stepwise_16bit(q, SHAPES_12[q], "f16", 1.0, tau, 1.0 / 3000, kind, 12, 29)
    print(f"q={q} tau={tau} {kind} f16: worst |err| / bound over 12 steps {worst:.3f}")
    assert worst <= 1.0


@pytest.mark.parametrize("q", [9, 19, 27])
def test_single_rate_at_tau_half_draws_no_noise(q):
    """Lambda = omega I at tau = 0.5: Lambda_v (2 - Lambda_v) = 0 for every
    mode, so phi = 0 (eq. phi_general) and a state at rest stays exactly at
    rest however large kT is; the paper's rates at tau = 0.5 keep the noise
    of the modes relaxed at rate 1."""
    shape = SHAPES_12[q]
    _, w = O.lattice(q)
    n = W.n_sites(shape)
    lam = rate_vector(q, 0.5, "single")
    with Lattice(q, shape, storage="f32", tau=0.5, kT=1.0 / 3000, lam=lam, seed=3) as lat:
        lat.step(40)
        assert np.array_equal(lat.get_populations(), np.repeat(w[:, None], n, axis=1))
        assert not np.any(lat.stats()[:, 2:])
    with Lattice(q, shape, storage="f32", tau=0.5, kT=1.0 / 3000, seed=3) as lat:
        lat.step(40)
        st = lat.stats()
    assert st[-1, 8:11].sum() > 0.0
