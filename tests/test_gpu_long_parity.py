"""Multi-step field parity on the aligned path: D3Q27 and D3Q19 64^3 (the
256^3 benchmark box scaled down; rows of 64 sites are whole cache lines in
FP32 and FP64, so the step takes the non-temporal stores and the
non-temporal loads of the c_x = 0 rows, as at 256^3) for 500 steps from rest
with the benchmark's parameters (rho0 = 1, tau = 0.8, kT = 1e-4, Philox
seed 1), every population of every site against the FP64 oracle.

Tolerances: FP64 1e-12 of the largest deviation |f - w rho0| (two FP64
algorithms and two libm implementations); FP32 3e-6 (1 + sqrt(steps)) of it
(each stored deviation rounded to 2^-24 of itself per step; the conserved
modes keep what rounding adds, a random walk in the steps).  The per-step
statistics rows are compared as well.  Needs an MI355X."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import Lattice, _lib

pytestmark = pytest.mark.gpu

SHAPE, STEPS, TAU, KT, SEED = (64, 64, 64), 500, 0.8, 1e-4, 1


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


_cache = {}


def _oracle(q):
    if q not in _cache:
        n = SHAPE[0] * SHAPE[1] * SHAPE[2]
        f = O.init_equilibrium(q, n, rho0=1.0)
        st = O.run(q, SHAPE, f, KT, O.paper_lambda(q, 1 / TAU), SEED, 0, 0, STEPS)
        _cache[q] = (f, st)
    return _cache[q]


@pytest.mark.parametrize("q", [27, 19])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_aligned_64cube_500_steps_match_oracle(q, storage):
    f_ref, st_ref = _oracle(q)
    n = f_ref.shape[1]
    with Lattice(q, SHAPE, storage=storage, tau=TAU, kT=KT, seed=SEED) as lat:
        # one workgroup per tile, as the benchmark launches the FP32 step
        lat.set_launch(64, 64 * 64)
        lat.step(STEPS)
        got = lat.get_populations()
        st = lat.stats()
    _, w = O.lattice(q)
    dev = np.abs(f_ref - w[:, None]).max()
    err = np.abs(got - f_ref).max() / dev
    tol = 1e-12 if storage == "f64" else 3e-6 * (1 + math.sqrt(STEPS))
    print(f"D3Q{q} 64^3 {storage}, {STEPS} steps: rel err {err:.3e} (tol {tol:.1e})")
    assert err < tol
    assert np.array_equal(st[:, 0], np.arange(STEPS))
    assert not np.any(st[:, 11])
    # mass: FP64 to the rounding of an N-term sum in another order (at most
    # N 2^-53 of the total mass N rho0); FP32 within the random walk of the
    # stored deviations' rounding, 6 sqrt(N q T) 2^-24 sigma
    sigma = math.sqrt(KT * w[0] * 3)
    mass_tol = n * 2.0 ** -53 * n if storage == "f64" else 6 * math.sqrt(n * q * STEPS) * 2 ** -24 * sigma
    assert np.abs(st[:, 1] - st_ref[:, 1]).max() < mass_tol
    # <u^2> per step: FP32 relative to the per-step value
    u2, u2_ref = st[1:, 8:11], st_ref[1:, 8:11]
    assert np.allclose(u2, u2_ref, rtol=1e-10 if storage == "f64" else 10 * tol, atol=0)
