"""Structure factor on the GPU (hipFFT path) against the oracle's
plain-definition spectra of the same trajectory, and its equilibrium value.
Needs an MI355X."""
import numpy as np
import pytest

import oracle as O
from oracle import spectra
from paper_2602_16486_amd import Lattice, _lib
from paper_2602_16486_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


@pytest.mark.parametrize("q,shape", [(9, (32, 24)), (19, (12, 10, 8)), (27, (12, 10, 8)), (27, (9, 7, 5))])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_structure_factor_matches_oracle(q, shape, storage):
    kT, tau, seed, nbins = 2e-4, 0.8, 5, 12
    n = W.n_sites(shape)
    f = O.init_equilibrium(q, n, 1.0)
    lam = O.paper_lambda(q, 1 / tau)
    sa = spectra.ShellAverager(shape, nbins)
    with Lattice(q, shape, storage=storage, tau=tau, kT=kT, seed=seed) as lat:
        lat.sk_reset(nbins)
        for k in range(6):
            lat.step(3)
            O.run(q, shape, f, kT, lam, seed, 0, 3 * k, 3)
            lat.sk_accumulate()
            sa.add(spectra.fields(q, shape, f, 1.0))
        got, ns = lat.sk_shells()
    ref = sa.shells()
    assert ns == 6
    assert np.array_equal(got[:, 1], ref[:, 1])
    assert np.allclose(got[:, 0], ref[:, 0], rtol=1e-12)
    # the spectral path is FP32 (fields and FFT) for every storage; FP32
    # storage adds the trajectory's own rounding
    tol = 1e-6 if storage == "f64" else 2e-4
    scale = np.abs(ref[:, 2:]).max(axis=0)
    assert np.all(np.abs(got[:, 2:] - ref[:, 2:]) <= tol * scale + 1e-300)


def test_equilibrium_structure_factor_on_gpu():
    """D2Q9 128^2 (rho0 = 1, tau = 0.8, kT = 1e-4): S_u = kT/rho0 and
    S_rho = 3 rho0 kT at every shell after equilibration."""
    kT = 1e-4
    with Lattice(9, (128, 128), storage="f32", tau=0.8, kT=kT, seed=9) as lat:
        lat.step(2000)
        lat.sk_reset(32)
        for _ in range(400):
            lat.step(5)
            lat.sk_accumulate()
        sh, ns = lat.sk_shells()
    w = sh[:, 1]
    s_u = 0.5 * (sh[:, 3] + sh[:, 4]) / kT
    s_rho = sh[:, 2] / (3 * kT)
    assert abs(np.average(s_u, weights=w) - 1) < 0.01
    assert abs(np.average(s_rho, weights=w) - 1) < 0.01
    big = w >= 300
    assert np.all(np.abs(s_u[big] - 1) < 0.05)
    assert np.all(np.abs(s_rho[big] - 1) < 0.05)
