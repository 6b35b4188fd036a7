"""Deterministic dynamics on the GPU (kT = 0): the Taylor-Green vortex of
Test 2 (Sec. 3) against its closed-form decay and against the FP64 oracle in
both central-moment bases, and the viscosity that each D3Q27 rate reading
gives.  Needs an MI355X."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import Lattice, _lib, rate_vector
from paper_2602_16486_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


def _velocity(q, f):
    c, _ = O.lattice(q)
    return (c.T @ f) / f.sum(axis=0)


def _tg_paper_setting_gpu(n, storage, re=1000.0, u0=1e-3):
    """Test 2 at Re = u0 N_y / nu = 1000 for one convective time N_y / u0,
    on the GPU.  Returns (populations, relative L2 velocity error, steps)."""
    nu = u0 * n / re
    tau = 0.5 + 3.0 * nu
    kappa = 2 * math.pi / n
    steps = int(round(n / u0))
    u = W.taylor_green((n, n), u0)
    with Lattice(9, (n, n), storage=storage, tau=tau, kT=0.0, flags=_lib.FLAG_NO_STATS) as lat:
        lat.init_equilibrium(u=u)
        lat.step(steps)
        f = lat.get_populations()
    un = _velocity(9, f)[:2]
    ua = u[:2] * math.exp(-2 * nu * kappa ** 2 * steps)
    return f, np.linalg.norm(un - ua) / np.linalg.norm(ua), steps


def test_taylor_green_paper_setting_matches_oracle_in_both_bases():
    """GPU (tensor-product transforms, FP64) = oracle with the orthogonal and
    with the non-orthogonal basis, to FP64 rounding accumulated over the run
    (Test 2: the two bases coincide without noise)."""
    n = 16
    f_gpu, err_gpu, steps = _tg_paper_setting_gpu(n, "f64")
    tau = 0.5 + 3.0 * 1e-3 * n / 1000.0
    for basis in (0, 1):
        f = O.init_equilibrium(9, n * n, rho0=1.0, u=W.taylor_green((n, n), 1e-3))
        O.run(9, (n, n), f, 0.0, O.paper_lambda(9, 1 / tau), seed=0, nsteps=steps, basis=basis)
        assert np.abs(f_gpu - f).max() <= steps * 2.0 ** -52 * np.abs(f).max(), f"basis {basis}"
    assert err_gpu < 0.03


def test_taylor_green_second_order_on_gpu():
    """Fig. 1: the L2 error of the decay falls as N^-2 (N = 16, 32, 64),
    FP64 storage."""
    err = [_tg_paper_setting_gpu(n, "f64")[1] for n in (16, 32, 64)]
    for a, b in zip(err, err[1:]):
        assert 1.9 < math.log(a / b, 2) < 2.1, err


def test_taylor_green_fp32_within_rounding_accumulation_of_fp64():
    """FP32 storage on the same runs: each step rounds every stored
    deviation to 2^-24 of itself; on this slowly decaying flow near
    omega = 2 the roundings repeat from step to step and add up linearly,
    so the FP32 velocity stays within q x steps x 2^-24 x max|f - w rho0| of
    the FP64 one (the FP32 floor of long deterministic runs: at N = 64,
    64000 steps, about 5e-4 of u0 is measured)."""
    _, w = O.lattice(9)
    for n in (16, 32, 64):
        f64, _, steps = _tg_paper_setting_gpu(n, "f64")
        f32, _, _ = _tg_paper_setting_gpu(n, "f32")
        bound = 9 * steps * 2.0 ** -24 * np.abs(f64 - w[:, None]).max()
        assert np.abs(_velocity(9, f32) - _velocity(9, f64)).max() <= bound, n


def _tg3_gpu(q, n, tau, kind, storage, t1=20, t2=80):
    shape = (n, n, 2)
    kappa = 2 * math.pi / n
    u = W.taylor_green(shape, 1e-3)
    lam = rate_vector(q, tau, kind)
    amp = []
    with Lattice(q, shape, storage=storage, tau=tau, kT=0.0, lam=lam, flags=_lib.FLAG_NO_STATS) as lat:
        lat.init_equilibrium(u=u)
        done = 0
        for t in (t1, t2):
            lat.step(t - done)
            done = t
            f = lat.get_populations()
            un = _velocity(q, f)
            amp.append((un[:2] * u[:2]).sum() / (u[:2] ** 2).sum())
    return math.log(amp[0] / amp[1]) / (2 * kappa ** 2 * (t2 - t1)), f, lam


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("tau", [0.6, 1.2])
def test_3d_rate_readings_viscosity_on_gpu(q, storage, tau):
    """Literal D3Q27 / D3Q19 rates (Lambda_4-6 = 1): the axis-aligned vortex
    decays with nu = 1/6 for any tau; isotropic rates (Lambda_4-9 = omega,
    general kernel): nu = c_s^2 (tau - 1/2).  FP64 populations equal the
    oracle's."""
    nu_p, f_p, lam_p = _tg3_gpu(q, 24, tau, "paper", storage)
    nu_i, f_i, lam_i = _tg3_gpu(q, 24, tau, "isotropic", storage)
    assert abs(nu_p * 6 - 1) < 0.01
    assert abs(nu_i / ((tau - 0.5) / 3) - 1) < 0.02
    if storage == "f64":
        shape = (24, 24, 2)
        for f_gpu, lam in ((f_p, lam_p), (f_i, lam_i)):
            f = O.init_equilibrium(q, 24 * 24 * 2, rho0=1.0, u=W.taylor_green(shape, 1e-3))
            O.run(q, shape, f, 0.0, lam, seed=0, nsteps=80)
            assert np.abs(f_gpu - f).max() <= 80 * 2.0 ** -52 * np.abs(f).max()
