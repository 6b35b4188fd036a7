"""Test 6 of Sec. 3 (relaxation-time sweep) on the GPU: D2Q9 from rest,
kT = 1/3000, rho0 = 1, over the paper's tau list, with the paper's rates
(the central-moment scheme) and with one rate for every mode (Lambda =
omega I, the single-rate operator of the special cases closing Sec. 2.3,
taken as the fluctuating BGK of the comparison).  The paper's claim: the
central-moment scheme stays finite with psi small at every tau down to 0.5,
while BGK breaks down, with non-finite statistics, as tau -> 0.5.

Box 64 x 64, 20000 steps, psi over the second half (FP32 storage, the
default path).  The band for psi at each tau is

    100 (9 kT / rho0 + 1 / N) + 5 s_b,

the nonlinear shift of <u^2> = <(j / rho)^2> above kT / rho0 (at most
9 kT / rho0 on D2Q9, the coefficient measured on this lattice, Tests 3-5),
the finite-size deficit 1 / N of a box with zero total momentum, and five
standard errors of the window mean, estimated from 10 batch means (at least
0.04 %).  Near tau = 0.5 the GPU statistics are also compared with the FP64
oracle's on the same run.  Needs an MI355X."""
import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import Lattice, _lib, rate_vector
from paper_2602_16486_amd import stats as S

pytestmark = pytest.mark.gpu

TAUS = (0.5, 0.5001, 0.5005, 0.501, 0.505, 0.51, 0.55, 0.7, 1.0, 1.5, 2.0, 5.0, 10.0, 50.0, 100.0)
SHAPE, STEPS, KT, RHO0, SEED = (64, 64), 20000, 1.0 / 3000, 1.0, 1
N = SHAPE[0] * SHAPE[1]
# single rate: the taus at which the runs go non-finite within STEPS steps
SINGLE_BREAKS = (0.5001, 0.5005, 0.501, 0.505)


@pytest.fixture(scope="module", autouse=True)
def _gpu_present():
    assert _lib.device_count() > 0, "no HIP device visible: the gpu tests need an MI355X"


def _run(tau, kind, storage="f32", steps=STEPS):
    with Lattice(9, SHAPE, storage=storage, rho0=RHO0, tau=tau, kT=KT, lam=rate_vector(9, tau, kind),
                 seed=SEED, series_capacity=steps) as lat:
        lat.step(steps)
        return lat.stats(raise_nonfinite=False)


def _psi_and_band(st):
    w0 = STEPS // 2
    psi = S.equipartition(st, N, KT, RHO0, 2, start=w0)["psi_percent"]
    e = st[w0:, 8:10].sum(axis=1) / (2 * N) / (KT / RHO0)
    sd = float(e.reshape(10, -1).mean(axis=1).std(ddof=1) / np.sqrt(10)) * 100
    band = 100 * (9 * KT / RHO0 + 1.0 / N) + 5 * max(sd, 0.008)
    return psi, band


@pytest.fixture(scope="module")
def sweep():
    out = {}
    for kind in ("paper", "single"):
        for tau in TAUS:
            out[(kind, tau)] = _run(tau, kind)
    return out


@pytest.mark.parametrize("tau", TAUS)
def test_central_moments_finite_and_psi_small(sweep, tau):
    st = sweep[("paper", tau)]
    assert np.array_equal(st[:, 0], np.arange(STEPS))
    assert not np.any(st[:, 11]), "non-finite statistics"
    psi, band = _psi_and_band(st)
    print(f"CM tau={tau}: psi {psi:.3f} % (band {band:.3f} %)")
    assert psi < band


@pytest.mark.parametrize("tau", TAUS)
def test_single_rate_breaks_down_near_tau_half(sweep, tau):
    st = sweep[("single", tau)]
    bad = np.nonzero(st[:, 11])[0]
    if tau == 0.5:
        # Lambda_v (2 - Lambda_v) = 0 for every mode: no noise, the rest
        # state stays exactly at rest, psi = 100 %
        assert bad.size == 0
        assert not np.any(st[:, 2:11])
        assert S.equipartition(st, N, KT, RHO0, 2, start=STEPS // 2)["psi_percent"] == 100.0
    elif tau in SINGLE_BREAKS:
        assert bad.size > 0, "expected the single-rate run to go non-finite"
        print(f"single rate tau={tau}: first non-finite step {bad[0]}")
        # once non-finite, every later step is
        assert np.all(st[bad[0]:, 11] > 0)
    else:
        assert bad.size == 0
        psi, band = _psi_and_band(st)
        print(f"single rate tau={tau}: psi {psi:.3f} % (band {band:.3f} %)")
        if tau >= 0.55:
            assert psi < band


def test_single_rate_error_grows_towards_tau_half(sweep):
    """At tau = 0.51, the smallest tau at which both schemes stay finite
    here, the single-rate psi is several times the central-moment one (the
    sharp increase of the BGK error as tau -> 0.5)."""
    psi_cm, _ = _psi_and_band(sweep[("paper", 0.51)])
    psi_single, band = _psi_and_band(sweep[("single", 0.51)])
    print(f"tau=0.51: psi CM {psi_cm:.3f} %, single rate {psi_single:.3f} %")
    assert psi_single > 3 * psi_cm and psi_single > band


@pytest.mark.parametrize("tau,kind", [(0.5, "paper"), (0.5001, "paper"), (0.5005, "paper"),
                                      (0.5001, "single"), (0.5005, "single"), (0.501, "single")])
def test_limit_runs_match_oracle(tau, kind):
    """The first 1000 steps in FP64 (GPU F64 storage) against the oracle:
    per-step velocity moments to FP64 rounding while finite, and the
    single-rate breakdown at the same step."""
    steps = 1000
    st = _run(tau, kind, storage="f64", steps=steps)
    f = O.init_equilibrium(9, N, rho0=RHO0)
    ref = O.run(9, SHAPE, f, KT, rate_vector(9, tau, kind), SEED, 0, 0, steps)
    bad, bad_ref = np.nonzero(st[:, 11])[0], np.nonzero(ref[:, 11])[0]
    assert (bad.size > 0) == (bad_ref.size > 0)
    if bad.size:
        print(f"{kind} tau={tau}: first non-finite step GPU {bad[0]}, oracle {bad_ref[0]}")
        assert bad[0] == bad_ref[0]
        # compare the steps well before the blow-up (growth amplifies the
        # rounding differences once the state departs from equilibrium)
        ok = np.arange(bad[0] // 2)
    else:
        ok = np.arange(steps)
    assert np.allclose(st[ok, 8:10], ref[ok, 8:10], rtol=1e-9, atol=1e-300)
    assert np.allclose(st[ok, 1], ref[ok, 1], rtol=1e-13)
