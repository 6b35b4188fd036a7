"""psi of Test 6 (Sec. 3): the absolute relative deviation, in percent, of
the component-averaged spatial velocity variance (1/2)(<u_x^2> + <u_y^2>)
from the equipartition target kT / rho0, with the variances averaged over
the window of recorded steps.  CPU only: pinned on synthetic series whose
psi is known in closed form, and on the oracle's own series against the
definition evaluated from the oracle's populations step by step."""
import numpy as np
import pytest

import oracle as O
from paper_2602_16486_amd import stats as S


def _series(u2x, u2y, n):
    """Statistics rows (cmf_stats columns) whose spatial means of u_x^2 and
    u_y^2 are the given per-step values."""
    t = len(u2x)
    s = np.zeros((t, 12))
    s[:, 0] = np.arange(t)
    s[:, 1] = n
    s[:, 8] = np.asarray(u2x) * n
    s[:, 9] = np.asarray(u2y) * n
    return s


@pytest.mark.parametrize("kT,rho0", [(1 / 3000, 1.0), (1e-4, 0.5), (2e-5, 4.0)])
def test_psi_closed_forms(kT, rho0):
    n, target = 4096, kT / rho0
    ones = np.ones(50)
    # exactly at the target: 0; no fluctuations at all: 100
    assert S.equipartition(_series(target * ones, target * ones, n), n, kT, rho0, 2)["psi_percent"] \
        == pytest.approx(0.0, abs=1e-12)
    assert S.equipartition(_series(0 * ones, 0 * ones, n), n, kT, rho0, 2)["psi_percent"] == 100.0
    # 2 % above or below: 2, whatever the sign
    for f in (1.02, 0.98):
        psi = S.equipartition(_series(f * target * ones, f * target * ones, n), n, kT, rho0, 2)
        assert psi["psi_percent"] == pytest.approx(2.0, rel=1e-12)
    # the components are averaged before the absolute value is taken
    psi = S.equipartition(_series(1.1 * target * ones, 0.9 * target * ones, n), n, kT, rho0, 2)
    assert psi["psi_percent"] == pytest.approx(0.0, abs=1e-12)
    # the time average runs over the window only
    u2 = np.concatenate([np.zeros(25), 1.05 * target * np.ones(25)])
    psi = S.equipartition(_series(u2, u2, n), n, kT, rho0, 2, start=25)
    assert psi["psi_percent"] == pytest.approx(5.0, rel=1e-12)


def test_psi_of_oracle_series_matches_definition():
    """D2Q9 16 x 12 from rest, kT = 1/3000, tau = 0.51 (a Test 6 point):
    psi from the oracle's statistics rows equals psi evaluated from its
    populations, u = sum c f / sum f at every site and step (eq. macro)."""
    q, shape, kT, tau, steps = 9, (16, 12), 1 / 3000, 0.51, 80
    n = shape[0] * shape[1]
    c, _ = O.lattice(q)
    lam = O.paper_lambda(q, 1 / tau)
    f = O.init_equilibrium(q, n, rho0=1.0)
    rows, u2 = [], []
    for t in range(steps):
        rho = f.sum(axis=0)
        u = (c[:, :2].T @ f) / rho
        u2.append((u ** 2).mean(axis=1))
        rows.append(O.run(q, shape, f, kT, lam, 5, 0, t, 1)[0])
    rows, u2 = np.array(rows), np.array(u2)
    assert np.allclose(rows[:, 8:10] / n, u2, rtol=1e-12, atol=1e-20)
    w0 = steps // 2
    psi_def = abs(kT - 0.5 * (u2[w0:, 0].mean() + u2[w0:, 1].mean())) / kT * 100
    psi = S.equipartition(rows, n, kT, 1.0, 2, start=w0)["psi_percent"]
    assert psi == pytest.approx(psi_def, rel=1e-10)
    assert 0.0 < psi_def < 100.0
