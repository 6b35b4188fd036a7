"""Pin of the oracle's structure factor: at equilibrium the linearised
invariant measure of the method (independent populations with variance
rho0 kT w_i / c_s^2, Sec. 2.2 'Structural properties') makes every mode
k != 0 carry S_rho = rho0 kT / c_s^2 and S_u = kT / rho0.  CPU only."""
import numpy as np

import oracle as O
from oracle import spectra


def test_equilibrium_structure_factor_is_flat():
    q, shape, kT, rho0 = 9, (32, 32), 1e-4, 1.0
    f = O.init_equilibrium(q, 1024, rho0)
    lam = O.paper_lambda(q, 1 / 0.8)
    O.run(q, shape, f, kT, lam, seed=3, nsteps=300)
    sa = spectra.ShellAverager(shape, 16)
    for k in range(150):
        O.run(q, shape, f, kT, lam, seed=3, step0=300 + 4 * k, nsteps=4)
        sa.add(spectra.fields(q, shape, f, rho0))
    sh = sa.shells()
    w = sh[:, 1]
    s_rho = sh[:, 2] / (3 * rho0 * kT)
    s_u = 0.5 * (sh[:, 3] + sh[:, 4]) / (kT / rho0)
    # mode-weighted means over all shells, and every populated shell
    assert abs(np.average(s_rho, weights=w) - 1) < 0.03
    assert abs(np.average(s_u, weights=w) - 1) < 0.03
    big = w >= 40
    assert np.all(np.abs(s_rho[big] - 1) < 0.12)
    assert np.all(np.abs(s_u[big] - 1) < 0.12)
    assert np.all(sh[:, 5] == 0.0)  # no u_z in 2-D


def test_shells_cover_every_mode_once():
    sa = spectra.ShellAverager((12, 10, 6), 20)
    sh = sa.shells()
    assert sh[:, 1].sum() == 12 * 10 * 6 - 1
