"""Pins of the oracle's D3Q19 lattice (Sec. 2.4) against the printed
constants, the printed equilibrium (and the reading taken where it fails),
the printed noise prefactors, closed-form properties, and the dynamics."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import paper_printed as PP
from paper_2602_16486_amd import workloads as W

CS2 = 1.0 / 3.0


def _frac(s):
    return float(Fraction(s))


def test_velocities_and_weights(paper):
    g = paper["d3q19"]
    c, w = O.lattice(19)
    c27, _ = O.lattice(27)
    # the set of Sec. 2.4, in the D3Q27 order without the corners
    keep = [i for i in range(27) if (c27[i] ** 2).sum() <= 2]
    assert np.array_equal(c, c27[keep])
    assert len({tuple(x) for x in c}) == 19
    for i in range(19):
        assert w[i] == pytest.approx(_frac(g["w_by_norm2"][str(int((c[i] ** 2).sum()))]), abs=1e-16)
    # isotropy up to fourth order (c_s^2 = 1/3)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    second = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(second, CS2 * np.eye(3), atol=1e-15)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(fourth, iso, atol=1e-15)


def test_basis_is_orthogonal_with_the_printed_norms(paper):
    M = O.transform(19)
    _, w = O.lattice(19)
    G = (M * w) @ M.T
    b = np.array([_frac(x) for x in paper["d3q19"]["b"]])
    assert np.allclose(G, np.diag(b), atol=1e-14)
    assert np.allclose(O.norms(19), b, atol=1e-15)


def test_paper_rates():
    lam = O.paper_lambda(19, 1.3)
    assert np.array_equal(lam, np.where(np.isin(np.arange(19), [7, 8, 9]), 1.3, 1.0))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_reading(seed):
    """k_eq = (rho, 0, ..., 0) (stated in Sec. 2.4) fixes f_eq = T(u)^-1 rho e_0.
    It equals the printed rest and face-diagonal populations, and differs from
    the printed axis populations by
    -rho [9 u_a^2 (u_b^2 + u_g^2) + 6 (u_b^4 + u_b^2 u_g^2 + u_g^4) - (u_b^2 + u_g^2)] / 6
    (a = the axis, b, g the other two), which is what restores mass
    conservation.  Second moments are those of Navier-Stokes to all orders."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.uniform(-1, 1)
    u = 0.08 * rng.uniform(-1, 1, 3)
    c, _ = O.lattice(19)
    f = O.equilibrium(19, rho, u)
    T = O.transform(19, u)
    assert np.allclose(T @ f, rho * np.eye(19)[0], atol=1e-15)
    assert f.sum() == pytest.approx(rho, abs=1e-15)
    assert np.allclose(c.T @ f, rho * u, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", f, c, c), rho * (np.outer(u, u) + CS2 * np.eye(3)), atol=1e-15)
    fp = PP.d3q19_printed_feq(rho, u, c)
    for i in range(19):
        nz = [a for a in range(3) if c[i][a] != 0]
        if len(nz) != 1:
            assert f[i] == pytest.approx(fp[i], abs=1e-15), i
        else:
            a = nz[0]
            ob = [x for x in range(3) if x != a]
            ub2, ug2 = u[ob[0]] ** 2, u[ob[1]] ** 2
            diff = -rho * (9 * u[a] ** 2 * (ub2 + ug2) + 6 * (ub2 ** 2 + ub2 * ug2 + ug2 ** 2) - (ub2 + ug2)) / 6
            assert f[i] - fp[i] == pytest.approx(diff, abs=1e-15), i
    # the printed form loses mass at second order
    assert abs(fp.sum() - rho) > 1e-4


def test_noise_prefactors_match_the_printed_post_collision_moments(paper):
    """At an equilibrium pre-collision state k = (rho, 0, ..., 0), so
    k*_v = phi_v eta_v for every noisy mode: compare with the printed k*."""
    rng = np.random.default_rng(7)
    rho, kT, omega = 1.05, 2e-4, 1.0 / 0.7
    u = 0.03 * rng.uniform(-1, 1, 3)
    f = O.equilibrium(19, rho, u)
    eta = rng.normal(size=19)
    lam = O.paper_lambda(19, omega)
    out = O.collide_site(19, f, eta, kT, lam)
    kstar = out["kstar"]
    env = {"rho": rho, "kT": kT, "cs": math.sqrt(CS2), "omega": omega, "sqrt": math.sqrt}
    assert kstar[0] == pytest.approx(rho, abs=1e-15)
    assert np.allclose(kstar[1:4], 0.0, atol=1e-15)
    for v, expr in paper["d3q19"]["prefactors"].items():
        v = int(v)
        assert kstar[v] == pytest.approx(eval(expr, {}, env) * eta[v], rel=1e-12, abs=1e-17), v


def test_second_reconstruction_path_is_rejected():
    f = O.equilibrium(19, 1.0, np.zeros(3))
    with pytest.raises(Exception):
        O.collide_site(19, f, np.zeros(19), 0.0, O.paper_lambda(19, 1.0), method=1)


def test_one_step_against_per_site_collisions_and_roll_streaming():
    """orc_run on D3Q19 = the per-site collision with the same normals,
    followed by periodic pull-equivalent streaming (numpy.roll)."""
    shape = (5, 4, 3)
    n = W.n_sites(shape)
    rho, u = W.random_macro(shape, 4, umax=0.03)
    f = O.init_equilibrium(19, n, rho=rho, u=u) + W.perturbation(19, n, 5, 5e-4)
    lam = O.paper_lambda(19, 1.0 / 0.8)
    c, _ = O.lattice(19)
    fs = np.zeros_like(f)
    for s in range(n):
        eta = O.normals(19, 9, 0, 0, s)
        fs[:, s] = O.collide_site(19, f[:, s].copy(), eta, 1e-4, lam)["fstar"]
    ref = np.zeros_like(f)
    for i in range(19):
        g = fs[i].reshape(shape[2], shape[1], shape[0])
        ref[i] = np.roll(g, shift=(c[i][2], c[i][1], c[i][0]), axis=(0, 1, 2)).ravel()
    g = f.copy()
    O.run(19, shape, g, 1e-4, lam, 9, 0, 0, 1)
    assert np.allclose(g, ref, atol=1e-15)


def test_conservation_and_equipartition():
    """Mass and momentum are conserved; <u_a^2> approaches kT / rho0
    (within the sampling error and the nonlinear shift of u = j / rho)."""
    shape = (8, 8, 8)
    n = W.n_sites(shape)
    kT = 1e-4
    f = O.init_equilibrium(19, n, rho0=1.0)
    st = O.run(19, shape, f, kT, O.paper_lambda(19, 1.0 / 0.8), 3, 0, 0, 1200)
    assert np.ptp(st[:, 1]) < 1e-11
    assert np.abs(st[:, 2:5]).max() < 1e-12
    u2 = st[200:, 8:11].mean(axis=0) / n / kT
    # white-noise std of one snapshot sqrt(2/N); about 20 independent samples
    assert np.all(np.abs(u2 - 1) < 6 * math.sqrt(2 / n) / math.sqrt(20) + 20 * kT)


def _tg_viscosity(tau, lam, n=24, t1=20, t2=80):
    shape = (n, n, 2)
    kappa = 2 * math.pi / n
    u = W.taylor_green(shape, 1e-3)
    f = O.init_equilibrium(19, 2 * n * n, rho0=1.0, u=u)
    c, _ = O.lattice(19)
    amp, done = [], 0
    for t in (t1, t2):
        O.run(19, shape, f, 0.0, lam, seed=0, step0=done, nsteps=t - done)
        done = t
        un = (c.T @ f) / f.sum(axis=0)
        amp.append((un[:2] * u[:2]).sum() / (u[:2] ** 2).sum())
    return math.log(amp[0] / amp[1]) / (2 * kappa ** 2 * (t2 - t1))


def test_taylor_green_viscosity_of_the_rate_readings():
    """As on D3Q27: the printed rates relax the diagonal second-order modes
    (4-6) at 1, so the axis-aligned vortex decays with nu = 1/6 whatever tau;
    with Lambda_4-9 = omega it decays with c_s^2 (tau - 1/2)."""
    for tau in (0.6, 1.2):
        lam = O.paper_lambda(19, 1 / tau)
        assert abs(_tg_viscosity(tau, lam) * 6 - 1) < 0.01
        lam[4:10] = 1 / tau
        assert abs(_tg_viscosity(tau, lam) / ((tau - 0.5) / 3) - 1) < 0.02
