"""Pins of the FP64 oracle against what the paper prints and what the
mathematics fixes (single-site algebra).  CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import paper_printed as P

CS2 = 1.0 / 3.0


def _frac(s):
    return float(Fraction(s))


def _weights_d3q27(paper):
    w = np.zeros(27)
    for lo, hi, val in paper["d3q27"]["w_groups"]:
        w[lo:hi + 1] = _frac(val)
    return w


def _norms_d3q27(paper):
    b = np.zeros(27)
    for lo, hi, val in paper["d3q27"]["b_groups"]:
        b[lo:hi + 1] = _frac(val)
    return b


# ---- lattices, bases, norms (Sec. 2.2, 2.3) -------------------------------

def test_lattices_match_printed(paper):
    c, w = O.lattice(9)
    assert c[:, 0].tolist() == paper["d2q9"]["cx"]
    assert c[:, 1].tolist() == paper["d2q9"]["cy"]
    assert np.allclose(w, [_frac(s) for s in paper["d2q9"]["w"]], rtol=0, atol=1e-16)
    c, w = O.lattice(27)
    assert c[:, 0].tolist() == paper["d3q27"]["cx"]
    assert c[:, 1].tolist() == paper["d3q27"]["cy"]
    assert c[:, 2].tolist() == paper["d3q27"]["cz"]
    assert np.allclose(w, _weights_d3q27(paper), rtol=0, atol=1e-16)
    # 27 distinct velocities covering {-1,0,1}^3
    assert len({tuple(v) for v in c.tolist()}) == 27


def test_norms_match_printed(paper):
    assert np.allclose(O.norms(9), [_frac(s) for s in paper["d2q9"]["b"]], rtol=1e-14, atol=0)
    assert np.allclose(O.norms(27), _norms_d3q27(paper), rtol=1e-14, atol=0)


@pytest.mark.parametrize("q", [9, 27])
def test_weighted_orthogonality(q):
    """sum_i w_i M_vi M_li = b_v delta_vl (Sec. 2.2 'Structural properties')."""
    _, w = O.lattice(q)
    M = O.transform(q)
    G = M @ np.diag(w) @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-15
    assert np.allclose(np.diag(G), O.norms(q), rtol=1e-14)


def test_d3q27_row15_reading():
    """Row 15 as printed, c_y^2 c_z - c_s^2 c_y, is not orthogonal to the other
    rows and has norm 4/27 != printed 2/27; the oracle's reading
    (c_y^2 - c_s^2) c_z is orthogonal with norm 2/27."""
    c, w = O.lattice(27)
    x, y, z = c[:, 0].astype(float), c[:, 1].astype(float), c[:, 2].astype(float)
    literal = y * y * z - CS2 * y
    M = O.transform(27)
    assert abs((w * literal * literal).sum() - 4.0 / 27.0) < 1e-15
    overlaps = np.abs(M @ (w * literal))
    overlaps[15] = 0.0
    assert overlaps.max() > 0.1
    assert abs((w * M[15] * M[15]).sum() - 2.0 / 27.0) < 1e-15


def test_d2q9_transform_is_shifted_basis():
    """T(u) row 5 is (c_x - u_x)(c_y - u_y) and row 8 is the shifted fourth-order
    polynomial (Sec. 2.2: T from M by c -> c - u)."""
    c, _ = O.lattice(9)
    u = np.array([0.07, -0.04])
    T = O.transform(9, u)
    cx, cy = c[:, 0] - u[0], c[:, 1] - u[1]
    assert np.allclose(T[5], cx * cy, atol=1e-15)
    assert np.allclose(T[8], (cx ** 2 - CS2) * (cy ** 2 - CS2), atol=1e-15)
    assert np.allclose(O.transform(9, np.zeros(2)), O.transform(9), atol=0)


# ---- equilibrium (eq. feq, Sec. 2.3) ----------------------------------------

def _psi(cc, u):
    # one-dimensional factor of the D2Q9/D3Q27 full-order equilibrium
    return np.where(cc == 0, 1.0 - CS2 - u * u, 0.5 * (CS2 + u * u + cc * u))


@pytest.mark.parametrize("q", [9, 27])
def test_equilibrium_product_form(q):
    """The maximal-order Hermite equilibrium equals rho * prod_a Psi(c_ia, u_a)."""
    c, w = O.lattice(q)
    rng = np.random.default_rng(11)
    d = 2 if q == 9 else 3
    for _ in range(20):
        rho = rng.uniform(0.5, 2.0)
        u = rng.uniform(-0.3, 0.3, d)
        feq = O.equilibrium(q, rho, u)
        prod = rho * np.prod([_psi(c[:, a], u[a]) for a in range(d)], axis=0)
        assert np.allclose(feq, prod, rtol=1e-14, atol=1e-16)
    # at rest f_eq = w rho (Sec. 3: rest start)
    assert np.allclose(O.equilibrium(q, 1.3, np.zeros(d)), 1.3 * w, rtol=1e-15)


@pytest.mark.parametrize("q", [9, 27])
def test_central_moments_of_equilibrium(q):
    """k_eq = T(u) f_eq = (rho, 0, ..., 0) (Sec. 2.2 and 2.3)."""
    rng = np.random.default_rng(5)
    d = 2 if q == 9 else 3
    for _ in range(10):
        rho, u = rng.uniform(0.5, 2), rng.uniform(-0.2, 0.2, d)
        k = O.transform(q, u) @ O.equilibrium(q, rho, u)
        assert abs(k[0] - rho) < 1e-14
        assert np.abs(k[1:]).max() < 1e-15


def test_second_order_equilibrium_offsets(paper):
    """A second-order equilibrium has the printed non-zero ghost central
    moments (Sec. 2.2, 'Structural properties'); pins T(u) against them."""
    c, w = O.lattice(9)
    rho, ux, uy = 1.2, 0.11, -0.07
    cu = c[:, 0] * ux + c[:, 1] * uy
    feq2 = w * rho * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - (ux ** 2 + uy ** 2) / (2 * CS2))
    k = O.transform(9, [ux, uy]) @ feq2
    expect = [eval(s, {"rho": rho, "ux": ux, "uy": uy}) for s in paper["d2q9"]["second_order_keq"]]
    assert np.allclose(k, expect, atol=1e-15)


def test_compact_d2q9_equilibrium_reading():
    """The compact D2Q9 equilibrium printed without 1/(4 c_s^8) on the
    H_xxyy term leaves k_8 != 0; with the factor (the general Hermite form) it
    vanishes.  The oracle takes the latter."""
    c, w = O.lattice(9)
    rho, ux, uy = 1.0, 0.1, 0.08
    cx, cy = c[:, 0].astype(float), c[:, 1].astype(float)
    cu = cx * ux + cy * uy
    base = (1 + cu / CS2 + ((cx * cx - CS2) * ux * ux + 2 * cx * cy * ux * uy + (cy * cy - CS2) * uy * uy)
            / (2 * CS2 ** 2)
            + ((cx * cx - CS2) * cy * ux * ux * uy + cx * (cy * cy - CS2) * ux * uy * uy) / (2 * CS2 ** 3))
    h4 = (cx * cx - CS2) * (cy * cy - CS2) * ux * ux * uy * uy
    T = O.transform(9, [ux, uy])
    literal = T @ (w * rho * (base + h4))
    general = T @ (w * rho * (base + h4 / (4 * CS2 ** 4)))
    assert abs(literal[8]) > 1e-5
    assert np.abs(general[1:]).max() < 1e-15
    assert np.allclose(w * rho * (base + h4 / (4 * CS2 ** 4)), O.equilibrium(9, rho, [ux, uy]), atol=1e-16)


def test_hermite_tensors_match_printed():
    """H^(2), H^(3), H^(4) of the oracle's recursion equal the printed tensor
    definitions (Sec. 2.2) for every index tuple and velocity."""
    d = lambda a, b: 1.0 if a == b else 0.0
    for cv in [(0, 0, 0), (1, 0, 0), (-1, 1, 0), (1, -1, 1), (0, 1, -1)]:
        cc = np.array(cv, dtype=float)
        for a in range(3):
            for b in range(3):
                assert abs(O.hermite(cc, [a, b]) - (cc[a] * cc[b] - CS2 * d(a, b))) < 1e-15
                for g in range(3):
                    h3 = cc[a] * cc[b] * cc[g] - CS2 * (cc[a] * d(b, g) + cc[b] * d(a, g) + cc[g] * d(a, b))
                    assert abs(O.hermite(cc, [a, b, g]) - h3) < 1e-15
                    for e in range(3):
                        h4 = (cc[a] * cc[b] * cc[g] * cc[e]
                              - CS2 * (cc[a] * cc[b] * d(g, e) + cc[a] * cc[g] * d(b, e) + cc[a] * cc[e] * d(b, g)
                                       + cc[b] * cc[g] * d(a, e) + cc[b] * cc[e] * d(a, g) + cc[g] * cc[e] * d(a, b))
                              + CS2 ** 2 * (d(a, b) * d(g, e) + d(a, g) * d(b, e) + d(a, e) * d(b, g)))
                        assert abs(O.hermite(cc, [a, b, g, e]) - h4) < 1e-15


# ---- collision (eq. cm_collision, eq. phi_general) --------------------------

def _prefactor(expr, rho, kT, omega):
    return eval(expr, {"sqrt": math.sqrt, "rho": rho, "kT": kT, "omega": omega, "cs": math.sqrt(CS2)})


@pytest.mark.parametrize("q,key", [(9, "d2q9"), (27, "d3q27")])
def test_noise_prefactors_match_printed(paper, q, key):
    """phi_v of eq. phi_general with the paper's Lambda equals the printed
    prefactor of every noisy post-collision central moment.  At equilibrium
    (k_v = 0 for v > 0) with eta = 1, k*_v = phi_v."""
    d = 2 if q == 9 else 3
    for rho, kT, omega in [(1.0, 1e-4, 1.25), (0.7, 3e-3, 1.9), (2.0, 1.0 / 3000, 1.0 / 0.55)]:
        u = np.linspace(0.02, 0.05, d)
        f = O.equilibrium(q, rho, u)
        lam = O.paper_lambda(q, omega)
        r = O.collide_site(q, f, np.ones(q), kT, lam)
        first = 3 if q == 9 else 4
        assert np.abs(r["kstar"][1:first]).max() < 1e-15
        assert abs(r["kstar"][0] - rho) < 1e-14
        for v, expr in paper[key]["prefactors"].items():
            v = int(v)
            assert r["kstar"][v] == pytest.approx(_prefactor(expr, rho, kT, omega), rel=1e-12, abs=1e-16)


def test_paper_lambda_matches_printed(paper):
    lam = O.paper_lambda(9, 1.7)
    expect = [1.7 if s == "omega" else float(s) for s in paper["d2q9"]["lambda"]]
    assert lam.tolist() == expect
    lam = O.paper_lambda(27, 1.7)
    assert lam[7:10].tolist() == [1.7] * 3
    assert np.all(np.delete(lam, [7, 8, 9]) == 1.0)


def test_d2q9_collision_matches_printed_equations():
    """Full single-site D2Q9 collision (macro, k4/k5, k*, r*, f*) equals the
    printed explicit equations of Sec. 2.2 at random states."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        u = rng.uniform(-0.15, 0.15, 2)
        rho = rng.uniform(0.6, 1.5)
        f = O.equilibrium(9, rho, u) + rng.uniform(-3e-3, 3e-3, 9)
        eta = rng.normal(size=9)
        omega, kT = rng.uniform(0.5, 1.99), 10 ** rng.uniform(-6, -2)
        r = O.collide_site(9, f, eta, kT, O.paper_lambda(9, omega))
        p = P.d2q9_printed_collision(f, eta, kT, omega)
        assert r["kpre"][4] == pytest.approx(p["k4"], abs=1e-15)
        assert r["kpre"][5] == pytest.approx(p["k5"], abs=1e-15)
        assert np.allclose(r["kstar"], p["kstar"], atol=2e-15)
        assert np.allclose(r["fstar"], p["fstar"], atol=2e-15)


def test_d2q9_deterministic_closed_forms():
    """Sec. 3 Test 2: without noise, the orthogonal and non-orthogonal bases
    give the same f*, equal to the printed non-orthogonal formulas and to the
    printed closed form of f0*."""
    rng = np.random.default_rng(7)
    for _ in range(30):
        u = rng.uniform(-0.15, 0.15, 2)
        f = O.equilibrium(9, rng.uniform(0.6, 1.5), u) + rng.uniform(-3e-3, 3e-3, 9)
        omega = rng.uniform(0.5, 1.99)
        lam = O.paper_lambda(9, omega)
        orth = O.collide_site(9, f, np.zeros(9), 0.0, lam)
        non = O.collide_site(9, f, np.zeros(9), 0.0, lam, basis=1)
        assert np.allclose(orth["fstar"], non["fstar"], atol=2e-15)
        assert np.allclose(non["fstar"], P.d2q9_printed_nonorth_deterministic(f, omega)["fstar"], atol=2e-15)
        assert orth["fstar"][0] == pytest.approx(P.d2q9_printed_f0_deterministic(f, omega), abs=2e-15)


def test_d3q27_offdiagonal_moments_match_printed(paper):
    """k_7, k_8, k_9 as the printed signed population sums minus rho u_a u_b."""
    c, _ = O.lattice(27)
    rng = np.random.default_rng(9)
    for _ in range(20):
        u = rng.uniform(-0.1, 0.1, 3)
        f = O.equilibrium(27, rng.uniform(0.7, 1.4), u) + rng.uniform(-1e-3, 1e-3, 27)
        r = O.collide_site(27, f, np.zeros(27), 0.0, O.paper_lambda(27, 1.3))
        rho, ux, uy, uz = r["macro"]
        for key, (a, b) in {"k7_signs": (ux, uy), "k8_signs": (ux, uz), "k9_signs": (uy, uz)}.items():
            s = sum(sgn * f[int(i)] for i, sgn in paper["d3q27"][key].items()) - rho * a * b
            v = {"k7_signs": 7, "k8_signs": 8, "k9_signs": 9}[key]
            assert r["kpre"][v] == pytest.approx(s, abs=1e-15)


@pytest.mark.parametrize("q", [9, 27])
def test_reconstruction_paths_agree(q):
    """f* = T(u)^-1 k* by LU equals f* = M^-1 N(-u) k* with M^-1 = W M^T B^-1,
    and T(u) f* reproduces k*."""
    rng = np.random.default_rng(13)
    d = 2 if q == 9 else 3
    for _ in range(20):
        u = rng.uniform(-0.2, 0.2, d)
        f = O.equilibrium(q, rng.uniform(0.6, 1.5), u) + rng.uniform(-2e-3, 2e-3, q)
        eta = rng.normal(size=q)
        lam = rng.uniform(0.3, 1.95, q)
        a = O.collide_site(q, f, eta, 1e-3, lam, method=0)
        b = O.collide_site(q, f, eta, 1e-3, lam, method=1)
        assert np.allclose(a["fstar"], b["fstar"], atol=1e-14)
        T = O.transform(q, a["macro"][1:1 + d])
        assert np.allclose(T @ a["fstar"], a["kstar"], atol=1e-14)


@pytest.mark.parametrize("q", [9, 19, 27])
def test_collision_conserves_mass_and_momentum(q):
    c, _ = O.lattice(q)
    rng = np.random.default_rng(17)
    d = 2 if q == 9 else 3
    for _ in range(20):
        f = O.equilibrium(q, rng.uniform(0.6, 1.5), rng.uniform(-0.2, 0.2, d)) + rng.uniform(-2e-3, 2e-3, q)
        r = O.collide_site(q, f, rng.normal(size=q), 1e-2, rng.uniform(0.3, 1.95, q))
        assert r["fstar"].sum() == pytest.approx(f.sum(), abs=1e-14)
        assert np.allclose(c.T @ r["fstar"], c.T @ f, atol=1e-14)


@pytest.mark.parametrize("q", [9, 19, 27])
def test_single_site_ou_stationary_variance(q):
    """Iterated noisy collisions at one site: each non-conserved central moment
    is a discrete OU process whose stationary variance is
    phi_v^2 / (Lambda_v (2 - Lambda_v)) = rho kT b_v / c_s^2 (the diagonal
    C_eq of Sec. 2.2), with vanishing cross-covariances.  Noise drawn from an
    independent numpy generator."""
    rng = np.random.default_rng(23)
    d = 2 if q == 9 else 3
    rho, kT = 1.1, 1e-3
    lam = O.paper_lambda(q, 1.4)
    f = O.equilibrium(q, rho, np.full(d, 0.05))
    nsamp = 6000
    ks = np.zeros((nsamp, q))
    for t in range(nsamp + 50):
        r = O.collide_site(q, f, rng.normal(size=q), kT, lam)
        if t >= 50:
            ks[t - 50] = r["kpre"]
        f = r["fstar"]
    first = 3 if q == 9 else 4
    target = rho * kT * O.norms(q) / CS2
    var = ks.var(axis=0)
    rel = var[first:] / target[first:] - 1.0
    # 6000 samples: relative standard error of a variance ~ sqrt(2/6000) = 1.8 %
    assert np.abs(rel).max() < 0.08
    assert abs(rel.mean()) < 0.02
    corr = np.corrcoef(ks[:, first:].T)
    assert np.abs(corr - np.eye(q - first)).max() < 0.08
