"""The paper's printed D2Q9 and D3Q19 formulas, typed as printed, used as pins
for the oracle (De Rosis & Zhou, arXiv 2602.16486).

Each function follows one block of printed equations:
  * ``d2q9_printed_collision`` -- Sec. 2.2: eq. (macro), eq. (pre_coll_rms),
    eq. (pre_coll_cms), eq. (post_coll_cms), eq. (post_coll_rms) and
    eq. (post_coll_pops).  r6* takes ``2 u_x k5*`` as printed in Sec. 2.2 (the
    Test 2 listing of Sec. 3 prints ``2 u_y k5*`` there; the Sec. 2.2 form is the
    one consistent with N^-1 k*).
  * ``d2q9_printed_f0_deterministic`` -- Sec. 3, Test 2: closed form of f0* in
    the absence of noise.
  * ``d2q9_printed_nonorth_deterministic`` -- Sec. 3, Test 2: post-collision
    central moments, raw moments and populations of the non-orthogonal basis.
  * ``d3q19_printed_feq`` -- Sec. 2.4: the fourth-order D3Q19 equilibrium
    (rest, axis and face-diagonal expressions).
"""
import math

import numpy as np

CS2 = 1.0 / 3.0
CS = math.sqrt(CS2)

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


def _macro(f):
    rho = f.sum()
    return rho, (CX @ f) / rho, (CY @ f) / rho


def d2q9_printed_collision(f, eta, kT, omega):
    """f* of one site from the printed D2Q9 equations; eta[3..8] are used."""
    f = np.asarray(f, dtype=float)
    rho, ux, uy = _macro(f)
    r4 = f[1] - f[2] + f[3] - f[4]
    r5 = f[5] - f[6] + f[7] - f[8]
    k4 = r4 - rho * (ux * ux - uy * uy)
    k5 = r5 - rho * ux * uy
    s = math.sqrt
    k = np.zeros(9)
    k[0] = rho
    k[3] = 2 * s(rho * kT * CS2) * eta[3]
    k[4] = (1 - omega) * k4 + 2 * s(rho * kT * CS2 * omega * (2 - omega)) * eta[4]
    k[5] = (1 - omega) * k5 + s(rho * kT * CS2 * omega * (2 - omega)) * eta[5]
    k[6] = s(2 * rho * kT) * CS2 * eta[6]
    k[7] = s(2 * rho * kT) * CS2 * eta[7]
    k[8] = 2 * s(rho * kT) * CS ** 3 * eta[8]
    r = np.zeros(9)
    r[0] = k[0]
    r[1] = rho * ux
    r[2] = rho * uy
    r[3] = k[3] + rho * (ux ** 2 + uy ** 2)
    r[4] = k[4] + rho * (ux ** 2 - uy ** 2)
    r[5] = k[5] + rho * ux * uy
    r[6] = k[6] + 2 * ux * k[5] + 0.5 * uy * (k[3] + k[4]) + rho * ux ** 2 * uy
    r[7] = k[7] + 2 * uy * k[5] + 0.5 * ux * (k[3] - k[4]) + rho * ux * uy ** 2
    r[8] = (k[8] + 2 * (ux * k[7] + uy * k[6]) + 4 * ux * uy * k[5]
            - 0.5 * (ux ** 2 - uy ** 2) * k[4] + 0.5 * (ux ** 2 + uy ** 2) * k[3]
            + rho * ux ** 2 * uy ** 2)
    fs = np.zeros(9)
    fs[0] = 4 * r[0] / 9 - 2 * r[3] / 3 + r[8]
    fs[1] = r[0] / 9 + r[1] / 3 + r[3] / 12 + r[4] / 4 - (r[7] + r[8]) / 2
    fs[2] = r[0] / 9 + r[2] / 3 + r[3] / 12 - r[4] / 4 - (r[6] + r[8]) / 2
    fs[3] = r[0] / 9 - r[1] / 3 + r[3] / 12 + r[4] / 4 + (r[7] - r[8]) / 2
    fs[4] = r[0] / 9 - r[2] / 3 + r[3] / 12 - r[4] / 4 + (r[6] - r[8]) / 2
    fs[5] = r[0] / 36 + (r[1] + r[2] + r[3]) / 12 + (r[5] + r[6] + r[7] + r[8]) / 4
    fs[6] = r[0] / 36 + (-r[1] + r[2] + r[3]) / 12 + (-r[5] + r[6] - r[7] + r[8]) / 4
    fs[7] = r[0] / 36 + (-r[1] - r[2] + r[3]) / 12 + (r[5] - r[6] - r[7] + r[8]) / 4
    fs[8] = r[0] / 36 + (r[1] - r[2] + r[3]) / 12 + (-r[5] - r[6] + r[7] + r[8]) / 4
    return {"k4": k4, "k5": k5, "kstar": k, "rstar": r, "fstar": fs}


def d2q9_printed_f0_deterministic(f, omega):
    """Test 2 closed form of the rest population after a noise-free collision."""
    f = np.asarray(f, dtype=float)
    rho, ux, uy = _macro(f)
    k4 = (f[1] - f[2] + f[3] - f[4]) - rho * (ux * ux - uy * uy)
    k5 = (f[5] - f[6] + f[7] - f[8]) - rho * ux * uy
    return (rho * (ux ** 2 * uy ** 2 - 2 * CS2 * (ux ** 2 + uy ** 2) + 4 * CS2 ** 2)
            + 0.5 * (uy ** 2 - ux ** 2) * (1 - omega) * k4 + 4 * ux * uy * (1 - omega) * k5)


def d2q9_printed_nonorth_deterministic(f, omega):
    """Test 2: noise-free collision in the non-orthogonal basis, printed form."""
    f = np.asarray(f, dtype=float)
    rho, ux, uy = _macro(f)
    k4 = (f[1] - f[2] + f[3] - f[4]) - rho * (ux * ux - uy * uy)
    k5 = (f[5] - f[6] + f[7] - f[8]) - rho * ux * uy
    k4s, k5s = (1 - omega) * k4, (1 - omega) * k5
    r = np.zeros(9)
    r[0] = rho
    r[1] = rho * ux
    r[2] = rho * uy
    r[3] = rho * (ux ** 2 + uy ** 2 + 2 * CS2)
    r[4] = k4s + rho * (ux ** 2 - uy ** 2)
    r[5] = k5s + rho * ux * uy
    r[6] = 2 * ux * k5s + 0.5 * uy * (2 * rho * CS2 + k4s) + rho * ux ** 2 * uy
    r[7] = 2 * k5s * uy + 0.5 * ux * (2 * rho * CS2 - k4s) + rho * ux * uy ** 2
    r[8] = (4 * ux * uy * k5s - 0.5 * (ux ** 2 - uy ** 2) * k4s
            + rho * (ux ** 2 * uy ** 2 + CS2 ** 2 + CS2 * (ux ** 2 + uy ** 2)))
    fs = np.zeros(9)
    fs[0] = r[0] - r[3] + r[8]
    fs[1] = (r[3] + r[4]) / 4 + (r[1] - r[7] - r[8]) / 2
    fs[2] = (r[3] - r[4]) / 4 + (r[2] - r[6] - r[8]) / 2
    fs[3] = (r[3] + r[4]) / 4 + (-r[1] + r[7] - r[8]) / 2
    fs[4] = (r[3] - r[4]) / 4 + (-r[2] + r[6] - r[8]) / 2
    fs[5] = (r[5] + r[6] + r[7] + r[8]) / 4
    fs[6] = (-r[5] + r[6] - r[7] + r[8]) / 4
    fs[7] = (r[5] - r[6] - r[7] + r[8]) / 4
    fs[8] = (-r[5] - r[6] + r[7] + r[8]) / 4
    return {"rstar": r, "fstar": fs}


def d3q19_printed_feq(rho, u, c):
    """Sec. 2.4 equilibrium for the velocities c ((19, 3) integers), as
    printed: rest, axis (one non-zero component alpha) and face-diagonal
    (components alpha, beta non-zero, gamma zero) populations."""
    u = np.asarray(u, dtype=float)
    u2 = float(u @ u)
    f = np.zeros(len(c))
    for i, ci in enumerate(c):
        nz = [a for a in range(3) if ci[a] != 0]
        if not nz:
            f[i] = rho * (1.0 / 3.0 + u2 / 6.0 + 0.5 * u2 * u2)
        elif len(nz) == 1:
            a = nz[0]
            cu = ci[a] * u[a]
            f[i] = rho * (1.0 / 18.0 + cu / 6.0 - u2 / 3.0 - 0.5 * cu * u2 + 0.5 * u2 * u2)
        else:
            a, b = nz
            g = 3 - a - b
            ca, cb = ci[a], ci[b]
            ua, ub, ug = u[a], u[b], u[g]
            f[i] = rho * (1.0 / 36.0 + (ca * ua + cb * ub) / 12.0 + 5.0 / 24.0 * (ua ** 2 + ub ** 2)
                          - ug ** 2 / 8.0 + ca * cb * ua * ub / 4.0
                          + (ca * ua ** 3 + cb * ub ** 3) / 8.0
                          + (ca * ua * ub ** 2 + cb * ub * ua ** 2) / 4.0
                          - (ua ** 4 + ub ** 4) / 8.0 + ua ** 2 * ub ** 2 / 4.0 + 3.0 / 8.0 * ug ** 4)
    return f
