#!/usr/bin/env python3
"""Generate cmflb_d3q19.h: the D3Q19 central-moment transforms as
straight-line device code (build-time tool; needs sympy, the library does
not).

D3Q19 (Sec. 2.4 of De Rosis & Zhou, arXiv 2602.16486): velocities {-1,0,1}^3
without the eight corners, in the D3Q27 order of Sec. 2.3 with the corners
left out; weights 1/3, 1/18, 1/36; the 19 basis polynomials P_v printed
there.  With M_vi = P_v(c_i) and T_vi(u) = P_v(c_i - u), the shift matrix
N(u) = T(u) M^-1 maps basis raw moments r = M f to central moments
k = N(u) r.  Because the basis is graded by polynomial degree and the
polynomials of degree < n restricted to the lattice are spanned by the basis
rows of degree < n, N(u) is block lower-triangular in the degree with unit
diagonal blocks, and so is N(u)^-1 (which is not N(-u) on this lattice).
M^-1 = W M^T B^-1 (weighted orthogonality, norms b_v = sum_i w_i P_v(c_i)^2).

Evaluation order, chosen for few operations:
* every basis polynomial has a definite parity in each coordinate, so both
  r = M d and d = M^-1 r go through the sign classes of each orbit of
  velocities with equal |c_a| (a butterfly of sums and differences);
* N(u)^-1 is applied row by row in the combinations D = 3 u_x^2 - |u|^2,
  E = u_y^2 - u_z^2 and the products u_a k_b that the rows share.  Its
  columns 1-3 are dropped: the central first moments k_1..k_3 vanish
  identically (before and after the collision), and callers pass them as
  zero.

Every emitted function is checked here symbolically against its definition.

    python gen_d3q19.py > cmflb_d3q19.h
"""
import itertools

import sympy as sp
from sympy.printing.c import C99CodePrinter

CX = [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0]
CY = [0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1]
CZ = [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1]
W = [sp.Rational(1, 3)] + [sp.Rational(1, 18)] * 6 + [sp.Rational(1, 36)] * 12
DEG = [0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 4, 4, 4]


def basis(x, y, z):
    c2 = x * x + y * y + z * z
    return [1, x, y, z, c2 - 1, 3 * x * x - c2, y * y - z * z, x * y, y * z, x * z,
            x * (3 * c2 - 5), y * (3 * c2 - 5), z * (3 * c2 - 5),
            x * (y * y - z * z), y * (z * z - x * x), z * (x * x - y * y),
            3 * c2 * c2 - 6 * c2 + 1, (2 * c2 - 3) * (3 * x * x - c2), (2 * c2 - 3) * (y * y - z * z)]


class _Printer(C99CodePrinter):
    """C for the compute type R: rational and integer constants as R(...)
    literals, small integer powers multiplied out."""

    def _print_Pow(self, e):
        base, ex = e.as_base_exp()
        if ex.is_Integer and 1 < int(ex) <= 4:
            return "(" + "*".join([self._print(base)] * int(ex)) + ")"
        return super()._print_Pow(e)

    def _print_Integer(self, n):
        return f"R({int(n)})"

    def _print_Rational(self, q):
        return f"R({float(q)!r})"

    def _print_Float(self, f):
        return f"R({float(f)!r})"


_PRINT = _Printer()


def emit(exprs, names, prefix):
    """C statements assigning exprs to names, with common subexpressions
    (temporaries named prefix0, prefix1, ...)."""
    repl, red = sp.cse(exprs, symbols=sp.numbered_symbols(prefix), optimizations="basic")
    out = [f"  const R {sym} = {_PRINT.doprint(e)};" for sym, e in repl]
    out += [f"  {name} = {_PRINT.doprint(e)};" for name, e in zip(names, red)]
    return out


class Lattice:
    def __init__(self):
        self.u = sp.symbols("ux uy uz")
        ux, uy, uz = self.u
        self.C = [(CX[i], CY[i], CZ[i]) for i in range(19)]
        self.T = sp.Matrix([[sp.expand(basis(CX[i] - ux, CY[i] - uy, CZ[i] - uz)[v]) for i in range(19)]
                            for v in range(19)])
        self.M = self.T.subs({ux: 0, uy: 0, uz: 0})
        self.b = [sum(W[i] * self.M[v, i] ** 2 for i in range(19)) for v in range(19)]
        self.Minv = sp.Matrix(19, 19, lambda i, v: W[i] * self.M[v, i] / self.b[v])
        assert sp.simplify(self.Minv * self.M - sp.eye(19)) == sp.zeros(19, 19)
        self.N = sp.expand(self.T * self.Minv)
        for v in range(19):
            for w in range(19):
                if DEG[w] > DEG[v]:
                    assert self.N[v, w] == 0
                if DEG[w] == DEG[v]:
                    assert self.N[v, w] == (1 if v == w else 0)
        # N^-1 by forward substitution, column by column
        self.Ninv = sp.zeros(19, 19)
        for c in range(19):
            x = [0] * 19
            for v in range(19):
                s = 1 if v == c else 0
                for w in range(v):
                    if self.N[v, w] != 0:
                        s -= self.N[v, w] * x[w]
                x[v] = sp.expand(s)
            for v in range(19):
                self.Ninv[v, c] = x[v]
        assert sp.expand(self.Ninv * self.N) == sp.eye(19)
        # per-coordinate parity of each basis polynomial (1 = odd)
        X, Y, Z = sp.symbols("X Y Z")
        P = [sp.expand(p) for p in basis(X, Y, Z)]
        self.parity = []
        for v in range(19):
            par = []
            for s in (X, Y, Z):
                flipped = P[v].subs(s, -s)
                assert sp.expand(flipped - P[v]) == 0 or sp.expand(flipped + P[v]) == 0
                par.append(0 if sp.expand(flipped - P[v]) == 0 else 1)
            self.parity.append(tuple(par))
        self.P_abs = lambda v, a: P[v].subs({X: a[0], Y: a[1], Z: a[2]})
        # orbits of velocities with equal |c_a|
        self.orbits = {}
        for i, c in enumerate(self.C):
            self.orbits.setdefault(tuple(abs(x) for x in c), []).append(i)

    def member(self, absc, signs):
        """index of the orbit member with the given signs on its nonzero axes"""
        nz = [a for a in range(3) if absc[a]]
        for i in self.orbits[absc]:
            if all((self.C[i][a] > 0) == (s > 0) for a, s in zip(nz, signs)):
                return i
        raise KeyError((absc, signs))


def orbit_tag(absc):
    return "".join(map(str, absc))


def class_tag(cls):
    return "".join(map(str, cls))


def axis_class(*axes):
    return tuple(1 if a in axes else 0 for a in range(3))


def gen_raw_moments(L, d):
    """r_v = sum_i P_v(c_i) d_i through the sign-class sums of each orbit."""
    lines, value, sym = [], {}, {}

    def define(name, expr_text, expr):
        lines.append(f"  const R {name} = {expr_text};")
        value[name] = expr
        return sp.Symbol(name)

    for absc in L.orbits:
        nz = [a for a in range(3) if absc[a]]
        t = orbit_tag(absc)
        if not nz:
            i = L.orbits[absc][0]
            sym[(absc, (0, 0, 0))] = d[i]
            continue
        if len(nz) == 1:
            p, m = L.member(absc, [1]), L.member(absc, [-1])
            sym[(absc, (0, 0, 0))] = define(f"w{t}_000", f"d[{p}] + d[{m}]", d[p] + d[m])
            sym[(absc, axis_class(nz[0]))] = define(f"w{t}_{class_tag(axis_class(nz[0]))}",
                                                     f"d[{p}] - d[{m}]", d[p] - d[m])
            continue
        a, b = nz
        pp, mm = L.member(absc, [1, 1]), L.member(absc, [-1, -1])
        pm, mp = L.member(absc, [1, -1]), L.member(absc, [-1, 1])
        define(f"s1_{t}", f"d[{pp}] + d[{mm}]", d[pp] + d[mm])
        define(f"a1_{t}", f"d[{pp}] - d[{mm}]", d[pp] - d[mm])
        define(f"s2_{t}", f"d[{pm}] + d[{mp}]", d[pm] + d[mp])
        define(f"a2_{t}", f"d[{pm}] - d[{mp}]", d[pm] - d[mp])
        for cls, op, x, y in (((0, 0, 0), "+", "s1", "s2"), (axis_class(a, b), "-", "s1", "s2"),
                              (axis_class(a), "+", "a1", "a2"), (axis_class(b), "-", "a1", "a2")):
            e = value[f"{x}_{t}"] + value[f"{y}_{t}"] if op == "+" else value[f"{x}_{t}"] - value[f"{y}_{t}"]
            sym[(absc, cls)] = define(f"w{t}_{class_tag(cls)}", f"{x}_{t} {op} {y}_{t}", e)
    exprs = []
    for v in range(19):
        e = 0
        cls = L.parity[v]
        for absc in L.orbits:
            if any(cls[a] and not absc[a] for a in range(3)):
                continue  # odd in an axis along which the orbit has c_a = 0
            coef = L.P_abs(v, absc)
            if coef != 0:
                e += coef * sym[(absc, cls)]
        exprs.append(e)
    # check: the sign-class sums reproduce M d
    subs = {sp.Symbol(k): val for k, val in value.items()}
    for v in range(19):
        assert sp.expand(exprs[v].subs(subs) - sum(L.M[v, i] * d[i] for i in range(19))) == 0
    return lines + emit(exprs, [f"r[{v}]" for v in range(19)], "a")


class Steps:
    """Straight-line code as named temporaries: define() records each one
    with its expression in earlier temporaries, expand() writes any
    expression back in the inputs (for the symbolic checks)."""

    def __init__(self):
        self.defs, self.value = [], {}

    def define(self, name, expr):
        sym = sp.Symbol(name)
        self.defs.append((sym, expr))
        self.value[sym] = sp.expand(sp.sympify(expr).subs(self.value))
        return sym

    def expand(self, expr):
        return sp.expand(sp.sympify(expr).subs(self.value))

    def lines(self):
        return [f"  const R {sym} = {_PRINT.doprint(e)};" for sym, e in self.defs]


def gen_shift_inverse(L, k):
    """r = N(u)^-1 k for k_1 = k_2 = k_3 = 0, written with the second
    central moments' combinations D = 3 u_x^2 - |u|^2 and E = u_y^2 - u_z^2
    and the products u_a k_7..k_9 shared between the rows; checked against
    the entries of N(u)^-1 (computed above by forward substitution)."""
    ux, uy, uz = L.u
    R = sp.Rational
    S = Steps()
    rho = k[0]
    uxx, uyy, uzz = S.define("uxx", ux * ux), S.define("uyy", uy * uy), S.define("uzz", uz * uz)
    uu = S.define("uu", uxx + uyy + uzz)
    D = S.define("dd", 3 * uxx - uu)
    E = S.define("ee", uyy - uzz)
    r = [None] * 19
    r[0] = rho
    r[1], r[2], r[3] = S.define("jx", rho * ux), S.define("jy", rho * uy), S.define("jz", rho * uz)
    y7, x7 = S.define("y7", uy * k[7]), S.define("x7", ux * k[7])
    z8, y8 = S.define("z8", uz * k[8]), S.define("y8", uy * k[8])
    z9, x9 = S.define("z9", uz * k[9]), S.define("x9", ux * k[9])
    r[4] = S.define("t4", k[4] + rho * uu)
    r[5] = S.define("t5", k[5] + rho * D)
    r[6] = S.define("t6", k[6] + rho * E)
    r[7] = S.define("t7", k[7] + r[1] * uy)
    r[8] = S.define("t8", k[8] + r[2] * uz)
    r[9] = S.define("t9", k[9] + r[1] * uz)
    A = S.define("aa", 3 * rho * uu + 5 * k[4])
    F = S.define("ff", A - k[5])
    s79, s78, s89 = S.define("s79", y7 + z9), S.define("s78", x7 + z8), S.define("s89", y8 + x9)
    d79, d87, d98 = S.define("d79", y7 - z9), S.define("d87", z8 - x7), S.define("d98", x9 - y8)
    h56p, h56m = S.define("h56p", r[5] + r[6]), S.define("h56m", r[5] - r[6])
    r[10] = S.define("t10", k[10] + ux * (A + 2 * k[5]) + 6 * s79)
    r[11] = S.define("t11", k[11] + uy * (F + 3 * k[6]) + 6 * s78)
    r[12] = S.define("t12", k[12] + uz * (F - 3 * k[6]) + 6 * s89)
    r[13] = S.define("t13", k[13] + ux * r[6] + 2 * d79)
    r[14] = S.define("t14", k[14] - R(1, 2) * uy * h56p + 2 * d87)
    r[15] = S.define("t15", k[15] + R(1, 2) * uz * h56m + 2 * d98)
    c1 = S.define("c1", ux * k[10] + uy * k[11] + uz * k[12])
    c2 = S.define("c2", ux * s79 + uy * z8)
    c3 = S.define("c3", uy * k[11] + uz * k[12])
    c4 = S.define("c4", uy * k[11] - uz * k[12])
    c5 = S.define("c5", uy * k[14] - uz * k[15])
    c6 = S.define("c6", uy * k[14] + uz * k[15])
    r[16] = S.define("t16", k[16] + 4 * c1 + 24 * c2 + uu * (rho * (3 * uu + 4) + 10 * k[4])
                     + 2 * D * k[5] + 6 * E * k[6])
    r[17] = S.define("t17", k[17] + D * (rho * (R(5, 3) - 3 * uxx - uu) - R(4, 3) * k[4])
                     + E * (3 * rho * E + 5 * k[6]) - R(1, 3) * (15 * uxx - uu) * k[5]
                     + 8 * ux * s79 - 16 * uy * z8 + R(4, 3) * ux * k[10] - R(2, 3) * c3 - 6 * c5)
    r[18] = S.define("t18", k[18] + E * (rho * (6 * uxx - 4 * uu + R(5, 3)) - R(4, 3) * k[4] + R(5, 3) * k[5])
                     + (5 * uxx - 3 * uu) * k[6] + 8 * ux * d79 + R(2, 3) * c4 + 4 * ux * k[13] - 2 * c6)
    zero = {k[1]: 0, k[2]: 0, k[3]: 0}
    for v in range(19):
        ref = sum(L.Ninv[v, c] * k[c] for c in range(19)).subs(zero)
        assert sp.expand(S.expand(r[v]) - ref) == 0, v
    return S.lines() + [f"  k[{v}] = {_PRINT.doprint(r[v])};" for v in range(1, 19)]


def gen_populations(L, r, d):
    """d_i = w_i sum_v P_v(c_i) r_v / b_v.  Every P_v is even or odd in
    each coordinate, so each orbit of equal |c_a| needs one sum per sign
    class and a butterfly over its members; the three axis orbits and the
    three face-diagonal orbits also share the parts of those sums that the
    permutations of the axes leave alike.  Checked against W M^T B^-1."""
    S = Steps()
    w0, w1, w2 = W[0], W[1], W[7]
    b = L.b

    def a(v, w):  # w r_v / b_v
        return (w / b[v]) * r[v]

    out = [None] * 19
    # axis orbits, |c|^2 = 1: even parts C + 2P, C - P + Q, C - P - Q
    C = S.define("pc", a(0, w1) - 2 * a(16, w1))
    P = S.define("pp", a(5, w1) - a(17, w1))
    Q = S.define("pq", a(6, w1) - a(18, w1))
    CP = S.define("pcp", C - P)
    even = [S.define("pex", C + 2 * P), S.define("pey", CP + Q), S.define("pez", CP - Q)]
    odd = [S.define(f"po{n}", a(1 + ax, w1) - 2 * a(10 + ax, w1)) for ax, n in enumerate("xyz")]
    for ax in range(3):
        cp, cm = [0, 0, 0], [0, 0, 0]
        cp[ax], cm[ax] = 1, -1
        out[L.C.index(tuple(cp))] = even[ax] + odd[ax]
        out[L.C.index(tuple(cm))] = even[ax] - odd[ax]
    # face-diagonal orbits, |c|^2 = 2
    C2 = S.define("fc", a(0, w2) + a(4, w2) + a(16, w2))
    P2 = S.define("fp", a(5, w2) + a(17, w2))
    Q2 = S.define("fq", a(6, w2) + a(18, w2))
    CP2 = S.define("fcp", C2 + P2)
    E2 = {(0, 1): S.define("fe110", CP2 + Q2), (0, 2): S.define("fe101", CP2 - Q2),
          (1, 2): S.define("fe011", C2 - 2 * P2)}
    X1 = [S.define(f"f{n}", a(1 + ax, w2) + a(10 + ax, w2)) for ax, n in enumerate("xyz")]
    A3 = [S.define(f"f{13 + ax}", a(13 + ax, w2)) for ax in range(3)]
    OO = {(0, 1): S.define("fxy", a(7, w2)), (0, 2): S.define("fxz", a(9, w2)),
          (1, 2): S.define("fyz", a(8, w2))}
    # class odd in axis a only: X1[a] +- (the mode 13 + a with its sign here)
    OA = {(0, 1): (S.define("fx110", X1[0] + A3[0]), S.define("fy110", X1[1] - A3[1])),
          (0, 2): (S.define("fx101", X1[0] - A3[0]), S.define("fz101", X1[2] + A3[2])),
          (1, 2): (S.define("fy011", X1[1] + A3[1]), S.define("fz011", X1[2] - A3[2]))}
    for (ax, bx), (oa, ob) in OA.items():
        t = f"{ax}{bx}"
        e1, e2 = S.define(f"e1_{t}", E2[(ax, bx)] + OO[(ax, bx)]), S.define(f"e2_{t}", E2[(ax, bx)] - OO[(ax, bx)])
        o1, o2 = S.define(f"o1_{t}", oa + ob), S.define(f"o2_{t}", oa - ob)
        for sa in (1, -1):
            for sb in (1, -1):
                c = [0, 0, 0]
                c[ax], c[bx] = sa, sb
                out[L.C.index(tuple(c))] = (e1 + sa * o1) if sa == sb else (e2 + sa * o2)
    # rest population: r_0 minus the other 18, whose sum is 2 (sum of the
    # axis even parts) + 4 (sum of the face-diagonal even parts).  Equal to
    # w_0 sum_v P_v(0) r_v / b_v, but the stored populations then sum to
    # r_0 up to unbiased rounding: the rounded constants w_0 / b_v, w_1 / b_v,
    # w_2 / b_v of the direct formula leave a fixed fraction of r_4 and r_16
    # (whose means are O(rho u^2), i.e. O(kT)) in the mass, a drift linear in
    # the number of steps in FP32.
    rest = S.define("prest", 2 * (even[0] + even[1] + even[2]) + 4 * (E2[(0, 1)] + E2[(0, 2)] + E2[(1, 2)]))
    out[0] = r[0] - rest
    for i in range(19):
        assert sp.expand(S.expand(out[i]) - sum(L.Minv[i, v] * r[v] for v in range(19))) == 0, i
    return S.lines() + [f"  d[{i}] = {_PRINT.doprint(out[i])};" for i in range(19)]


def main():
    L = Lattice()
    d = [sp.Symbol(f"d[{i}]") for i in range(19)]
    r = [sp.Symbol(f"r[{i}]") for i in range(19)]
    k = [sp.Symbol(f"k[{i}]") for i in range(19)]

    lines = [
        "// cmflb_d3q19.h -- D3Q19 central-moment transforms (Sec. 2.4 basis),",
        "// generated by gen_d3q19.py; do not edit by hand.",
        "//",
        "// r = M d: basis raw moments; k = N(u) r: central moments;",
        "// r = N(u)^-1 k for k_1 = k_2 = k_3 = 0; d = M^-1 r = W M^T B^-1 r.",
        "// M d and M^-1 r go through the sign-class sums of each orbit of",
        "// velocities with equal |c_a| (every P_v is even or odd in each c_a).",
        "#pragma once",
        "",
        "#include <hip/hip_runtime.h>",
        "",
        "namespace cmf {",
        "namespace d3q19 {",
        "",
        "// r_v = sum_i P_v(c_i) d_i",
        "template <typename R>",
        "__device__ __forceinline__ void raw_moments(const R *d, R *r) {",
    ]
    lines += gen_raw_moments(L, d)
    lines += ["}", "",
              "// k = N(u) r, in place",
              "template <typename R>",
              "__device__ __forceinline__ void shift_forward(R *r, R ux, R uy, R uz) {"]
    lines += emit([sp.expand(sum(L.N[v, w] * r[w] for w in range(19))) for v in range(19)],
                  [f"const R k{v}" for v in range(19)], "s")
    lines += [f"  r[{v}] = k{v};" for v in range(19)]
    lines += ["}", "",
              "// r = N(u)^-1 k, in place, for central moments with k_1 = k_2 = k_3 = 0",
              "// (the central first moments, zero by construction); k_1..k_3 are not",
              "// read, r_1..r_3 = k_0 u_a are written",
              "template <typename R>",
              "__device__ __forceinline__ void shift_inverse(R *k, R ux, R uy, R uz) {"]
    lines += gen_shift_inverse(L, k)
    lines += ["}", "",
              "// d_i = w_i sum_v P_v(c_i) r_v / b_v",
              "template <typename R>",
              "__device__ __forceinline__ void populations(const R *r, R *d) {"]
    lines += gen_populations(L, r, d)
    lines += ["}", "", "}  // namespace d3q19", "}  // namespace cmf"]
    print("\n".join(lines))


if __name__ == "__main__":
    main()
