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
* N(u)^-1 is applied as a polynomial matrix in u.  Its columns 1-3 are
  dropped: the central first moments k_1..k_3 vanish identically (before
  and after the collision), and callers pass them as zero.

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


def reduced_form(e, u):
    """The cheapest of a few equivalent forms of a polynomial entry of
    N(u)^-1, written in u_a and the squares uxx, uyy, uzz, uu = |u|^2."""
    ux, uy, uz = u
    A, B, C, U2 = sp.symbols("uxx uyy uzz uu")
    q = 0
    for (i, j, k), coef in sp.Poly(sp.expand(e), ux, uy, uz).terms():
        q += coef * A ** (i // 2) * B ** (j // 2) * C ** (k // 2) * ux ** (i % 2) * uy ** (j % 2) * uz ** (k % 2)
    cands = [sp.expand(e), q, sp.factor(q)]
    for var, rest in ((A, B + C), (B, A + C), (C, A + B)):
        s = sp.expand(q.subs(var, U2 - rest))
        cands += [s, sp.factor(s)]
    if q.free_symbols:
        cands.append(sp.horner(q))
    return min(cands, key=sp.count_ops)


def gen_shift_inverse(L, k):
    """r = N(u)^-1 k for k_1 = k_2 = k_3 = 0."""
    ux, uy, uz = L.u
    A, B, C, U2 = sp.symbols("uxx uyy uzz uu")
    exprs = []
    for v in range(19):
        e = 0 if v in (1, 2, 3) else k[v]
        for c in range(19):
            if c == v or c in (1, 2, 3) or L.Ninv[v, c] == 0:
                continue
            e += reduced_form(L.Ninv[v, c], L.u) * k[c]
        exprs.append(e)
    back = {A: ux ** 2, B: uy ** 2, C: uz ** 2, U2: ux ** 2 + uy ** 2 + uz ** 2}
    zero = {k[1]: 0, k[2]: 0, k[3]: 0}
    for v in range(19):
        ref = sum(L.Ninv[v, c] * k[c] for c in range(19)).subs(zero)
        assert sp.expand(exprs[v].subs(back) - ref) == 0
    lines = ["  const R uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;",
             "  const R uu = uxx + uyy + uzz;"]
    lines += emit(exprs, [f"const R t{v}" for v in range(19)], "q")
    lines += [f"  k[{v}] = t{v};" for v in range(19)]
    return lines


def gen_populations(L, r, d):
    """d_i = w_i sum_v P_v(c_i) r_v / b_v: per orbit, one sum per sign class,
    then the inverse butterfly over the orbit's members."""
    exprs, names, gval = [], [], {}
    for absc in L.orbits:
        w = W[L.orbits[absc][0]]
        nz = [a for a in range(3) if absc[a]]
        for n in range(len(nz) + 1):
            for axes in itertools.combinations(nz, n):
                cls = axis_class(*axes)
                e = 0
                for v in range(19):
                    if L.parity[v] == cls:
                        e += w * L.P_abs(v, absc) / L.b[v] * r[v]
                name = f"g{orbit_tag(absc)}_{class_tag(cls)}"
                exprs.append(sp.expand(e))
                names.append(f"const R {name}")
                gval[(absc, cls)] = sp.expand(e)
    lines = emit(exprs, names, "p")
    out = {}
    for absc in L.orbits:
        nz = [a for a in range(3) if absc[a]]
        t = orbit_tag(absc)
        g = lambda cls: f"g{t}_{class_tag(cls)}"
        if not nz:
            i = L.orbits[absc][0]
            lines.append(f"  d[{i}] = {g((0, 0, 0))};")
            out[i] = gval[(absc, (0, 0, 0))]
        elif len(nz) == 1:
            ca = axis_class(nz[0])
            p, m = L.member(absc, [1]), L.member(absc, [-1])
            lines += [f"  d[{p}] = {g((0, 0, 0))} + {g(ca)};", f"  d[{m}] = {g((0, 0, 0))} - {g(ca)};"]
            out[p] = gval[(absc, (0, 0, 0))] + gval[(absc, ca)]
            out[m] = gval[(absc, (0, 0, 0))] - gval[(absc, ca)]
        else:
            a, b = nz
            ca, cb, cab = axis_class(a), axis_class(b), axis_class(a, b)
            pp, mm = L.member(absc, [1, 1]), L.member(absc, [-1, -1])
            pm, mp = L.member(absc, [1, -1]), L.member(absc, [-1, 1])
            lines += [f"  const R e1_{t} = {g((0, 0, 0))} + {g(cab)};",
                      f"  const R e2_{t} = {g((0, 0, 0))} - {g(cab)};",
                      f"  const R o1_{t} = {g(ca)} + {g(cb)};",
                      f"  const R o2_{t} = {g(ca)} - {g(cb)};",
                      f"  d[{pp}] = e1_{t} + o1_{t};", f"  d[{mm}] = e1_{t} - o1_{t};",
                      f"  d[{pm}] = e2_{t} + o2_{t};", f"  d[{mp}] = e2_{t} - o2_{t};"]
            G = lambda cls: gval[(absc, cls)]
            out[pp] = G((0, 0, 0)) + G(cab) + G(ca) + G(cb)
            out[mm] = G((0, 0, 0)) + G(cab) - G(ca) - G(cb)
            out[pm] = G((0, 0, 0)) - G(cab) + G(ca) - G(cb)
            out[mp] = G((0, 0, 0)) - G(cab) - G(ca) + G(cb)
    for i in range(19):
        assert sp.expand(out[i] - sum(L.Minv[i, v] * r[v] for v in range(19))) == 0
    return lines


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
