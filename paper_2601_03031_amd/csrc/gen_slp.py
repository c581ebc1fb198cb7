"""Generate slp_progs.hpp: straight-line programs (SLPs) over F_p for the
wave-cooperative engine in slp.hpp.

A program is a dataflow graph of base-field operations, produced by running the
formulas of the BN254 tower, the twist and the pairing on tracer values.  The
scheduler packs it into levels of at most 64 independent operations; one wavefront
executes a level per step, lane t doing the t-th operation of the level.
Operations:
  MUL  dst = a * b                                  (Montgomery product)
  LIN  dst = ka * a + sb * b + sc * c  (mod p)      ka in [-15, 15], sb, sc in {-1, 0, 1}
Linear combinations are kept symbolic by the tracer and materialised only where a
product or an output needs them, so chains of additions fuse into few LIN operations.
Slots are 32-byte field elements in LDS.  An operand field holds a 3-bit segment and
a 9-bit offset: segment 0 is absolute, segments 1..7 are bases the caller sets before
running a relocatable program.

Programs:
  * Miller-loop bodies for the optimal ate pairing, software-pipelined: the T-chain
    (doubling / addition of the twist point, with line coefficients) runs one step
    ahead of the f-chain (squaring of the accumulator times the pending lines).  The
    loop follows the non-adjacent form of 6u + 2; the closing additions use pi(Q)
    and -pi^2(Q);
  * F_p12 operations for the final exponentiation (relocatable: X in segment 1, Y in
    segment 2, D in segment 3): product, Granger-Scott cyclotomic square, Frobenius
    powers, conjugate, the norm down to F_p and the easy part from the inverse norm.

Run:  python gen_slp.py > slp_progs.hpp      (the build does this)
      python gen_slp.py --check              (run every program on random inputs
                                              against plain polynomial arithmetic)
"""
from __future__ import annotations

import random
import sys

U = 0x44E992B44A6909F1
P = 36 * U**4 + 36 * U**3 + 24 * U**2 + 6 * U + 1
R = 36 * U**4 + 36 * U**3 + 18 * U**2 + 6 * U + 1
RMONT = 1 << 256
LANES = 64
KMAX = 127

OP_NOP, OP_MUL, OP_LIN = 0, 1, 2


# ============================================================================ tracer
ENC_NTERM = 16  # term positions of an encoded operation
ENC_SIDE = 8    # a product's second factor starts at this term position
# Trace-time limits (set per program by build_all from TRACE_LIMITS): terms of a linear
# operation and terms of one factor of a product
NTERM = 16


class Prog:
    """SSA values: ('in', name) | ('const', x) | ('lin', terms) | ('mul', termsA, termsB);
    terms are tuples of (value id, small integer coefficient)"""

    def __init__(self, name):
        self.name = name
        self.vals = []
        self.inputs = {}
        self.outputs = {}
        self.consts = {}
        self.memo = {}
        self.zero = self.const(0)

    def new(self, node):
        key = node if node[0] in ("lin", "mul") else None
        if key is not None and key in self.memo:
            return self.memo[key]
        self.vals.append(node)
        v = len(self.vals) - 1
        if key is not None:
            self.memo[key] = v
        return v

    def inp(self, name):
        v = self.new(("in", name))
        self.inputs[name] = v
        return F(self, {v: 1})

    def const(self, x):
        x %= P
        if x not in self.consts:
            self.consts[x] = self.new(("const", x))
        return self.consts[x]

    def fconst(self, x):
        return F(self, {self.const(x): 1})

    def out(self, name, f):
        self.outputs[name] = f.atom()


def canon(terms):
    return tuple(sorted((k, c) for k, c in terms.items() if c != 0))


class F:
    """a base-field value: a small-integer linear combination of atoms (value ids)"""
    __slots__ = ("p", "t")

    def __init__(self, p, terms):
        self.p = p
        self.t = {k: c for k, c in terms.items() if c != 0}

    def _lin(self, o, s):
        t = dict(self.t)
        for k, c in o.t.items():
            t[k] = t.get(k, 0) + s * c
        return F(self.p, t)

    def __add__(self, o):
        return self._lin(o, 1)

    def __sub__(self, o):
        return self._lin(o, -1)

    def __neg__(self):
        return F(self.p, {k: -c for k, c in self.t.items()})

    def scale(self, k):
        return F(self.p, {a: c * k for a, c in self.t.items()})

    def __mul__(self, o):
        if not self.t or not o.t:
            return F(self.p, {})
        A, B = operand_terms(self.p, self.t), operand_terms(self.p, o.t)
        a, b = canon(A), canon(B)
        if b < a:
            a, b = b, a
        return F(self.p, {self.p.new(("mul", a, b)): 1})

    def sqr(self):
        return self * self

    def mul(self, o):
        return self * o

    def atom(self):
        if not self.t:
            return self.p.zero
        if len(self.t) == 1:
            (k, c), = self.t.items()
            if c == 1:
                return k
        a = materialise(self.p, self.t)
        self.t = {a: 1}
        return a


SIDE = 8


def operand_terms(p, t):
    """a factor of a product: coefficients within [-KMAX, KMAX], at most SIDE terms"""
    t = fit_coeffs(p, dict(t))
    if len(t) > SIDE:
        t = {materialise(p, t): 1}
    return t


def fit_coeffs(p, t):
    """rewrite terms whose coefficient exceeds KMAX through an intermediate LIN"""
    for k, c in list(t.items()):
        if abs(c) > KMAX:
            s = 1 if c > 0 else -1
            a = abs(c)
            f1 = next((d for d in range(KMAX, 1, -1) if a % d == 0 and a // d <= KMAX), None)
            del t[k]
            if f1:
                v = p.new(("lin", ((k, f1),)))
                t[v] = t.get(v, 0) + s * (a // f1)
            else:
                v = p.new(("lin", ((k, KMAX),)))
                t[v] = t.get(v, 0) + s * (a // KMAX)
                if a % KMAX:
                    t[k] = t.get(k, 0) + s * (a % KMAX)
            return fit_coeffs(p, {kk: cc for kk, cc in t.items() if cc})
    return t


def materialise(p, terms):
    """LIN operations computing sum c_k x_k, NTERM terms per operation, shallow tree"""
    t = fit_coeffs(p, {k: c for k, c in terms.items() if c != 0})
    if not t:
        return p.zero
    if len(t) == 1:
        (k, c), = t.items()
        if c == 1:
            return k
    items = sorted(t.items(), key=lambda kc: (-abs(kc[1]), kc[0]))
    if len(items) <= NTERM:
        return p.new(("lin", canon(dict(items))))
    n = len(items)
    g = -(-(n - NTERM) // (NTERM - 1))          # sub-sums needed
    raw = items[:NTERM - g]
    rest = items[NTERM - g:]
    subs = []
    per = -(-len(rest) // g)
    for i in range(0, len(rest), per):
        subs.append((materialise(p, dict(rest[i:i + per])), 1))
    return p.new(("lin", canon(dict(raw + subs))))


# ============================================================================ tower
def zero2(p):
    return F2(F(p, {}), F(p, {}))


class F2:
    __slots__ = ("c0", "c1")

    def __init__(self, c0, c1):
        self.c0, self.c1 = c0, c1

    def __add__(s, o):
        return F2(s.c0 + o.c0, s.c1 + o.c1)

    def __sub__(s, o):
        return F2(s.c0 - o.c0, s.c1 - o.c1)

    def __neg__(s):
        return F2(-s.c0, -s.c1)

    def scale(s, k):
        return F2(s.c0.scale(k), s.c1.scale(k))

    def is_zero(s):
        return not s.c0.t and not s.c1.t

    def mul(s, o, kara=False):
        if s.is_zero() or o.is_zero():
            return zero2(s.c0.p)
        a0, a1, b0, b1 = s.c0, s.c1, o.c0, o.c1
        if kara:
            v0, v1 = a0 * b0, a1 * b1
            return F2(v0 - v1, (a0 + a1) * (b0 + b1) - v0 - v1)
        return F2(a0 * b0 - a1 * b1, a0 * b1 + a1 * b0)

    def sqr(s):
        a0, a1 = s.c0, s.c1
        return F2((a0 + a1) * (a0 - a1), (a0 * a1).scale(2))

    def mul_fp(s, x):
        return F2(s.c0 * x, s.c1 * x)

    def mul_xi(s):  # (9 + i)(a0 + a1 i) = (9 a0 - a1) + (a0 + 9 a1) i
        return F2(s.c0.scale(9) - s.c1, s.c0 + s.c1.scale(9))

    def conj(s):
        return F2(s.c0, -s.c1)

    def mul_const(s, c):
        p = s.c0.p
        k0, k1 = c[0] % P, c[1] % P
        r0, r1 = F(p, {}), F(p, {})
        if k0:
            g = p.fconst(k0)
            r0 = r0 + s.c0 * g
            r1 = r1 + s.c1 * g
        if k1:
            g = p.fconst(k1)
            r0 = r0 - s.c1 * g
            r1 = r1 + s.c0 * g
        return F2(r0, r1)


class F6:
    __slots__ = ("c",)

    def __init__(self, c0, c1, c2):
        self.c = (c0, c1, c2)

    def __add__(s, o):
        return F6(*(x + y for x, y in zip(s.c, o.c)))

    def __sub__(s, o):
        return F6(*(x - y for x, y in zip(s.c, o.c)))

    def __neg__(s):
        return F6(*(-x for x in s.c))

    def mul(s, o, kara2=True):
        a0, a1, a2 = s.c
        b0, b1, b2 = o.c
        v0, v1, v2 = a0.mul(b0, kara2), a1.mul(b1, kara2), a2.mul(b2, kara2)
        c0 = v0 + ((a1 + a2).mul(b1 + b2, kara2) - v1 - v2).mul_xi()
        c1 = (a0 + a1).mul(b0 + b1, kara2) - v0 - v1 + v2.mul_xi()
        c2 = (a0 + a2).mul(b0 + b2, kara2) - v0 + v1 - v2
        return F6(c0, c1, c2)

    def mul_v(s):  # v (c0 + c1 v + c2 v^2) = xi c2 + c0 v + c1 v^2
        return F6(s.c[2].mul_xi(), s.c[0], s.c[1])


class F12:
    __slots__ = ("a", "b")

    def __init__(self, a, b):
        self.a, self.b = a, b

    def coeffs(self):  # memory order c0.c0.c0, c0.c0.c1, ..., c1.c2.c1
        out = []
        for h in (self.a, self.b):
            for q in h.c:
                out += [q.c0, q.c1]
        return out

    @staticmethod
    def of(cs):
        f2 = [F2(cs[2 * j], cs[2 * j + 1]) for j in range(6)]
        return F12(F6(*f2[:3]), F6(*f2[3:]))

    def mul(s, o, kara2=True):
        t0, t1 = s.a.mul(o.a, kara2), s.b.mul(o.b, kara2)
        c1 = (s.a + s.b).mul(o.a + o.b, kara2) - t0 - t1
        return F12(t0 + t1.mul_v(), c1)

    def sqr(s, kara2=True):
        # complex squaring over F_p6: t = a b, c0 = (a + b)(a + v b) - t - v t, c1 = 2t
        a, b = s.a, s.b
        t = a.mul(b, kara2)
        m = (a + b).mul(a + b.mul_v(), kara2)
        return F12(m - t - t.mul_v(), t + t)

    def conj(s):
        return F12(s.a, -s.b)


# ============================================================================ constants
def f2mul_int(a, b):
    return ((a[0] * b[0] - a[1] * b[1]) % P, (a[0] * b[1] + a[1] * b[0]) % P)


def f2pow_int(a, e):
    r = (1, 0)
    while e:
        if e & 1:
            r = f2mul_int(r, a)
        a = f2mul_int(a, a)
        e >>= 1
    return r


def f2inv_int(a):
    n = pow(a[0] * a[0] + a[1] * a[1], -1, P)
    return (a[0] * n % P, -a[1] * n % P)


XI = (9, 1)
TWIST_B = f2mul_int((3, 0), f2inv_int(XI))     # b' = 3 / xi
B3 = f2mul_int((3, 0), TWIST_B)                # 3 b'
B9 = f2mul_int((9, 0), TWIST_B)                # 9 b'
GAM1 = [f2pow_int(XI, k * (P - 1) // 6) for k in range(6)]
GAM2 = [f2pow_int(XI, k * (P * P - 1) // 6) for k in range(6)]
GAM3 = [f2pow_int(XI, k * (P**3 - 1) // 6) for k in range(6)]
assert all(g[1] == 0 for g in GAM2)
FROB_TX, FROB_TY = GAM1[2], GAM1[3]            # twist Frobenius: (conj(x) tx, conj(y) ty)
FROB2_TX = f2pow_int(XI, (P * P - 1) // 3)
FROB2_TY = f2pow_int(XI, (P * P - 1) // 2)
assert FROB2_TX[1] == 0 and FROB2_TY[1] == 0


def frob12(f, e):
    """f^{p^e}, e = 1, 2, 3: the F_p2 coefficient of w^k (k = 2q + h) maps to conj^e(c) gamma_e[k]"""
    p = f.a.c[0].c0.p
    out = []
    for h, half in enumerate((f.a, f.b)):
        for q, c in enumerate(half.c):
            k = 2 * q + h
            if e & 1:
                c = c.conj()
            if k == 0:
                out.append(c)
            elif e == 2:
                g = p.fconst(GAM2[k][0])
                out.append(F2(c.c0 * g, c.c1 * g))
            else:
                out.append(c.mul_const(GAM1[k] if e == 1 else GAM3[k]))
    return F12(F6(*out[:3]), F6(*out[3:]))


# ============================================================================ pairing formulas
def line_dbl(T, xP, yP):
    """T = (X, Y, Z) homogeneous projective on y^2 = x^3 + b'.  Returns 2T (scaled by 4)
    and the tangent at T evaluated at P up to an F_p2 factor, as (l0, l1, l3) meaning
    l0 + l1 w + l3 w^3:  l0 = 2YZ yP, l1 = -3X^2 xP, l3 = Y^2 - 3b'Z^2."""
    X, Y, Z = T
    XX, YY, ZZ = X.sqr(), Y.sqr(), Z.sqr()
    XY, YZ = X.mul(Y), Y.mul(Z)
    F9 = ZZ.mul_const(B9)                  # 9 b' Z^2
    E = ZZ.mul_const(B3)                   # 3 b' Z^2
    X3 = XY.mul(YY - F9).scale(2)          # 2 XY (Y^2 - 9b'Z^2)
    Y3 = (YY + F9).sqr() - E.sqr().scale(12)
    Z3 = YY.mul(YZ).scale(8)               # 8 Y^3 Z
    l0 = YZ.scale(2).mul_fp(yP)
    l1 = XX.scale(-3).mul_fp(xP)
    l3 = YY - E
    return (X3, Y3, Z3), (l0, l1, l3)


def line_add(T, Q, xP, yP):
    """T projective, Q = (xQ, yQ) affine: T + Q and the line through T and Q at P:
    l0 = lam yP, l1 = -theta xP, l3 = theta xQ - lam yQ  (theta = Y - yQ Z, lam = X - xQ Z)."""
    X, Y, Z = T
    xQ, yQ = Q
    th = Y - yQ.mul(Z)
    la = X - xQ.mul(Z)
    C, D = th.sqr(), la.sqr()
    E2 = la.mul(D)
    F2_ = Z.mul(C)
    G2 = X.mul(D)
    H2 = E2 + F2_ - G2.scale(2)
    X3 = la.mul(H2)
    Y3 = th.mul(G2 - H2) - Y.mul(E2)
    Z3 = Z.mul(E2)
    l0 = la.mul_fp(yP)
    l1 = (-th).mul_fp(xP)
    l3 = th.mul(xQ) - la.mul(yQ)
    return (X3, Y3, Z3), (l0, l1, l3)


def line_to_f12(l):
    """l0 + l1 w + l3 w^3 = (l0, 0, 0) + (l1, l3, 0) w"""
    l0, l1, l3 = l
    z = zero2(l0.c0.p)
    return F12(F6(l0, z, z), F6(l1, l3, z))


def sparse01(x, b0, b1, kara2=True):
    """(x0 + x1 v + x2 v^2)(b0 + b1 v)"""
    x0, x1, x2 = x.c
    v0, v1 = x0.mul(b0, kara2), x1.mul(b1, kara2)
    c0 = v0 + x2.mul(b1, kara2).mul_xi()
    c1 = (x0 + x1).mul(b0 + b1, kara2) - v0 - v1
    c2 = x2.mul(b0, kara2) + v1
    return F6(c0, c1, c2)


def mul_by_line(f, l, kara2=True):
    """f (a + b w) with a = (l0, 0, 0), b = (l1, l3, 0)"""
    l0, l1, l3 = l
    f0, f1 = f.a, f.b
    t0 = F6(*(c.mul(l0, kara2) for c in f0.c))
    t1 = sparse01(f1, l1, l3, kara2)
    m = sparse01(f0 + f1, l0 + l1, l3, kara2)
    return F12(t0 + t1.mul_v(), m - t0 - t1)


def line_mul_line(la, lb):
    """(a0 + a1 w + a3 w^3)(b0 + b1 w + b3 w^3), w^6 = xi:
    w^0: a0b0; w^1: a0b1 + a1b0; w^2: a1b1; w^3: a0b3 + a3b0; w^4: a1b3 + a3b1; w^6 -> xi: a3b3"""
    a0, a1, a3 = la
    b0, b1, b3 = lb
    p = a0.c0.p
    z = zero2(p)
    t00, t11, t33 = a0.mul(b0), a1.mul(b1), a3.mul(b3)
    c = {0: t00 + t33.mul_xi(), 1: a0.mul(b1) + a1.mul(b0), 2: t11, 3: a0.mul(b3) + a3.mul(b0),
         4: a1.mul(b3) + a3.mul(b1), 5: z}
    # w^k, k = 2q + h  ->  (h, q)
    h0 = F6(c[0], c[2], c[4])
    h1 = F6(c[1], c[3], c[5])
    return F12(h0, h1)


def twist_frob(Q):
    xQ, yQ = Q
    return (xQ.conj().mul_const(FROB_TX), yQ.conj().mul_const(FROB_TY))


def twist_frob2_neg(Q):
    xQ, yQ = Q
    p = xQ.c0.p
    gx, gy = p.fconst(FROB2_TX[0]), p.fconst(-FROB2_TY[0])
    return (F2(xQ.c0 * gx, xQ.c1 * gx), F2(yQ.c0 * gy, yQ.c1 * gy))


def naf(k):
    d = []
    while k:
        if k & 1:
            z = 2 - (k % 4)
            k -= z
        else:
            z = 0
        d.append(z)
        k //= 2
    return d[::-1]


ATE = 6 * U + 2
ATE_NAF = naf(ATE)          # most significant first, leading digit 1


# ============================================================================ programs
def f2_in(p, name):
    return F2(p.inp(name + ".0"), p.inp(name + ".1"))


def f12_in(p, name):
    return F12.of([p.inp("%s.%d" % (name, k)) for k in range(12)])


def f2_out(p, name, v):
    p.out(name + ".0", v.c0)
    p.out(name + ".1", v.c1)


def f12_out(p, name, f):
    for k, c in enumerate(f.coeffs()):
        p.out("%s.%d" % (name, k), c)


def line_in(p, name):
    return tuple(f2_in(p, "%s.%d" % (name, k)) for k in range(3))


def line_out(p, name, l):
    for k, c in enumerate(l):
        f2_out(p, "%s.%d" % (name, k), c)


def pt_in(p, name):
    return tuple(f2_in(p, "%s.%s" % (name, c)) for c in "XYZ")


def pt_out(p, name, T):
    for c, v in zip("XYZ", T):
        f2_out(p, "%s.%s" % (name, c), v)


def miller_programs():
    """Bodies of the pipelined Miller loop over the NAF digits d_1 .. d_n of 6u + 2
    (d_0 = 1 is the starting T = Q).  State: f, T, pending lines L1 (and L2 when an
    addition followed the doubling), P = (xP, yP), Q = (xQ, yQ), nyQ = -yQ.

      ml_start<a>    : (T, L1) = dbl(Q); addition step a (0, +1, -1) gives L2
      ml_body<n><a>  : f = f^2 * pending (f = pending on the first body);
                       (T, L1) = dbl(T); addition step a gives L2
      ml_final<n>    : f = f^2 * pending, times the lines of T + pi(Q) and of
                       (T + pi(Q)) - pi^2(Q)
    n is the number of pending lines (1 or 2)."""
    progs = {}

    def common(p):
        xP, yP = p.inp("xP"), p.inp("yP")
        xQ, yQ = f2_in(p, "xQ"), f2_in(p, "yQ")
        return xP, yP, (xQ, yQ)

    def add_step(p, T, Q, a, xP, yP):
        if a == 1:
            return line_add(T, Q, xP, yP)
        return line_add(T, (Q[0], -Q[1]), xP, yP)

    for a in (0, 1, -1):
        p = Prog("ml_start%s" % "0pm"[a])
        xP, yP, Q = common(p)
        one = F2(p.fconst(1), p.fconst(0))
        T, l1 = line_dbl((Q[0], Q[1], one), xP, yP)
        if a:
            T, l2 = add_step(p, T, Q, a, xP, yP)
        pt_out(p, "T", T)
        line_out(p, "L1", l1)
        if a:
            line_out(p, "L2", l2)
        progs[p.name] = p
    for npend in (1, 2):
        for a in (0, 1, -1):
            for first in (0, 1):
                p = Prog("ml_body%d%s%s" % (npend, "0pm"[a], "_first" if first else ""))
                xP, yP, Q = common(p)
                L1 = line_in(p, "L1")
                L2 = line_in(p, "L2") if npend == 2 else None
                if first:
                    f = line_to_f12(L1) if npend == 1 else line_mul_line(L1, L2)
                else:
                    f = f12_in(p, "f").sqr()
                    f = mul_by_line(f, L1) if npend == 1 else f.mul(line_mul_line(L1, L2))
                f12_out(p, "f", f)
                T, l1 = line_dbl(pt_in(p, "T"), xP, yP)
                if a:
                    T, l2 = add_step(p, T, Q, a, xP, yP)
                pt_out(p, "T", T)
                line_out(p, "L1", l1)
                if a:
                    line_out(p, "L2", l2)
                progs[p.name] = p
    for npend in (1, 2):
        p = Prog("ml_final%d" % npend)
        xP, yP, Q = common(p)
        L1 = line_in(p, "L1")
        L2 = line_in(p, "L2") if npend == 2 else None
        f = f12_in(p, "f").sqr()
        f = mul_by_line(f, L1) if npend == 1 else f.mul(line_mul_line(L1, L2))
        T = pt_in(p, "T")
        T, la = line_add(T, twist_frob(Q), xP, yP)
        _, lb = line_add(T, twist_frob2_neg(Q), xP, yP)
        f12_out(p, "f", f.mul(line_mul_line(la, lb)))
        progs[p.name] = p
    return progs


def miller_sequence():
    d = ATE_NAF
    assert d[0] == 1
    seq = ["ml_start%s" % "0pm"[d[1]]]
    pend = 2 if d[1] else 1
    for i in range(2, len(d)):
        seq.append("ml_body%d%s%s" % (pend, "0pm"[d[i]], "_first" if i == 2 else ""))
        pend = 2 if d[i] else 1
    seq.append("ml_final%d" % pend)
    return seq


MILLER_STATE = (["xP", "yP", "xQ.0", "xQ.1", "yQ.0", "yQ.1"] + ["f.%d" % k for k in range(12)]
                + ["T.%s.%d" % (c, k) for c in "XYZ" for k in (0, 1)]
                + ["L%d.%d.%d" % (n, j, k) for n in (1, 2) for j in range(3) for k in (0, 1)])


def cyclo_sqr(X):
    """Granger-Scott squaring of a cyclotomic element over the three F_p4 pairs
    (w^0, w^3), (w^1, w^4), (w^2, w^5), with s = w^3, s^2 = xi."""
    a, b = X.a, X.b
    g = {0: a.c[0], 2: a.c[1], 4: a.c[2], 1: b.c[0], 3: b.c[1], 5: b.c[2]}   # by power of w

    def fp4_sqr(x, y):  # (x + y s)^2 with s^2 = xi: (x^2 + xi y^2, 2xy)
        t0, t1 = x.sqr(), y.sqr()
        return t0 + t1.mul_xi(), (x + y).sqr() - t0 - t1

    z0, z1 = g[0], g[3]
    z2, z3 = g[1], g[4]
    z4, z5 = g[2], g[5]
    t0, t1 = fp4_sqr(z0, z1)
    n0 = (t0 - z0).scale(2) + t0
    n1 = (t1 + z1).scale(2) + t1
    t0, t1 = fp4_sqr(z2, z3)
    t2, t3 = fp4_sqr(z4, z5)
    n4 = (t0 - z4).scale(2) + t0
    n5 = (t1 + z5).scale(2) + t1
    t0 = t3.mul_xi()
    n2 = (t0 + z2).scale(2) + t0
    n3 = (t2 - z3).scale(2) + t2
    h = {0: n0, 3: n1, 1: n2, 4: n3, 2: n4, 5: n5}
    return F12(F6(h[0], h[2], h[4]), F6(h[1], h[3], h[5]))


def fe_programs():
    progs = {}

    def mk(name, fn, n_in):
        p = Prog(name)
        X = f12_in(p, "X")
        args = [X] + ([f12_in(p, "Y")] if n_in == 2 else [])
        f12_out(p, "D", fn(*args))
        progs[name] = p

    mk("f12_mul", lambda X, Y: X.mul(Y), 2)
    mk("f12_csqr", cyclo_sqr, 1)
    mk("f12_csqr_mul", lambda X, Y: cyclo_sqr(X).mul(Y), 2)
    # (the conjugate is the inverse in the cyclotomic subgroup: its sign changes fold into
    # the product's coefficients, so this costs the levels of f12_csqr_mul)
    mk("f12_csqr_cmul", lambda X, Y: cyclo_sqr(X).mul(Y.conj()), 2)
    mk("f12_frob1", lambda X: frob12(X, 1), 1)
    mk("f12_frob2", lambda X: frob12(X, 2), 1)
    mk("f12_frob3", lambda X: frob12(X, 3), 1)
    mk("f12_conj", lambda X: X.conj(), 1)
    mk("f12_conj_mul", lambda X, Y: X.conj().mul(Y), 2)
    mk("f12_frob2_mul", lambda X, Y: frob12(X, 2).mul(Y), 2)
    # norm: n6 = X conj(X) = a^2 - v b^2 in F_p6; the F_p6 inverse of n6 is (A, B, C) / n2
    # with A = c0^2 - xi c1 c2, B = xi c2^2 - c0 c1, C = c1^2 - c0 c2,
    # n2 = c0 A + xi (c2 B + c1 C); t = n2 conj(n2) in F_p
    p = Prog("fe_norm")
    X = f12_in(p, "X")
    n6 = X.a.mul(X.a) - X.b.mul(X.b).mul_v()
    c0, c1, c2 = n6.c
    A = c0.sqr() - c1.mul(c2).mul_xi()
    B = c2.sqr().mul_xi() - c0.mul(c1)
    C = c1.sqr() - c0.mul(c2)
    n2 = c0.mul(A) + (c2.mul(B) + c1.mul(C)).mul_xi()
    for nm, v in (("nA", A), ("nB", B), ("nC", C), ("n2", n2)):
        f2_out(p, nm, v)
    p.out("t", n2.c0 * n2.c0 + n2.c1 * n2.c1)
    progs[p.name] = p
    # easy part from tinv = t^{-1}: n6^{-1} = (A, B, C) conj(n2) tinv and
    # conj(X) X^{-1} = conj(X)^2 n6^{-1}
    p = Prog("fe_easy")
    X = f12_in(p, "X")
    A, B, C, n2 = (f2_in(p, nm) for nm in ("nA", "nB", "nC", "n2"))
    ti = p.inp("tinv")
    n2i = n2.conj().mul_fp(ti)
    n6i = F6(A.mul(n2i), B.mul(n2i), C.mul(n2i))
    cx2 = X.conj().sqr()
    f12_out(p, "D", F12(cx2.a.mul(n6i), cx2.b.mul(n6i)))
    progs[p.name] = p
    return progs


UNAF = naf(U)


def wnaf(k, w):
    """width-w signed digits of k (odd digits |d| < 2^(w-1), most significant first)"""
    d = []
    while k:
        if k & 1:
            z = k % (1 << w)
            if z >= 1 << (w - 1):
                z -= 1 << w
            k -= z
        else:
            z = 0
        d.append(z)
        k //= 2
    return d[::-1]


UW4 = wnaf(U, 4)


def fe_sequence():
    """Final exponentiation f^((p^12 - 1)/r) as calls of the F_p12 programs on buffers of
    12 slots: easy part conj(f) f^{-1}, then (.)^{p^2} (.); hard part through f^u, f^{u^2},
    f^{u^3} and the p-power split (p^4 - p^2 + 1)/r = l0 + l1 p + l2 p^2 + l3 p^3 with
    l3 = 1, l2 = 6u^2 + 1, l1 = -36u^3 - 18u^2 - 12u + 1, l0 = -36u^3 - 30u^2 - 18u - 2.
    Entries are (program, X, Y, D) buffer numbers; "INV" inverts the norm on one lane.
    Buffer 0 holds the input; the result is left in the buffer returned."""
    seq = []
    nbuf = [1]
    free = []

    def alloc():
        if free:
            return free.pop()
        nbuf[0] += 1
        return nbuf[0] - 1

    def call(prog, X, Y=None):
        D = alloc()
        seq.append((prog, X, X if Y is None else Y, D))
        return D

    def release(*bs):
        for b in bs:
            free.append(b)

    seq.append(("fe_norm", 0, 0, 0))
    seq.append(("INV", 0, 0, 0))
    f1 = call("fe_easy", 0)
    f = call("f12_frob2_mul", f1, f1)
    release(f1)

    def pow_u(x):
        # x^u over the width-4 signed digits of u (14 nonzero of 63 against 24 for the NAF):
        # the odd powers x^3, x^5, x^7 first, a negative digit multiplies by the conjugate
        x2 = call("f12_csqr", x)
        tab = {1: x}
        for e in (3, 5, 7):
            tab[e] = call("f12_mul", tab[e - 2], x2)
        release(x2)
        assert UW4[0] == 1
        acc = x
        for d in UW4[1:]:
            if d == 0:
                nxt = call("f12_csqr", acc)
            else:
                nxt = call("f12_csqr_mul" if d > 0 else "f12_csqr_cmul", acc, tab[abs(d)])
            if acc != x:
                release(acc)
            acc = nxt
        release(tab[3], tab[5], tab[7])
        return acc

    a = pow_u(f)
    b = pow_u(a)
    c = pow_u(b)
    c2 = call("f12_csqr", c)
    c4 = call("f12_csqr", c2)
    release(c2)
    c8 = call("f12_csqr", c4)
    release(c4)
    c9 = call("f12_mul", c8, c)
    release(c8, c)
    c18 = call("f12_csqr", c9)
    release(c9)
    c36 = call("f12_csqr", c18)
    release(c18)
    b2 = call("f12_csqr", b)
    b3 = call("f12_mul", b2, b)
    release(b2, b)
    b6 = call("f12_csqr", b3)
    release(b3)
    b12 = call("f12_csqr", b6)
    b18 = call("f12_mul", b12, b6)
    b30 = call("f12_mul", b18, b12)
    release(b12)
    a2 = call("f12_csqr", a)
    a3 = call("f12_mul", a2, a)
    release(a2, a)
    a6 = call("f12_csqr", a3)
    release(a3)
    a12 = call("f12_csqr", a6)
    a18 = call("f12_mul", a12, a6)
    release(a6)
    f2 = call("f12_csqr", f)
    t = call("f12_mul", c36, b30)
    release(b30)
    u_ = call("f12_mul", a18, f2)
    release(a18, f2)
    t0n = call("f12_mul", t, u_)                 # conj(t0n) = f^{l0}
    release(t, u_)
    v = call("f12_mul", c36, b18)
    release(c36, b18)
    v2 = call("f12_mul", v, a12)
    release(v, a12)
    t1 = call("f12_conj_mul", v2, f)             # f^{l1}
    release(v2)
    t2 = call("f12_mul", b6, f)                  # f^{l2}
    release(b6)
    ft1 = call("f12_frob1", t1)
    release(t1)
    r1 = call("f12_conj_mul", t0n, ft1)          # f^{l0} (f^{l1})^p
    release(t0n, ft1)
    f3 = call("f12_frob3", f)
    release(f)
    r2 = call("f12_frob2_mul", t2, f3)           # (f^{l2})^{p^2} f^{p^3}
    release(t2, f3)
    res = call("f12_mul", r1, r2)
    return seq, res, nbuf[0]


# ============================================================================ G2 scalar multiplication (GLS)
# psi(x, y) = (conj(x) tx, conj(y) ty) acts on G2 as multiplication by lam = p mod r = 6u^2.
# A scalar k is split as k = sum_j k_j lam^j (mod r), |k_j| < 2^65, with the reduced lattice
# basis below (rows b satisfy b0 + b1 lam + b2 lam^2 + b3 lam^3 = 0 mod r) and Babai rounding
# with the constants G (c_i = floor(k G_i / 2^256), k_j = [j = 0] k - sum_i c_i b_ij).
GLS_B = [[2 * U + 1, 0, 2 * U, 1], [2 * U, U + 1, -U, U], [U + 1, U, U, -2 * U], [2 * U + 1, -U, -(U + 1), -U]]


def gls_constants():
    from fractions import Fraction
    n = 4
    M = [[Fraction(x) for x in row] + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(GLS_B)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    alpha = M[0][n:]
    G = [round(a * 2**256) for a in alpha]
    assert all(0 <= g < 2**192 for g in G)
    return G


def gls_decompose(k):
    G = gls_constants()
    c = [(k * g) >> 256 for g in G]
    return [(k if j == 0 else 0) - sum(c[i] * GLS_B[i][j] for i in range(4)) for j in range(4)]


def j_dbl(T):
    X, Y, Z = T
    A, B = X.sqr(), Y.sqr()
    C = B.sqr()
    D = ((X + B).sqr() - A - C).scale(2)
    E = A.scale(3)
    X3 = E.sqr() - D.scale(2)
    Y3 = E.mul(D - X3) - C.scale(8)
    Z3 = Y.mul(Z).scale(2)
    return (X3, Y3, Z3)


def j_add(T1, T2):
    """add-2007-bl; returns the sum and (H, r): H = 0 means equal x, then r = 0 means equal points"""
    X1, Y1, Z1 = T1
    X2, Y2, Z2 = T2
    Z1Z1, Z2Z2 = Z1.sqr(), Z2.sqr()
    U1, U2 = X1.mul(Z2Z2), X2.mul(Z1Z1)
    S1, S2 = Y1.mul(Z2).mul(Z2Z2), Y2.mul(Z1).mul(Z1Z1)
    H = U2 - U1
    I = H.scale(2).sqr()
    J = H.mul(I)
    rr = (S2 - S1).scale(2)
    V = U1.mul(I)
    X3 = rr.sqr() - J - V.scale(2)
    Y3 = rr.mul(V - X3) - S1.mul(J).scale(2)
    Z3 = ((Z1 + Z2).sqr() - Z1Z1 - Z2Z2).mul(H)
    return (X3, Y3, Z3), H, S2 - S1


def j_madd(T1, A):
    """madd-2007-bl: T1 Jacobian plus A = (x2, y2) affine"""
    X1, Y1, Z1 = T1
    x2, y2 = A
    Z1Z1 = Z1.sqr()
    U2 = x2.mul(Z1Z1)
    S2 = y2.mul(Z1).mul(Z1Z1)
    H = U2 - X1
    HH = H.sqr()
    I = HH.scale(4)
    J = H.mul(I)
    rr = (S2 - Y1).scale(2)
    V = X1.mul(I)
    X3 = rr.sqr() - J - V.scale(2)
    Y3 = rr.mul(V - X3) - Y1.mul(J).scale(2)
    Z3 = (Z1 + H).sqr() - Z1Z1 - HH
    return (X3, Y3, Z3), H, S2 - Y1


def jac_in(p, name):
    return tuple(F2(p.inp("%s.%d" % (name, 2 * c)), p.inp("%s.%d" % (name, 2 * c + 1))) for c in range(3))


def jac_out(p, name, T):
    for c, v in enumerate(T):
        p.out("%s.%d" % (name, 2 * c), v.c0)
        p.out("%s.%d" % (name, 2 * c + 1), v.c1)


def g2_programs():
    progs = {}
    # psi images of Q (B0 = Q)
    p = Prog("g2_psi")
    Q = (f2_in(p, "xQ"), f2_in(p, "yQ"))
    Bj = Q
    for j in (1, 2, 3):
        Bj = twist_frob(Bj)
        f2_out(p, "B%d.x" % j, Bj[0])
        f2_out(p, "B%d.y" % j, Bj[1])
    progs[p.name] = p
    # table TB[d] = sum_{j in d} B_j (Jacobian), the single-bit entries with Z = 1
    p = Prog("g2_table")
    one = F2(p.fconst(1), p.fconst(0))
    B = [(f2_in(p, "xQ"), f2_in(p, "yQ"))] + [(f2_in(p, "B%d.x" % j), f2_in(p, "B%d.y" % j)) for j in range(1, 4)]
    TB = {}
    for j in range(4):
        TB[1 << j] = (B[j][0], B[j][1], one)
    for d in range(1, 16):
        if d & (d - 1) == 0:
            continue
        lo = d & -d
        TB[d], _, _ = j_add(TB[d - lo], TB[lo])
    for d in range(1, 16):
        jac_out(p, "TB%d" % d, TB[d])
    progs[p.name] = p
    p = Prog("g2_dbl")
    jac_out(p, "T", j_dbl(jac_in(p, "T")))
    progs[p.name] = p
    p = Prog("g2_add")
    T, H, r = j_add(jac_in(p, "T"), jac_in(p, "A"))
    jac_out(p, "T", T)
    f2_out(p, "H", H)
    f2_out(p, "RR", r)
    progs[p.name] = p
    p = Prog("g2_madd")
    T, H, r = j_madd(jac_in(p, "T"), (F2(p.inp("A.0"), p.inp("A.1")), F2(p.inp("A.2"), p.inp("A.3"))))
    jac_out(p, "T", T)
    f2_out(p, "H", H)
    f2_out(p, "RR", r)
    progs[p.name] = p
    # to affine: t = N(Z); then Zi = conj(Z) / t, x = X Zi^2, y = Y Zi^3
    p = Prog("g2_norm")
    Z = F2(p.inp("T.4"), p.inp("T.5"))
    p.out("t", Z.c0 * Z.c0 + Z.c1 * Z.c1)
    progs[p.name] = p
    p = Prog("g2_aff")
    X, Y, Z = jac_in(p, "T")
    Zi = Z.conj().mul_fp(p.inp("tinv"))
    Zi2 = Zi.sqr()
    f2_out(p, "ax", X.mul(Zi2))
    f2_out(p, "ay", Y.mul(Zi2.mul(Zi)))
    progs[p.name] = p
    return progs


# G1 (y^2 = x^3 + 3 over F_p) on the engine: GLV with phi(x, y) = (beta x, y)
GLV_BETA = 0x59E26BCEA0D48BACD4F263F1ACDB5C4F5763473177FFFFFE
GLV_LAM = 0xB3C4D79D41A917585BFC41088D8DAAA78B17EA66B99C90DD


def g1_jin(p, name):
    return tuple(p.inp("%s.%d" % (name, c)) for c in range(3))


def g1_jout(p, name, T):
    for c, v in enumerate(T):
        p.out("%s.%d" % (name, c), v)


def g1_programs():
    progs = {}
    p = Prog("g1_phi")
    p.out("B1.x", p.inp("xP") * p.fconst(GLV_BETA))
    progs[p.name] = p
    # table TB[d0 + 4 d1] = d0 B0 + d1 B1 (Jacobian) for the joint 2-bit windows; B0 in
    # (xP, yP), B1 in (B1.x, B1.y), signs applied by the caller
    p = Prog("g1_table")
    one = p.fconst(1)
    B0 = (p.inp("xP"), p.inp("yP"))
    B1 = (p.inp("B1.x"), p.inp("B1.y"))
    TB = {1: (B0[0], B0[1], one), 4: (B1[0], B1[1], one)}
    TB[2] = j_dbl(TB[1])
    TB[3], _, _ = j_madd(TB[2], B0)
    TB[8] = j_dbl(TB[4])
    TB[12], _, _ = j_madd(TB[8], B1)
    for d1 in (1, 2, 3):
        for d0 in (1, 2, 3):
            TB[d0 + 4 * d1], _, _ = j_add(TB[4 * d1], TB[d0])
    for d in range(1, 16):
        g1_jout(p, "TB%d" % d, TB[d])
    progs[p.name] = p
    p = Prog("g1_dbl")
    g1_jout(p, "T", j_dbl(g1_jin(p, "T")))
    progs[p.name] = p
    p = Prog("g1_dbl2")
    g1_jout(p, "T", j_dbl(j_dbl(g1_jin(p, "T"))))
    progs[p.name] = p
    p = Prog("g1_dbl2_add")
    T, H, r = j_add(j_dbl(j_dbl(g1_jin(p, "T"))), g1_jin(p, "A"))
    g1_jout(p, "T", T)
    p.out("H", H)
    p.out("RR", r)
    progs[p.name] = p
    p = Prog("g1_add")
    T, H, r = j_add(g1_jin(p, "T"), g1_jin(p, "A"))
    g1_jout(p, "T", T)
    p.out("H", H)
    p.out("RR", r)
    progs[p.name] = p
    p = Prog("g1_madd")
    T, H, r = j_madd(g1_jin(p, "T"), (p.inp("A.0"), p.inp("A.1")))
    g1_jout(p, "T", T)
    p.out("H", H)
    p.out("RR", r)
    progs[p.name] = p
    p = Prog("g1_aff")
    X, Y, Z = g1_jin(p, "T")
    zi = p.inp("tinv")
    zi2 = zi * zi
    p.out("ax", X * zi2)
    p.out("ay", Y * (zi2 * zi))
    progs[p.name] = p
    return progs


G1_STATE = (["T.%d" % k for k in range(3)] + ["xP", "yP", "B1.x", "B1.y"]
            + ["TB%d.%d" % (d, k) for d in range(1, 16) for k in range(3)]
            + ["H", "RR", "tinv", "ax", "ay"])


G2_STATE = (["T.%d" % k for k in range(6)] + ["xQ.0", "xQ.1", "yQ.0", "yQ.1"]
            + ["B%d.%s.%d" % (j, c, k) for j in range(1, 4) for c in "xy" for k in (0, 1)]
            + ["TB%d.%d" % (d, k) for d in range(1, 16) for k in range(6)]
            + ["H.0", "H.1", "RR.0", "RR.1", "t", "tinv", "ax.0", "ax.1", "ay.0", "ay.1"])


# ============================================================================ scheduling
def operands(v):
    if v[0] == "mul":
        return tuple(k for k, _ in v[1]) + tuple(k for k, _ in v[2])
    if v[0] == "lin":
        return tuple(k for k, _ in v[1])
    return ()


# Cost of a level in cycles of the interpreter (one wavefront): a fixed part, a part per
# group of four term positions loaded (the union over the level's operations) and the
# Montgomery product of a level with products (measured on gfx950).
LEVEL_BASE, LEVEL_GROUP, LEVEL_MUL = 880, 430, 1310


def op_groups(v):
    """term groups an operation's encoding uses (see encode_op)"""
    if v[0] == "mul":
        na, nb = len(v[1]), len(v[2])
        return ((1 << -(-na // 4)) - 1) | (((1 << -(-nb // 4)) - 1) << 2)
    return (1 << -(-len(v[1]) // 4)) - 1


def levels_cost(p, levels):
    c = 0
    for ops in levels:
        gm = 0
        mul = False
        for i in ops:
            gm |= op_groups(p.vals[i])
            mul = mul or p.vals[i][0] == "mul"
        c += LEVEL_BASE + LEVEL_GROUP * bin(gm).count("1") + (LEVEL_MUL if mul else 0)
    return c


def schedule(p, lanes=LANES):
    """The cheaper of the two stage schedules below (as early / as late as possible)."""
    a = schedule_phases(p, lanes, late=False)
    b = schedule_phases(p, lanes, late=True)
    return b if levels_cost(p, b[0]) <= levels_cost(p, a[0]) else a


def schedule_phases(p, lanes=LANES, late=False):
    """Stage scheduling: a product's stage is its multiplicative depth (products on the
    longest path from the inputs), so all products of one depth share one level (split
    only beyond the lane count).  Additions run in a phase between two product levels,
    levelised by their depth within the phase: the phase right after the products they
    depend on, or (late) the last phase before their first use, so that additions that
    only feed outputs or later products share levels that exist anyway."""
    vals = p.vals
    n = len(vals)
    live = [False] * n
    stack = list(p.outputs.values())
    while stack:
        i = stack.pop()
        if live[i]:
            continue
        live[i] = True
        stack.extend(operands(vals[i]))
    is_op = [live[i] and vals[i][0] in ("mul", "lin") for i in range(n)]
    md = [0] * n      # multiplicative depth
    ld = [0] * n      # depth in additions since the last product
    for i in range(n):
        if not is_op[i]:
            continue
        ops_ = [a for a in operands(vals[i]) if is_op[a]]
        if vals[i][0] == "mul":
            md[i] = 1 + max([md[a] for a in ops_] + [0])
            ld[i] = 0
        else:
            m = max([md[a] for a in ops_] + [0])
            md[i] = m
            ld[i] = 1 + max([ld[a] for a in ops_ if md[a] == m] + [0])
    # a product at depth k must follow the additions of phase k-1 that feed it
    maxd = max([md[i] for i in range(n) if is_op[i]] + [0])
    phase = list(md)
    if late:
        users = [[] for _ in range(n)]
        for i in range(n):
            if is_op[i]:
                for a in set(operands(vals[i])):
                    users[a].append(i)
        outset = set(p.outputs.values())
        for i in reversed(range(n)):
            if not (is_op[i] and vals[i][0] == "lin"):
                continue
            lim = maxd if i in outset else 1 << 30
            for c in users[i]:
                lim = min(lim, md[c] - 1 if vals[c][0] == "mul" else phase[c])
            assert md[i] <= lim < 1 << 30
            phase[i] = lim
        for i in range(n):
            if is_op[i] and vals[i][0] == "lin":
                ld[i] = 1 + max([ld[a] for a in operands(vals[i])
                                 if is_op[a] and vals[a][0] == "lin" and phase[a] == phase[i]] + [0])
    buckets = {}
    for i in range(n):
        if not is_op[i]:
            continue
        if vals[i][0] == "mul":
            key = (md[i] - 1, 1 << 20)          # after phase md-1 additions
        else:
            key = (phase[i], ld[i])
        buckets.setdefault(key, []).append(i)
    levels = []
    level_of = [-1] * n
    for key in sorted(buckets):
        ops_ = sorted(buckets[key])
        for k in range(0, len(ops_), lanes):
            L = len(levels)
            levels.append(ops_[k:k + lanes])
            for i in ops_[k:k + lanes]:
                level_of[i] = L
    return levels, level_of, live


def compile_prog(p, io_slot, const_slot, temp_base, temp_limit, lanes=LANES):
    """Schedule p and assign slots.  io_slot(name) gives the encoded slot of an input or
    output name (an output with the name of an input replaces it), const_slot(x) the slot
    of a constant.  Returns (levels of encoded op tuples, highest temp slot used + 1)."""
    levels, level_of, live = schedule(p, lanes)
    vals = p.vals
    n = len(vals)
    nlev = len(levels)
    slot = [None] * n
    for name, v in p.inputs.items():
        slot[v] = io_slot(name)
    for x, v in p.consts.items():
        slot[v] = const_slot(x)
    last = [-1] * n
    for i in range(n):
        if level_of[i] >= 0:
            for a in operands(vals[i]):
                last[a] = max(last[a], level_of[i])
    outs = {}
    for name, v in p.outputs.items():
        outs.setdefault(v, []).append(name)
    for v in outs:
        last[v] = nlev
    # last read of the value held in each io slot at entry
    held_read = {}
    for name, v in p.inputs.items():
        held_read[io_slot(name)] = last[v]
    free = list(range(temp_limit - 1, temp_base - 1, -1))
    busy = []
    used = temp_base
    copies = []
    for i in sorted((i for i in range(n) if level_of[i] >= 0), key=lambda i: (level_of[i], i)):
        L = level_of[i]
        keep = []
        for rl, s in busy:
            (free if rl <= L else keep).append(s if rl <= L else (rl, s))
        busy = keep
        names = outs.get(i, [])
        # write in place when this is the only output of the value and the slot's entry
        # value is not read after this level
        if len(names) == 1 and held_read.get(io_slot(names[0]), -1) <= L:
            slot[i] = io_slot(names[0])
            continue
        if not free:
            raise RuntimeError("%s: out of temp slots" % p.name)
        s = free.pop()
        used = max(used, s + 1)
        slot[i] = s
        busy.append((last[i], s))
        for nm in names:
            copies.append((nm, i))
    # outputs that are inputs or constants of the program, or that share a value
    for v, names in outs.items():
        if level_of[v] < 0:
            for nm in names:
                if slot[v] != io_slot(nm):
                    copies.append((nm, v))
    enc = []
    for ops in levels:
        row = []
        for i in ops:
            v = vals[i]
            if v[0] == "mul":
                za = (const_slot(0), 0)
                ta = tuple((slot[k], c) for k, c in v[1]) + (za,) * (ENC_SIDE - len(v[1]))
                row.append((OP_MUL, slot[i], ENC_SIDE, ta + tuple((slot[k], c) for k, c in v[2])))
            else:
                row.append((OP_LIN, slot[i], len(v[1]), tuple((slot[k], c) for k, c in v[1])))
        enc.append(row)
    if copies:
        row = [(OP_LIN, io_slot(nm), 1, ((slot[v], 1),)) for nm, v in copies]
        for k in range(0, len(row), lanes):
            enc.append(row[k:k + lanes])
    return enc, used


# ============================================================================ kernels
class Kernel:
    """programs that share one LDS slot map: named state slots, constants, temps"""

    def __init__(self, name, progs, state, segs=None, lanes=LANES):
        self.name = name
        self.state = {nm: i for i, nm in enumerate(state)}
        self.segs = segs or {}
        consts = sorted(set(x for p in progs.values() for x in p.consts) | {0, 1})
        self.cbase = len(state)
        self.cslot = {x: self.cbase + k for k, x in enumerate(consts)}
        self.consts = consts
        self.tbase = self.cbase + len(consts)
        self.progs = {}
        self.ntemps = self.tbase
        for nm, p in progs.items():
            enc, used = compile_prog(p, self.io_slot, lambda x: self.cslot[x % P], self.tbase, 512, lanes)
            self.progs[nm] = enc
            self.ntemps = max(self.ntemps, used)
        self.nslots = self.ntemps

    def io_slot(self, name):
        head = name.split(".")[0]
        if head in self.segs:
            seg = self.segs[head]
            assert 1 <= seg <= 3  # the interpreter packs the bases of segments 1..3 only
            off = int(name.split(".")[1])
            return (seg << 9) | off
        return self.state[name]


def encode_op(op):
    """384-bit op: kind (2) | dst (12) | group mask (4) | 16 x (slot 12 | coefficient 8,
    two's complement); a product multiplies the sum of terms [0, 8) by the sum of terms
    [8, 16); unused terms have slot 0 and coefficient 0.  The mask has bit g set when
    some operation of the level uses a term in positions 4g .. 4g + 3 (uniform over the
    level)."""
    kind, dst, gmask, terms = op
    assert 0 <= dst < 4096 and len(terms) <= ENC_NTERM and 0 <= gmask < 16
    # the interpreter adds 65536 p to each factor (or the sum): the scaled coefficient
    # magnitudes must stay below 32768 so that the sum is positive (slots are below 2p)
    if kind == OP_MUL:
        assert 32 * sum(abs(c) for _, c in terms[:ENC_SIDE]) < 32768 and sum(abs(c) for _, c in terms[ENC_SIDE:]) < 32768
    else:
        assert sum(abs(c) for _, c in terms) < 32768
    x = kind | (dst << 2) | (gmask << 14)
    for i, (s, c) in enumerate(terms):
        assert 0 <= s < 4096 and -KMAX <= c <= KMAX
        x |= ((s | ((c & 255) << 12)) << (18 + 20 * i))
    return x


def term_groups(op):
    """bit g set when op has a nonzero coefficient in term positions 4g .. 4g + 3"""
    m = 0
    for i, (_, c) in enumerate(op[3]):
        if c:
            m |= 1 << (i // 4)
    return m


OP_WORDS = 6


TRACE_LIMITS = ((8, 4), (12, 4), (16, 4), (8, 8), (12, 8), (16, 8))


def cheapest(make):
    """trace every program under each (NTERM, SIDE) limit and keep, per program, the trace
    whose schedule costs least"""
    global NTERM, SIDE
    best = {}
    saved = NTERM, SIDE
    for nt, sd in TRACE_LIMITS:
        NTERM, SIDE = nt, sd
        for nm, p in make().items():
            c = levels_cost(p, schedule(p)[0])
            if nm not in best or c < best[nm][0]:
                best[nm] = (c, p)
    NTERM, SIDE = saved
    return {nm: p for nm, (c, p) in best.items()}


_BUILT = []


def build_all():
    if not _BUILT:
        mk = Kernel("ml", cheapest(miller_programs), MILLER_STATE)
        fe_state = ["t", "tinv"] + ["%s.%d" % (nm, k) for nm in ("nA", "nB", "nC", "n2") for k in (0, 1)]
        fk = Kernel("fe", cheapest(fe_programs), fe_state, segs={"X": 1, "Y": 2, "D": 3})
        gk = Kernel("g2", cheapest(g2_programs), G2_STATE, segs={"A": 2})
        g1k = Kernel("g1", cheapest(g1_programs), G1_STATE, segs={"A": 2})
        _BUILT.append((mk, fk, gk, g1k))
    return _BUILT[0]


# ============================================================================ emission
def limbs(x):
    return [(x >> (32 * i)) & 0xFFFFFFFF for i in range(8)]


M29 = (1 << 29) - 1
OFF_MULT = 65536          # offset multiple of p added to every linear combination


def limbs29(x):
    return [(x >> (29 * i)) & M29 for i in range(9)]


def emit_radix():
    """constants of the radix-2^29 lane arithmetic"""
    o = []
    o.append("static constexpr uint32_t P29[9] = {%s};" % ", ".join("0x%08xu" % v for v in limbs29(P)))
    o.append("static constexpr uint32_t PINV29 = 0x%08xu;  // -p^{-1} mod 2^29" % ((-pow(P, -1, 1 << 29)) % (1 << 29)))
    off = OFF_MULT * P
    ol = [(off >> (29 * i)) & M29 for i in range(8)] + [off >> 232]
    o.append("static constexpr int64_t OFF29[9] = {%s};  // %d p: limbs 0..7, then everything from bit 232" % (
        ", ".join("%dll" % v for v in ol), OFF_MULT))
    assert P >> 232 < (1 << 29)
    o.append("static constexpr double INVP232 = %r;  // 2^232 / p" % (float(2**232) / P))
    return o


def emit(kernels):
    o = []
    w = o.append
    w("// Generated by gen_slp.py -- straight-line programs for the wave-cooperative engine.")
    w("#pragma once")
    w("#include <cstdint>")
    w("namespace slp {")
    for line in emit_radix():
        w(line)
    allops = []
    descs = []
    for k in kernels:
        w("// kernel %s: %d slots (%d state, %d constants)" % (k.name, k.nslots, len(k.state), len(k.consts)))
        assert k.nslots <= 512  # absolute slots are 9-bit offsets in segment 0
        w("static constexpr int %s_NSLOT = %d;" % (k.name.upper(), k.nslots))
        w("static constexpr int %s_CBASE = %d;" % (k.name.upper(), k.cbase))
        w("static constexpr int %s_NCONST = %d;" % (k.name.upper(), len(k.consts)))
        for nm, s in k.state.items():
            w("static constexpr int %s_%s = %d;" % (k.name.upper(), nm.replace(".", "_"), s))
        for nm, enc in k.progs.items():
            width = max(1, max(len(r) for r in enc))
            descs.append((k.name, nm, len(allops), len(enc), width))
            w("static constexpr int PROG_%s = %d;" % (nm.upper(), len(descs) - 1))
            for row in enc:
                # term groups in use by the level (products split their terms at ENC_SIDE)
                gm = 0
                for op in row:
                    gm |= term_groups(op)
                assert all(op[0] != OP_MUL or op[2] == ENC_SIDE for op in row)
                allops += [encode_op((op[0], op[1], gm, op[3])) for op in row] + [0] * (width - len(row))
    w("struct ProgDesc { uint32_t off; uint16_t nlev; uint16_t width; };")
    w("__device__ const ProgDesc PROGS[%d] = {" % len(descs))
    for kn, nm, off, nlev, width in descs:
        w("  {%du, %du, %du},  // %s" % (off, nlev, width, nm))
    w("};")
    w("static constexpr int OP_WORDS = %d;" % OP_WORDS)
    w("__device__ const uint64_t OPS[%d][%d] = {" % (len(allops), OP_WORDS))
    for x in allops:
        assert x >> (64 * OP_WORDS) == 0
        w("  {%s}," % ", ".join("0x%xull" % ((x >> (64 * k)) & (2**64 - 1)) for k in range(OP_WORDS)))
    w("};")
    for k in kernels:
        w("__device__ const uint32_t %s_CONSTS[%d][9] = {" % (k.name.upper(), len(k.consts)))
        for x in k.consts:
            w("  {%s}," % ", ".join("0x%08xu" % v for v in limbs29(x * RMONT % P)))
        w("};")
    mk = kernels[0]
    seq = miller_sequence()
    w("static constexpr int ML_SEQ_LEN = %d;" % len(seq))
    w("__device__ const uint8_t ML_SEQ[%d][1] = {%s};" % (len(seq), ", ".join("{PROG_%s}" % s.upper() for s in seq)))
    w("__device__ const uint8_t F12_MUL_CALL[1][4] = {{PROG_F12_MUL, 0, 1, 2}};")
    seqf, res_buf, nb = fe_sequence()
    w("static constexpr int FE_NBUF = %d;" % nb)
    w("static constexpr int FE_RESULT = %d;" % res_buf)
    w("static constexpr int FE_SEQ_LEN = %d;" % len(seqf))
    w("static constexpr int PROG_INV = 255;")
    w("__device__ const uint8_t FE_SEQ[%d][4] = {" % len(seqf))
    for prog, X, Y, D in seqf:
        w("  {%s, %d, %d, %d}," % ("PROG_INV" if prog == "INV" else "PROG_%s" % prog.upper(), X, Y, D))
    w("};")
    G = gls_constants()
    w("// GLS decomposition on G2: lattice basis rows (signed) and rounding constants G_i")
    w("static constexpr int64_t GLS_B_NEG[4][4] = {%s};" % ", ".join(
        "{%s}" % ", ".join("%d" % (1 if x < 0 else 0) for x in row) for row in GLS_B))
    w("static constexpr uint64_t GLS_B_ABS[4][4] = {%s};" % ", ".join(
        "{%s}" % ", ".join("0x%xull" % abs(x) for x in row) for row in GLS_B))
    w("static constexpr uint32_t GLS_G[4][6] = {%s};" % ", ".join(
        "{%s}" % ", ".join("0x%08xu" % ((g >> (32 * i)) & 0xFFFFFFFF) for i in range(6)) for g in G))
    w("}  // namespace slp")
    return "\n".join(o) + "\n"


# ============================================================================ checks
def run_levels(levels, S, segbase=(0, 0, 0, 0, 0, 0, 0, 0)):
    def res(x):
        return segbase[x >> 9] + (x & 511) if x >> 9 else x
    for row in levels:
        out = []
        for kind, dst, na, terms in row:
            if kind == OP_MUL:
                a = sum(c * S[res(s)] for s, c in terms[:na])
                b = sum(c * S[res(s)] for s, c in terms[na:])
                out.append((res(dst), a * b % P))
            else:
                out.append((res(dst), sum(c * S[res(s)] for s, c in terms) % P))
        for d, v in out:
            S[d] = v


# plain reference: F_p12 as F_p2[w] / (w^6 - xi); coefficient j = 3h + q is w^{2q + h}
def ref_from_mem(cs):
    poly = [None] * 6
    for j in range(6):
        h, q = divmod(j, 3)
        poly[2 * q + h] = (cs[2 * j] % P, cs[2 * j + 1] % P)
    return poly


def ref_to_mem(poly):
    cs = [0] * 12
    for k in range(6):
        q, h = divmod(k, 2)
        j = 3 * h + q
        cs[2 * j], cs[2 * j + 1] = poly[k]
    return cs


def ref_mul(a, b):
    acc = [(0, 0)] * 11
    for i in range(6):
        for j in range(6):
            t = f2mul_int(a[i], b[j])
            acc[i + j] = ((acc[i + j][0] + t[0]) % P, (acc[i + j][1] + t[1]) % P)
    out = list(acc[:6])
    for k in range(6, 11):
        t = f2mul_int(acc[k], XI)
        out[k - 6] = ((out[k - 6][0] + t[0]) % P, (out[k - 6][1] + t[1]) % P)
    return out


def ref_pow(a, e):
    r = [(1, 0)] + [(0, 0)] * 5
    while e:
        if e & 1:
            r = ref_mul(r, a)
        a = ref_mul(a, a)
        e >>= 1
    return r


def ref_conj(a):  # w -> -w
    return [(c[0], c[1]) if k % 2 == 0 else ((-c[0]) % P, (-c[1]) % P) for k, c in enumerate(a)]


def ref_frob(a):
    """x -> x^p: coefficient k gets conj(c) gamma1[k]"""
    return [f2mul_int((c[0], (-c[1]) % P), GAM1[k]) for k, c in enumerate(a)]


def ref_inv(a):
    return ref_pow(a, P**12 - 2)


def ref_miller(xP, yP, Q):
    """affine Miller loop of the optimal ate pairing, lines in the w-polynomial form"""
    def add_aff(T, S):
        (x1, y1), (x2, y2) = T, S
        if T == S:
            lam = f2mul_int(f2mul_int((3, 0), f2mul_int(x1, x1)), f2inv_int(f2mul_int((2, 0), y1)))
        else:
            lam = f2mul_int(((y2[0] - y1[0]) % P, (y2[1] - y1[1]) % P), f2inv_int(((x2[0] - x1[0]) % P, (x2[1] - x1[1]) % P)))
        x3 = ((f2mul_int(lam, lam)[0] - x1[0] - x2[0]) % P, (f2mul_int(lam, lam)[1] - x1[1] - x2[1]) % P)
        t = f2mul_int(lam, ((x1[0] - x3[0]) % P, (x1[1] - x3[1]) % P))
        y3 = ((t[0] - y1[0]) % P, (t[1] - y1[1]) % P)
        # line yP - lam xP w + (lam x1 - y1) w^3
        l = [(0, 0)] * 6
        l[0] = (yP, 0)
        lx = f2mul_int(lam, (xP, 0))
        l[1] = ((-lx[0]) % P, (-lx[1]) % P)
        m = f2mul_int(lam, x1)
        l[3] = ((m[0] - y1[0]) % P, (m[1] - y1[1]) % P)
        return (x3, y3), l
    f = [(1, 0)] + [(0, 0)] * 5
    T = Q
    negQ = (Q[0], (0, 0) if Q[1] == (0, 0) else ((-Q[1][0]) % P, (-Q[1][1]) % P))
    for d in ATE_NAF[1:]:
        f = ref_mul(f, f)
        T, l = add_aff(T, T)
        f = ref_mul(f, l)
        if d:
            T, l = add_aff(T, Q if d == 1 else negQ)
            f = ref_mul(f, l)
    Q1 = (f2mul_int((Q[0][0], (-Q[0][1]) % P), FROB_TX), f2mul_int((Q[1][0], (-Q[1][1]) % P), FROB_TY))
    Q2 = (f2mul_int(Q[0], FROB2_TX), f2mul_int(Q[1], ((-FROB2_TY[0]) % P, 0)))
    T, l = add_aff(T, Q1)
    f = ref_mul(f, l)
    T, l = add_aff(T, Q2)
    f = ref_mul(f, l)
    return f


def check():
    rng = random.Random(5)
    mk, fk, gk, g1k = build_all()
    for k in (mk, fk, gk, g1k):
        for nm, enc in k.progs.items():
            nmul = sum(1 for r in enc for op in r if op[0] == OP_MUL)
            nmlev = sum(1 for r in enc if any(op[0] == OP_MUL for op in r))
            print("%-22s levels %4d  mul-levels %3d  MUL %5d  LIN %5d  width %2d" %
                  (nm, len(enc), nmlev, nmul, sum(len(r) for r in enc) - nmul, max(len(r) for r in enc)),
                  file=sys.stderr)
        print("kernel %s: %d slots" % (k.name, k.nslots), file=sys.stderr)
    # F_p12 programs against the polynomial reference
    fprogs = fe_programs()
    base = {"X": fk.nslots, "Y": fk.nslots + 12, "D": fk.nslots + 24}
    seg = (0, base["X"], base["Y"], base["D"], 0, 0, 0, 0)
    for trial in range(3):
        S = [rng.randrange(P) for _ in range(fk.nslots + 36)]
        for x, s in fk.cslot.items():
            S[s] = x
        X = S[base["X"]:base["X"] + 12]
        Y = S[base["Y"]:base["Y"] + 12]
        rx, ry = ref_from_mem(X), ref_from_mem(Y)
        cyc = ref_mul(ref_conj(rx), ref_inv(rx))
        cyc = ref_mul(ref_frob(ref_frob(cyc)), cyc)        # cyclotomic element
        want = {"f12_mul": ref_mul(rx, ry), "f12_frob1": ref_frob(rx), "f12_frob2": ref_frob(ref_frob(rx)),
                "f12_frob3": ref_frob(ref_frob(ref_frob(rx))), "f12_conj": ref_conj(rx),
                "f12_conj_mul": ref_mul(ref_conj(rx), ry), "f12_frob2_mul": ref_mul(ref_frob(ref_frob(rx)), ry)}
        for nm, wv in want.items():
            S2 = list(S)
            run_levels(fk.progs[nm], S2, seg)
            got = S2[base["D"]:base["D"] + 12]
            assert got == ref_to_mem(wv), nm
        # cyclotomic squaring on a cyclotomic input
        S2 = list(S)
        S2[base["X"]:base["X"] + 12] = ref_to_mem(cyc)
        run_levels(fk.progs["f12_csqr"], S2, seg)
        assert S2[base["D"]:base["D"] + 12] == ref_to_mem(ref_mul(cyc, cyc)), "csqr"
        S2 = list(S)
        S2[base["X"]:base["X"] + 12] = ref_to_mem(cyc)
        run_levels(fk.progs["f12_csqr_mul"], S2, seg)
        assert S2[base["D"]:base["D"] + 12] == ref_to_mem(ref_mul(ref_mul(cyc, cyc), ry)), "csqr_mul"
        # norm + easy part
        S2 = list(S)
        run_levels(fk.progs["fe_norm"], S2, seg)
        t = S2[fk.state["t"]]
        S2[fk.state["tinv"]] = pow(t, -1, P)
        run_levels(fk.progs["fe_easy"], S2, seg)
        assert S2[base["D"]:base["D"] + 12] == ref_to_mem(ref_mul(ref_conj(rx), ref_inv(rx))), "easy part"
    print("F_p12 programs ok", file=sys.stderr)
    seqf, res_buf, nb = fe_sequence()
    print("final exponentiation: %d calls, %d buffers, %d levels (%d with products)" % (
        len(seqf), nb, sum(len(fk.progs[c[0]]) for c in seqf if c[0] != "INV"),
        sum(1 for c in seqf if c[0] != "INV" for r in fk.progs[c[0]] if any(op[0] == OP_MUL for op in r))),
        file=sys.stderr)
    bufbase = fk.nslots
    S = [0] * (bufbase + 12 * nb)
    for x, sl in fk.cslot.items():
        S[sl] = x
    fin = [rng.randrange(P) for _ in range(12)]
    S[bufbase:bufbase + 12] = fin
    for prog, X, Y, D in seqf:
        if prog == "INV":
            S[fk.state["tinv"]] = pow(S[fk.state["t"]], -1, P)
            continue
        run_levels(fk.progs[prog], S, (0, bufbase + 12 * X, bufbase + 12 * Y, bufbase + 12 * D, 0, 0, 0, 0))
    got = S[bufbase + 12 * res_buf:bufbase + 12 * res_buf + 12]
    assert got == ref_to_mem(ref_pow(ref_from_mem(fin), (P**12 - 1) // R)), "final exponentiation"
    print("final exponentiation ok", file=sys.stderr)
    # Miller loop: pipelined programs vs the affine reference, compared after the
    # final exponentiation (the two differ by factors in proper subfields)
    g2 = ((10857046999023057135944570762232829481370756359578518086990519993285655852781,
           11559732032986387107991004021392285783925812861821192530917403151452391805634),
          (8495653923123431417604973247489272438418190587263600148770280649306958101930,
           4082367875863433681332203403145435568316851327593401208105741076214120093531))
    xP, yP = 1, 2
    S = [0] * mk.nslots
    for x, s in mk.cslot.items():
        S[s] = x
    st = mk.state
    S[st["xP"]], S[st["yP"]] = xP, yP
    S[st["xQ.0"]], S[st["xQ.1"]], S[st["yQ.0"]], S[st["yQ.1"]] = g2[0][0], g2[0][1], g2[1][0], g2[1][1]
    for nm in miller_sequence():
        run_levels(mk.progs[nm], S)
    f = ref_from_mem([S[st["f.%d" % k]] for k in range(12)])
    g = ref_miller(xP, yP, g2)
    e = (P**12 - 1) // R
    assert ref_pow(f, e) == ref_pow(g, e), "Miller loop"
    print("Miller loop ok (%d bodies)" % len(miller_sequence()), file=sys.stderr)
    check_g2(gk, rng)
    check_g1(g1k, rng)


def f2add(a, b):
    return ((a[0] + b[0]) % P, (a[1] + b[1]) % P)


def f2sub(a, b):
    return ((a[0] - b[0]) % P, (a[1] - b[1]) % P)


def aff_add(A, B):
    """affine addition on the twist (None = identity)"""
    if A is None:
        return B
    if B is None:
        return A
    if A[0] == B[0]:
        if f2add(A[1], B[1]) == (0, 0):
            return None
        lam = f2mul_int(f2mul_int((3, 0), f2mul_int(A[0], A[0])), f2inv_int(f2mul_int((2, 0), A[1])))
    else:
        lam = f2mul_int(f2sub(B[1], A[1]), f2inv_int(f2sub(B[0], A[0])))
    x3 = f2sub(f2sub(f2mul_int(lam, lam), A[0]), B[0])
    return (x3, f2sub(f2mul_int(lam, f2sub(A[0], x3)), A[1]))


def aff_mul(A, k):
    R_ = None
    for bit in bin(k)[2:]:
        R_ = aff_add(R_, R_)
        if bit == "1":
            R_ = aff_add(R_, A)
    return R_


G2GEN = ((10857046999023057135944570762232829481370756359578518086990519993285655852781,
          11559732032986387107991004021392285783925812861821192530917403151452391805634),
         (8495653923123431417604973247489272438418190587263600148770280649306958101930,
          4082367875863433681332203403145435568316851327593401208105741076214120093531))


def check_g2(gk, rng):
    lam = P % R
    st = gk.state
    def setpt(S, name, pt):  # Jacobian with Z = 1 from affine
        (x0, x1), (y0, y1) = pt
        for k, v in enumerate((x0, x1, y0, y1, 1, 0)):
            S[st["%s.%d" % (name, k)]] = v
    def getaff(S, name):
        v = [S[st["%s.%d" % (name, k)]] for k in range(6)]
        X, Y, Z = (v[0], v[1]), (v[2], v[3]), (v[4], v[5])
        if Z == (0, 0):
            return None
        zi = f2inv_int(Z)
        zi2 = f2mul_int(zi, zi)
        return (f2mul_int(X, zi2), f2mul_int(Y, f2mul_int(zi2, zi)))
    for trial in range(2):
        Q = aff_mul(G2GEN, rng.randrange(1, R))
        S = [0] * gk.nslots
        for x, sl in gk.cslot.items():
            S[sl] = x
        S[st["xQ.0"]], S[st["xQ.1"]], S[st["yQ.0"]], S[st["yQ.1"]] = Q[0][0], Q[0][1], Q[1][0], Q[1][1]
        run_levels(gk.progs["g2_psi"], S)
        for j in (1, 2, 3):
            got = ((S[st["B%d.x.0" % j]], S[st["B%d.x.1" % j]]), (S[st["B%d.y.0" % j]], S[st["B%d.y.1" % j]]))
            assert got == aff_mul(Q, pow(lam, j, R)), "psi"
        run_levels(gk.progs["g2_table"], S)
        for d in range(1, 16):
            want = None
            for j in range(4):
                if d >> j & 1:
                    want = aff_add(want, aff_mul(Q, pow(lam, j, R)))
            assert getaff(S, "TB%d" % d) == want, ("table", d)
        # doubling, addition (with a Jacobian operand at segment 2), mixed addition, to affine
        A = aff_mul(G2GEN, rng.randrange(1, R))
        setpt(S, "T", Q)
        run_levels(gk.progs["g2_dbl"], S)
        assert getaff(S, "T") == aff_add(Q, Q), "dbl"
        T2 = aff_add(Q, Q)
        base = st["TB5.0"]
        run_levels(gk.progs["g2_add"], S, (0, 0, base, 0, 0, 0, 0, 0))
        assert getaff(S, "T") == aff_add(T2, getaff(S, "TB5")), "add"
        T3 = getaff(S, "T")
        Sa = list(S) + [A[0][0], A[0][1], A[1][0], A[1][1]]
        run_levels(gk.progs["g2_madd"], Sa, (0, 0, len(S), 0, 0, 0, 0, 0))
        assert getaff(Sa, "T") == aff_add(T3, A), "madd"
        run_levels(gk.progs["g2_norm"], Sa)
        Sa[st["tinv"]] = pow(Sa[st["t"]], -1, P)
        run_levels(gk.progs["g2_aff"], Sa)
        assert ((Sa[st["ax.0"]], Sa[st["ax.1"]]), (Sa[st["ay.0"]], Sa[st["ay.1"]])) == aff_add(T3, A), "aff"
        # degenerate addition reports H = 0 and r = 0
        setpt(S, "T", Q)
        setpt(S, "TB1", Q)
        run_levels(gk.progs["g2_add"], S, (0, 0, st["TB1.0"], 0, 0, 0, 0, 0))
        assert S[st["H.0"]] % P == 0 and S[st["H.1"]] % P == 0 and S[st["RR.0"]] % P == 0 and S[st["RR.1"]] % P == 0
    # decomposition
    for k in [0, 1, R - 1] + [rng.randrange(R) for _ in range(2000)]:
        kj = gls_decompose(k)
        assert (sum(kj[j] * pow(lam, j, R) for j in range(4)) - k) % R == 0 and max(abs(x) for x in kj) < 2**65
    print("G2 programs and GLS decomposition ok", file=sys.stderr)


def g1_aff_add(A, B):
    if A is None:
        return B
    if B is None:
        return A
    if A[0] == B[0]:
        if (A[1] + B[1]) % P == 0:
            return None
        l = 3 * A[0] * A[0] * pow(2 * A[1], -1, P) % P
    else:
        l = (B[1] - A[1]) * pow(B[0] - A[0], -1, P) % P
    x = (l * l - A[0] - B[0]) % P
    return (x, (l * (A[0] - x) - A[1]) % P)


def g1_aff_mul(A, k):
    R_ = None
    for bit in bin(k)[2:]:
        R_ = g1_aff_add(R_, R_)
        if bit == "1":
            R_ = g1_aff_add(R_, A)
    return R_


def check_g1(g1k, rng):
    st = g1k.state
    def setj(S, name, pt):
        S[st[name + ".0"]], S[st[name + ".1"]], S[st[name + ".2"]] = pt[0], pt[1], 1
    def getj(S, name):
        X, Y, Z = (S[st["%s.%d" % (name, k)]] % P for k in range(3))
        if Z == 0:
            return None
        zi = pow(Z, -1, P)
        return (X * zi * zi % P, Y * zi * zi * zi % P)
    for trial in range(3):
        Pt = g1_aff_mul((1, 2), rng.randrange(1, R))
        S = [0] * g1k.nslots
        for x, sl in g1k.cslot.items():
            S[sl] = x
        S[st["xP"]], S[st["yP"]] = Pt
        run_levels(g1k.progs["g1_phi"], S)
        assert (S[st["B1.x"]] % P, Pt[1]) == g1_aff_mul(Pt, GLV_LAM), "phi"
        S[st["B1.y"]] = Pt[1]
        run_levels(g1k.progs["g1_table"], S)
        for d in range(1, 16):
            want = g1_aff_add(g1_aff_mul(Pt, d & 3), g1_aff_mul(Pt, (d >> 2) * GLV_LAM % R)) if d & 3 else \
                g1_aff_mul(Pt, (d >> 2) * GLV_LAM % R)
            assert getj(S, "TB%d" % d) == want, ("table", d)
        setj(S, "T", Pt)
        run_levels(g1k.progs["g1_dbl"], S)
        assert getj(S, "T") == g1_aff_mul(Pt, 2), "dbl"
        run_levels(g1k.progs["g1_dbl2"], S)
        assert getj(S, "T") == g1_aff_mul(Pt, 8), "dbl2"
        run_levels(g1k.progs["g1_dbl2_add"], S, (0, 0, st["TB7.0"], 0, 0, 0, 0, 0))
        T32 = g1_aff_add(g1_aff_mul(Pt, 32), getj(S, "TB7"))
        assert getj(S, "T") == T32, "dbl2_add"
        # Jacobian addition with a Jacobian operand (Z != 1)
        Sj = list(S)
        setj(Sj, "T", g1_aff_mul(Pt, 5))
        run_levels(g1k.progs["g1_add"], Sj, (0, 0, st["TB6.0"], 0, 0, 0, 0, 0))
        assert getj(Sj, "T") == g1_aff_add(g1_aff_mul(Pt, 5), getj(S, "TB6")), "add"
        A = g1_aff_mul((1, 2), rng.randrange(1, R))
        Sa = list(S) + [A[0], A[1]]
        run_levels(g1k.progs["g1_madd"], Sa, (0, 0, len(S), 0, 0, 0, 0, 0))
        assert getj(Sa, "T") == g1_aff_add(T32, A), "madd"
        Z = Sa[st["T.2"]] % P
        Sa[st["tinv"]] = pow(Z, -1, P)
        run_levels(g1k.progs["g1_aff"], Sa)
        assert (Sa[st["ax"]] % P, Sa[st["ay"]] % P) == g1_aff_add(T32, A), "aff"
        # degenerate: 4T + A with A = 4T reports H = 0 and r = 0
        setj(S, "T", Pt)
        Tq = g1_aff_mul(Pt, 4)
        setj(S, "TB1", Tq)
        run_levels(g1k.progs["g1_dbl2_add"], S, (0, 0, st["TB1.0"], 0, 0, 0, 0, 0))
        assert S[st["H"]] % P == 0 and S[st["RR"]] % P == 0, "degenerate"
    print("G1 programs ok", file=sys.stderr)


if __name__ == "__main__":
    if "--check" in sys.argv:
        check()
    else:
        sys.stdout.write(emit(list(build_all())))
