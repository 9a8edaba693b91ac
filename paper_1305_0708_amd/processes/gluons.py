"""n-gluon processes (g g -> (n-2) g): colour-ordered HEGET call chains.

Colour.  With Tr(T^a T^b) = delta/2 the paper's colour factors expand into
single traces: the triple-gluon factor i f^abc (Sec. 4.2.3) is
2 [Tr(a b c) - Tr(b a c)], the quartic factors f^abe f^cde (Sec. 4.2.4) give
-2 [Tr(abcd) - Tr(abdc) - Tr(bacd) + Tr(badc)] after the internal line is
contracted, and every internal gluon line contracts two traces with a factor
1/2 (the 1/N parts cancel inside each commutator).  Collecting the coefficient
of one cyclic ordering gives the colour-ordered rules used here:

  3-vertex, cyclic (1, 2, 3):      2 vvv(1, 2, 3)
  4-vertex, cyclic (1, 2, 3, 4):   -2 Gamma(1, 2, 3, 4) + 2 Gamma(1, 4, 2, 3)
  internal line:                   1/2 x (the HEGET current's propagator)

so M = sum_sigma Tr(T^a0 T^a_sigma(1) ...) A(0, sigma) with A built from the
same vvvxxx / jvvxxx / ggggxx / jgggxx calls as the Feynman diagrams.  The
jamps are the partial amplitudes A(0, sigma) of the (n-1)! trace orderings.
Only the (n-2)! orderings with the last leg at the end, A(0, tau, n-1), are
evaluated; the others follow exactly from the Kleiss-Kuijf relations
A(0, alpha, n-1, beta) = (-1)^|beta| sum_{shuffles rho of alpha and reversed
beta} A(0, rho, n-1).  The trace-basis colour matrix C[s][t] =
sum_col Tr(0 s) conj(Tr(0 t)) is computed exactly by the Fierz identity.
"""
import itertools
import math
from fractions import Fraction

from .. import ir
from ..ir import V, P_ZERO, Leg, Call, Coupling, Process

_CACHE = {}


# ------------------------------------------------------------ exact colour algebra
def _fierz(traces, N=3):
    """sum over repeated gluon labels of a product of traces (exact, SU(N))"""
    work = [(Fraction(1), [list(t) for t in traces])]
    total = Fraction(0)
    while work:
        c, trs = work.pop()
        lab = next((t[0] for t in trs if t), None)
        if lab is None:
            total += c * Fraction(N) ** len(trs)
            continue
        pos = [(i, j) for i, t in enumerate(trs) for j, x in enumerate(t) if x == lab]
        (i1, j1), (i2, j2) = pos
        rest = [t for k, t in enumerate(trs) if k not in (i1, i2)]
        if i1 == i2:
            t = trs[i1]
            a, b = t[j2 + 1:] + t[:j1], t[j1 + 1:j2]
            work.append((c / 2, rest + [a, b]))
            work.append((-c / (2 * N), rest + [a + b]))
        else:
            x = trs[i1][j1 + 1:] + trs[i1][:j1]
            y = trs[i2][j2 + 1:] + trs[i2][:j2]
            work.append((c / 2, rest + [x + y]))
            work.append((-c / (2 * N), rest + [x, y]))
    return total


def trace_orderings(n):
    """all (n-1)! orderings (0, perm of 1..n-1), lexicographic"""
    return [(0,) + p for p in itertools.permutations(range(1, n))]


def ddm_orderings(n):
    """the (n-2)! orderings (0, perm of 1..n-2, n-1)"""
    return [(0,) + p + (n - 1,) for p in itertools.permutations(range(1, n - 1))]


def colour_matrix(n):
    """exact trace-basis colour matrix; C[s][t] depends only on s^-1 t"""
    key = ("C", n)
    if key in _CACHE:
        return _CACHE[key]
    orders = trace_orderings(n)
    index = {o: k for k, o in enumerate(orders)}
    first = {}
    for o in orders:
        first[o] = _fierz([list(orders[0]), list(reversed(o))])
    C = []
    for s in orders:
        inv = {lab: k for k, lab in enumerate(s)}     # relabel s -> identity
        row = []
        for t in orders:
            row.append(first[tuple(inv[x] for x in t)])
        C.append(row)
    _CACHE[key] = C
    return C


def kk_matrix(n):
    """K[t][d]: A(t) = sum_d K[t][d] A(ddm_d) (Kleiss-Kuijf), integer entries"""
    key = ("K", n)
    if key in _CACHE:
        return _CACHE[key]
    ddm = ddm_orderings(n)
    dindex = {o: k for k, o in enumerate(ddm)}
    last = n - 1
    K = []
    for t in trace_orderings(n):
        rest = t[1:]
        p = rest.index(last)
        alpha, beta = rest[:p], rest[p + 1:]
        row = [0] * len(ddm)
        sign = (-1) ** len(beta)
        for shuffle in _shuffles(list(alpha), list(reversed(beta))):
            row[dindex[(0,) + tuple(shuffle) + (last,)]] += sign
        K.append(row)
    _CACHE[key] = K
    return K


def _shuffles(a, b):
    if not a:
        yield list(b)
        return
    if not b:
        yield list(a)
        return
    for s in _shuffles(a[1:], b):
        yield [a[0]] + s
    for s in _shuffles(a, b[1:]):
        yield [b[0]] + s


def ddm_colour_matrix(n):
    """K^T C K: the colour matrix in the basis of the (n-2)! evaluated jamps"""
    key = ("CD", n)
    if key in _CACHE:
        return _CACHE[key]
    C, K = colour_matrix(n), kk_matrix(n)
    m, d = len(C), len(K[0])
    CK = [[sum(C[s][t] * K[t][j] for t in range(m) if K[t][j]) for j in range(d)] for s in range(m)]
    out = [[sum(K[s][i] * CK[s][j] for s in range(m) if K[s][i]) for j in range(d)] for i in range(d)]
    _CACHE[key] = out
    return out


# ------------------------------------------------------------- call chains
def gg_ng(n=6, sqrt_s=1000.0, cut_pt=20.0, cut_dr=0.4, basis="trace"):
    """g g -> (n-2) g with the generation cut (pT > cut_pt, Delta R > cut_dr).

    basis "trace": the (n-1)! trace-basis flows A(0, sigma) with the dense
    (n-1)! x (n-1)! colour matrix (120 x 120 for n = 6), each flow the
    Kleiss-Kuijf combination of the evaluated orderings (the flow map); the
    colour form runs on MFMA from 32 flows on.  basis "ddm": the (n-2)!
    evaluated orderings are the flows, with K^T C K as colour matrix.

    The IR is an ordering template: the calls of one colour ordering over leg
    positions 0..n-1 (position 0 is the root leg 0), evaluated for each of the
    (n-2)! orderings (0, tau, n-1).  A current of an ordered range L of
    positions is the sum of jvv(J_A, J_B) over splits L = A|B and of
    jggg(J_B, J_C, J_A) - jggg(J_A, J_B, J_C) over splits A|B|C (vadd / vsub);
    the partial amplitude is sum 2 vvv(J_A, J_B, w_0) over two-way splits plus
    sum [-2 gggg(J_A, J_B, J_C, w_0) + 2 gggg(J_A, w_0, J_B, J_C)] over three-way
    splits of positions 1..n-1.
    """
    legs = [Leg(V, True, colour=8, name="g"), Leg(V, True, colour=8, name="g")] + \
           [Leg(V, False, colour=8, name="g") for _ in range(n - 2)]
    cpl = [Coupling("ggg"), Coupling("gggg")]
    G3, G4 = 0, 1
    calls = []
    nxt = [n]
    seq = list(range(1, n))                 # positions after the root
    cur = {}

    def new_slot():
        s = nxt[0]
        nxt[0] += 1
        return s

    def current(i, j):                      # ordered range seq[i:j]
        if j - i == 1:
            return seq[i]
        if (i, j) in cur:
            return cur[(i, j)]
        terms = []
        for m in range(i + 1, j):
            s = new_slot()
            calls.append(Call("jvv", (current(i, m), current(m, j)), s, G3, P_ZERO))
            terms.append((s, 1.0))
        for m in range(i + 1, j):
            for l in range(m + 1, j):
                a, b, c = current(i, m), current(m, l), current(l, j)
                s1 = new_slot()
                calls.append(Call("jggg", (b, c, a), s1, G4, P_ZERO))
                s2 = new_slot()
                calls.append(Call("jggg", (a, b, c), s2, G4, P_ZERO))
                terms += [(s1, 1.0), (s2, -1.0)]
        acc = terms[0][0]
        for slot, sign in terms[1:]:
            s = new_slot()
            calls.append(Call("vadd" if sign > 0 else "vsub", (acc, slot), s, -1, P_ZERO))
            acc = s
        cur[(i, j)] = acc
        return acc

    terms = []
    amp = 0
    L = len(seq)
    for m in range(1, L):
        calls.append(Call("vvv", (current(0, m), current(m, L), 0), amp, G3))
        terms.append((amp, 2.0))
        amp += 1
    for m in range(1, L):
        for l in range(m + 1, L):
            a, b, c = current(0, m), current(m, l), current(l, L)
            calls.append(Call("gggg", (a, b, c, 0), amp, G4))
            terms.append((amp, -2.0))
            amp += 1
            calls.append(Call("gggg", (a, 0, b, c), amp, G4))
            terms.append((amp, 2.0))
            amp += 1
    orders = ddm_orderings(n)
    name = {4: "gg_gg", 5: "gg_3g", 6: "gg_4g"}.get(n, f"gg_{n - 2}g")
    if basis == "trace":
        colour, flow_map = colour_matrix(n), [list(r) for r in kk_matrix(n)]
    elif basis == "ddm":
        colour, flow_map = ddm_colour_matrix(n), None
        name += "_ddm"
    else:
        raise ValueError(f"unknown colour basis {basis!r}")
    # the two innermost helicity loops of an ordering's nest unrolled: measured on
    # MI355X, C2's DDM kernel 96.1 -> 92.4 ms per 2^20 events (FP64), the seven-gluon
    # kernel 205.6 -> 190.5 ms per 2^16; unrolling three or more loops was slower
    proc = Process(name, legs, cpl, calls, n_amps=amp, n_flows=len(colour), jamp=[list(terms)] * len(orders),
                   colour=colour, helicities=ir.all_helicities(legs), sqrt_s=sqrt_s, n_a_n_b=64,
                   symmetry=math.factorial(n - 2), cut_pt=cut_pt, cut_dr=cut_dr, cut_enabled=n > 4,
                   orderings=[tuple(o) for o in orders], flow_map=flow_map, template_unroll=2)
    return proc.validate()
