"""u ubar -> t tbar + n gluons: every tree-level Feynman diagram as HEGET calls.

The builder plays MadGraph's part for the paper's long-amplitude process
u ubar -> t tbar g g g (Sec. 5.3-5.5): it enumerates the Feynman diagrams,
emits one HEGET call per distinct sub-diagram (a wavefunction shared by every
diagram that contains it), one amplitude call per diagram, and decomposes each
diagram's colour factor into a basis of colour flows.

Legs: 0 u (incoming), 1 ubar (incoming), 2 t (outgoing), 3 tbar (outgoing),
4 .. 3+n gluons (outgoing).  In HEGET terms u and tbar are flowing-in spinors
|fi>, ubar and t flowing-out <fo|.  Each diagram is written from the vertex
where the ubar line ends: iov(U(S1), ubar, G(S2)), with U(S1) the u line from
leg 0 carrying the gluon sub-diagrams attached along it (fvi calls) and G(S2)
an off-shell gluon holding the whole t line (the t line closed by jio between
its tbar side, fvi calls from leg 3, and its t side, fvo calls from leg 2;
gluons joined by jvv and, one call per colour structure, jggg).

Colour.  The colour factors of the HEGET outputs (the library's couplings
g_qq = g_ggg = g_s, g_gggg = g_s^2 and the vertex signs of Sec. 4.2):
quark-gluon vertex -T^a, triple-gluon vertex i f^abc, and for the quartic
vertex the paper's three calls (Sec. 4.2.4)

    jggg(A, B, C): f^abe f^cde,   jggg(C, A, B): f^ace f^dbe,   jggg(B, C, A): f^ade f^bce

with a, b, c the colours of A, B, C and d the output's.  A gluon current is
kept as the matrix G = G^a T^a, in which these become commutators:
i f^abc T^c = [A, B], and the quartic terms -[[A, B], C], -[B, [A, C]] and
[A, [B, C]].  A quark line closing into a gluon gives, by the Fierz identity,
-1/2 (outer product - (1/N) trace x identity).  Every colour factor is thus a
sum of products of open strings (T^a1 T^a2 ...)_ij between the external quark
indices, with exact rational coefficients; each distinct product of two strings
is one colour flow, and the colour matrix of the flows is the sum over all
explicit colours of conj(flow) x flow.
"""
import functools
import itertools
from fractions import Fraction

import numpy as np

from .. import ir
from ..ir import F, V, P_ZERO, P_TOP, Leg, Call, Coupling, Process

N_C = 3
G_QQ, GGG, GGGG = 0, 1, 2

# index symbols: external quark indices (u column, ubar row, t row, tbar column)
# and the free row / column index of a node's colour tensor
I_U, I_UB, I_T, I_TB = "i0", "i1", "i2", "i3"
ROW, COL = "k", "l"


# --------------------------------------------------------------- colour strings
# A colour structure is a product of segments (start, gluons, end) meaning
# (T^g1 T^g2 ...)_{start end} (a Kronecker delta when there is no gluon) and of
# closed traces Tr(T^g1 ...).  An expression maps structures to coefficients.
def _canon(segs, traces):
    tr = []
    for t in traces:
        rots = [t[i:] + t[:i] for i in range(len(t))]
        tr.append(min(rots))
    return (tuple(sorted(segs)), tuple(sorted(tr)))


def _contract(segs, traces, sym):
    """join the segment that ends at index sym with the one that starts there"""
    a = next(s for s in segs if s[2] == sym)
    b = next(s for s in segs if s[0] == sym)
    rest = [s for s in segs if s is not a and s is not b]
    if a is b:
        if not a[1]:
            return rest, traces, Fraction(N_C)
        return rest, traces + [a[1]], Fraction(1)
    return rest + [(a[0], a[1] + b[1], b[2])], traces, Fraction(1)


def _rename(segs, old, new):
    return [(new if s[0] == old else s[0], s[1], new if s[2] == old else s[2]) for s in segs]


def _add(out, key, c):
    v = out.get(key, Fraction(0)) + c
    if v:
        out[key] = v
    else:
        out.pop(key, None)


def _product(x, y, sym_x, sym_y, scale=Fraction(1)):
    """sum over the shared index: x's index sym_x contracted with y's sym_y"""
    out = {}
    for (sx, tx), cx in x.items():
        for (sy, ty), cy in y.items():
            segs = _rename(list(sx), sym_x, "#") + _rename(list(sy), sym_y, "#")
            segs, traces, f = _contract(segs, list(tx) + list(ty), "#")
            _add(out, _canon(segs, traces), scale * cx * cy * f)
    return out


def _lin(*terms):
    out = {}
    for c, e in terms:
        for k, v in e.items():
            _add(out, k, c * v)
    return out


def mat_mul(a, b):
    """(A B)_{kl} of two gluon matrices"""
    return _product(_rename_expr(a, COL, "r"), _rename_expr(b, ROW, "s"), "r", "s")


def _rename_expr(e, old, new):
    return {_canon(_rename(list(s), old, new), list(t)): c for (s, t), c in e.items()}


def comm(a, b):
    return _lin((Fraction(1), mat_mul(a, b)), (Fraction(-1), mat_mul(b, a)))


def mat_col(g, q):
    """(G q)_k of a gluon matrix and a column vector"""
    return _product(_rename_expr(g, COL, "r"), _rename_expr(q, ROW, "s"), "r", "s")


def row_mat(q, g):
    """(q G)_l of a row vector and a gluon matrix"""
    return _product(_rename_expr(q, COL, "r"), _rename_expr(g, ROW, "s"), "r", "s")


def outer(col, row):
    """col_k row_l (no index shared)"""
    out = {}
    for (sx, tx), cx in col.items():
        for (sy, ty), cy in row.items():
            _add(out, _canon(list(sx) + list(sy), list(tx) + list(ty)), cx * cy)
    return out


def row_col(row, col):
    """the number row . col"""
    return _product(_rename_expr(row, COL, "r"), _rename_expr(col, ROW, "r"), "r", "r")


def _single(seg):
    return {_canon([seg], []): Fraction(1)}


# ------------------------------------------------------------------ diagrams
class _Builder:
    def __init__(self, ng):
        self.ng, self.nl = ng, 4 + ng
        self.gluons = frozenset(range(4, self.nl))
        self.calls = []
        self.slot = self.nl
        self.memo = {}
        self.amps = []   # (colour expression) per amplitude, in amplitude-index order

    def g_ok(self, s):
        if not s or 0 in s or 1 in s or ((2 in s) != (3 in s)):
            return False
        return len(s) > 1 or next(iter(s)) in self.gluons

    def _new(self, op, ins, cpl, prop):
        out = self.slot
        self.slot += 1
        self.calls.append(Call(op, tuple(ins), out, cpl, prop))
        return out

    @staticmethod
    def _splits(s, must):
        """proper non-empty subsets of s that contain every leg of must"""
        items = sorted(s)
        for r in range(1, len(items)):
            for sub in itertools.combinations(items, r):
                sub = frozenset(sub)
                if must <= sub:
                    yield sub

    def gluon(self, s):
        """every sub-diagram ending in an off-shell gluon: [(slot, colour matrix)]"""
        key = ("g", s)
        if key in self.memo:
            return self.memo[key]
        out = []
        if len(s) == 1:
            (g,) = s
            out.append((g, _single((ROW, (g,), COL))))
        else:
            low = min(s)
            for a in self._splits(s, {low}):
                b = s - a
                if self.g_ok(a) and self.g_ok(b):
                    for sa, ca in self.gluon(a):
                        for sb, cb in self.gluon(b):
                            out.append((self._new("jvv", (sa, sb), GGG, P_ZERO), comm(ca, cb)))
                r = s - a
                if len(r) < 2:
                    continue
                for bb in self._splits(r, {min(r)}):
                    c = r - bb
                    if not (self.g_ok(a) and self.g_ok(bb) and self.g_ok(c)):
                        continue
                    for sa, ca in self.gluon(a):
                        for sb, cb in self.gluon(bb):
                            for sc, cc in self.gluon(c):
                                one = Fraction(1)
                                t1 = _lin((-one, comm(comm(ca, cb), cc)))
                                t2 = _lin((-one, comm(cb, comm(ca, cc))))
                                t3 = comm(ca, comm(cb, cc))
                                out.append((self._new("jggg", (sa, sb, sc), GGGG, P_ZERO), t1))
                                out.append((self._new("jggg", (sc, sa, sb), GGGG, P_ZERO), t2))
                                out.append((self._new("jggg", (sb, sc, sa), GGGG, P_ZERO), t3))
            if 2 in s and 3 in s:
                for a in self._splits(s, {3}):
                    if 2 in a:
                        continue
                    for sf, cf in self.quark("tb", a):
                        for so, co in self.quark("t", s - a):
                            col = _lin((Fraction(-1, 2), outer(cf, co)),
                                       (Fraction(1, 2 * N_C), outer(row_col(co, cf), _single((ROW, (), COL)))))
                            out.append((self._new("jio", (sf, so), G_QQ, P_ZERO), col))
        self.memo[key] = out
        return out

    def quark(self, kind, s):
        """sub-diagrams ending in an off-shell quark of the u line ("u", column
        from leg 0), the t line's tbar side ("tb", column from leg 3) or its t
        side ("t", row from leg 2): [(slot, colour vector)]"""
        key = (kind, s)
        if key in self.memo:
            return self.memo[key]
        own = {"u": 0, "tb": 3, "t": 2}[kind]
        out = []
        if s == frozenset([own]):
            seg = {"u": (ROW, (), I_U), "tb": (ROW, (), I_TB), "t": (I_T, (), COL)}[kind]
            out.append((own, _single(seg)))
        else:
            prop = P_ZERO if kind == "u" else P_TOP
            for q in self._splits(s, {own}):
                r = s - q
                if not self.g_ok(r):
                    continue
                for sq, cq in self.quark(kind, q):
                    for sg, cg in self.gluon(r):
                        if kind == "t":
                            slot = self._new("fvo", (sq, sg), G_QQ, prop)
                            col = _lin((Fraction(-1), row_mat(cq, cg)))
                        else:
                            slot = self._new("fvi", (sq, sg), G_QQ, prop)
                            col = _lin((Fraction(-1), mat_col(cg, cq)))
                        out.append((slot, col))
        self.memo[key] = out
        return out

    def build(self):
        rest = frozenset(range(self.nl)) - {1}
        for r in range(1, len(rest) + 1):
            for s1 in itertools.combinations(sorted(rest), r):
                s1 = frozenset(s1)
                if 0 not in s1 or not self.g_ok(rest - s1):
                    continue
                for su, cu in self.quark("u", s1):
                    for sg, cg in self.gluon(rest - s1):
                        amp = len(self.amps)
                        self.calls.append(Call("iov", (su, 1, sg), amp, G_QQ, P_ZERO))
                        # -(G U)_{i1}
                        c = _lin((Fraction(-1), _rename_expr(mat_col(cg, cu), ROW, I_UB)))
                        self.amps.append(c)
        return self


# ------------------------------------------------------------- colour basis
def _flow_values(flows, ng):
    """each flow's value for every explicit colour assignment (i0, i1, i2, i3,
    a_4, ...): array [n_flows][3, 3, 3, 3, 8, ...]"""
    T = np.zeros((8, 3, 3), dtype=np.complex128)
    h = 0.5
    T[0, 0, 1] = T[0, 1, 0] = h
    T[1, 0, 1], T[1, 1, 0] = -0.5j, 0.5j
    T[2, 0, 0], T[2, 1, 1] = h, -h
    T[3, 0, 2] = T[3, 2, 0] = h
    T[4, 0, 2], T[4, 2, 0] = -0.5j, 0.5j
    T[5, 1, 2] = T[5, 2, 1] = h
    T[6, 1, 2], T[6, 2, 1] = -0.5j, 0.5j
    T[7, 0, 0] = T[7, 1, 1] = h / np.sqrt(3.0)
    T[7, 2, 2] = -1.0 / np.sqrt(3.0)
    letters = "abcdefgh"
    quark = {I_U: "p", I_UB: "q", I_T: "r", I_TB: "s"}
    out_idx = "pqrs" + letters[:ng]
    vals = []
    for segs, traces in flows:
        assert not traces
        ops, subs, inner = [], [], iter("ABCDEFGHIJKLMNO")
        for start, glue, end in segs:
            if not glue:
                ops.append(np.eye(3))
                subs.append(quark[start] + quark[end])
                continue
            # (T^g1 T^g2 ...)_{start end}: one internal index between neighbours
            idx = [quark[start]] + [next(inner) for _ in range(len(glue) - 1)] + [quark[end]]
            for j, g in enumerate(glue):
                ops.append(T)
                subs.append(letters[g - 4] + idx[j] + idx[j + 1])
        vals.append(np.einsum(",".join(subs) + "->" + out_idx, *ops))
    return np.array(vals).reshape(len(flows), -1)


def _rational(x, what):
    f = Fraction(float(x)).limit_denominator(10 ** 6)
    if abs(float(f) - x) > 1e-9 * max(1.0, abs(x)):
        raise ValueError(f"{what}: {x} is not a simple fraction")
    return f


@functools.lru_cache(maxsize=None)
def _build(ng):
    b = _Builder(ng).build()
    flows = sorted({k for c in b.amps for k in c})
    index = {k: f for f, k in enumerate(flows)}
    jamp = [[] for _ in flows]
    for a, c in enumerate(b.amps):
        for k, coef in c.items():
            jamp[index[k]].append((a, float(coef)))
    vals = _flow_values(flows, ng)
    C = (vals.conj() @ vals.T).real
    colour = [[_rational(C[i, j], "colour matrix") for j in range(len(flows))] for i in range(len(flows))]
    return b.calls, len(b.amps), flows, jamp, colour


def uu_ttbar_gluons(ng=3, sqrt_s=1000.0, name=None, parts=None):
    """u ubar -> t tbar + ng gluons at fixed sqrt_s, stable tops (on-shell
    external top spinors), every final particle with pT > 20 GeV and Delta R
    > 0.4 (the cut applies to the tops as well).  Phase space: the collision
    decays to t + X, X to tbar + Y, ... in flat two-body steps."""
    calls, n_amps, flows, jamp, colour = _build(ng)
    parts_mixed = 0
    if parts is None:
        # the function division, measured on MI355X for three gluons (393
        # amplitudes, ms per 2^18 events): about 15 amplitudes per device
        # function in FP64 (27 parts: 240 ms; 24: 245; 20: 270; 10: 506), about
        # 57 in FP32 (7 parts: 146 ms; 6: 149; 8: 148; 10: 152; 5: 155).  Two
        # gluons: two parts, where one would do, so that the small process runs
        # the divided code too.
        parts, parts_mixed = (-(-n_amps // 15), -(-n_amps // 57)) if ng >= 3 else (2 if ng == 2 else 1, 0)
    legs = [Leg(F, True, +1, colour=3, name="u"), Leg(F, True, -1, colour=3, name="ubar"),
            Leg(F, False, +1, particle=P_TOP, colour=3, name="t"),
            Leg(F, False, -1, particle=P_TOP, colour=3, name="tbar")]
    legs += [Leg(V, False, colour=8, name="g") for _ in range(ng)]
    cpl = [Coupling("g_qq"), Coupling("ggg"), Coupling("gggg")]
    fin = list(range(2, 4 + ng))
    tree = []
    for k in range(len(fin) - 1):
        d1 = fin[k + 1] if k == len(fin) - 2 else -(k + 2)
        tree.append((P_ZERO, ir.PS_FLAT, fin[k], d1))
    sym = 1
    for k in range(2, ng + 1):
        sym *= k
    # beyond one gluon the diagram sum is evaluated helicity row by row: the
    # loop nest would keep too many currents live at once
    return Process(name or f"uu_tt{'g' * ng}", legs, cpl, list(calls), n_amps=n_amps, n_flows=len(flows),
                   jamp=jamp, colour=colour, helicities=ir.all_helicities(legs), sqrt_s=sqrt_s,
                   n_a_n_b=9, symmetry=sym, cut_enabled=ng > 0, cut_pt=20.0, cut_dr=0.4, ps_tree=tree,
                   helicity_schedule="rows" if ng >= 2 else "nest", row_parts=parts,
                   row_parts_mixed=parts_mixed).validate()


def flow_strings(ng):
    """the colour flows of the basis, each a pair of strings (start, gluons, end)"""
    return [segs for segs, _ in _build(ng)[2]]
