"""Process IR: the data a process is created from.

The IR plays the role the paper gives to MadGraph's generated amplitude
routine as converted by MG2CUDA (Sec. 5): external legs, the list of
HEGET-style vertex/propagator calls (Sec. 4, Tables of external-line and vertex
functions), the decomposition of the amplitudes into colour flows (jamps) and
the colour matrix (Sec. 5.4), plus the helicity combinations to sum over.

It is plain data; ``heget_process_create`` receives it as C structs
(``include/heget.h``) and ``codegen`` turns the structural part into a
straight-line HIP kernel.  SM parameter values, the helicity table and the cut
thresholds are runtime data and are not part of the kernel's fingerprint.
"""
from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Optional, Tuple
import math
import struct

# leg kinds
F, V, S = 0, 1, 2
# particle ids used for masses / widths (index into the runtime mass table)
P_ZERO, P_W, P_Z, P_TOP, P_H = 0, 1, 2, 3, 4
PARTICLE_NAMES = {P_ZERO: "zero", P_W: "W", P_Z: "Z", P_TOP: "top", P_H: "H"}

# call opcodes (HEGET function equivalents)
OPS = [
    "iov", "fvi", "fvo", "jio",            # FFV
    "ios", "fsi", "fso", "hio",            # FFS
    "vvv", "jvv",                          # VVV
    "gggg", "jggg", "wwww", "jwww",        # VVVV
    "vvs", "jvs", "hvv",                   # VVS
    "vvss", "jvss", "hvvs",                # VVSS
    "sss", "hss", "ssss", "hsss",          # SSS, SSSS
    "vadd", "vsub",                        # sums of currents with one momentum
]
OP = {name: i for i, name in enumerate(OPS)}
AMP_OPS = {"iov", "ios", "vvv", "gggg", "wwww", "vvs", "vvss", "sss", "ssss"}
# kind of the output wavefunction of each current op
OUT_KIND = {"fvi": F, "fvo": F, "jio": V, "fsi": F, "fso": F, "hio": S, "jvv": V, "jggg": V,
            "jwww": V, "jvs": V, "hvv": S, "jvss": V, "hvvs": S, "hss": S, "hsss": S,
            "vadd": V, "vsub": V}
# ops whose output carries the momentum of their first input (not the sum)
LINEAR_OPS = {"vadd", "vsub"}
MFMA_MIN_FLOWS = 32
COLOUR_FORMS = {"dense": 0, "compressed": 1}
DIVISIONS = {"fused": 0, "split": 1}
# input kinds per op (in argument order)
IN_KINDS = {
    "iov": (F, F, V), "fvi": (F, V), "fvo": (F, V), "jio": (F, F),
    "ios": (F, F, S), "fsi": (F, S), "fso": (F, S), "hio": (F, F),
    "vvv": (V, V, V), "jvv": (V, V),
    "gggg": (V, V, V, V), "jggg": (V, V, V), "wwww": (V, V, V, V), "jwww": (V, V, V),
    "vvs": (V, V, S), "jvs": (V, S), "hvv": (V, V),
    "vvss": (V, V, S, S), "jvss": (V, S, S), "hvvs": (V, V, S),
    "sss": (S, S, S), "hss": (S, S), "ssss": (S, S, S, S), "hsss": (S, S, S),
    "vadd": (V, V), "vsub": (V, V),
}

# coupling kinds (values are derived from the SM inputs by the library)
CPL_KINDS = ["gamma_ff", "z_ff", "w_ff", "g_qq", "ggg", "gggg", "wwz", "wwa",
             "wwh", "zzh", "wwhh", "zzhh", "hhh", "hhhh", "hbb", "wwww", "wwzz"]
CPL = {name: i for i, name in enumerate(CPL_KINDS)}
# What the library's coupling values fix whatever the SM inputs (its
# coupling_values; the same facts are checked there at create): every kind is
# real except the W W H and Z Z H couplings (complex masses in the
# complex-mass scheme); the fermion kinds with a vector coupling have g1 = g0;
# the W-fermion coupling is left-handed (g1 = 0), and a boson vertex has no g1.
# The generated kernels take them as constants, so the compiler drops the
# arithmetic on the zero parts; the values that remain are used as before.
CPL_COMPLEX = {"wwh", "zzh"}
CPL_G1_EQ_G0 = {"gamma_ff", "g_qq", "hbb"}
CPL_G1_FREE = {"z_ff"}


@dataclass(frozen=True)
class Leg:
    kind: int            # F, V or S
    incoming: bool
    flow: int = 1        # fermions: +1 particle, -1 antiparticle
    particle: int = P_ZERO
    colour: int = 1      # 1, 3 or 8
    name: str = ""


@dataclass(frozen=True)
class Coupling:
    kind: str
    charge: float = 0.0  # electric charge Q (gamma_ff, z_ff)
    t3: float = 0.0      # weak isospin T3 (z_ff)
    particle: int = P_ZERO  # reserved


@dataclass(frozen=True)
class Call:
    op: str
    ins: Tuple[int, ...]
    out: int             # output slot (currents) or amplitude index (amplitude ops)
    cpl: int = -1        # index into Process.couplings
    prop: int = P_ZERO   # propagator particle of a current


PS_FLAT, PS_BREIT_WIGNER = 0, 1


def validate_ps_tree(tree, legs, window):
    """the resonance tree: node 0 the collision, every final leg and every
    other node the daughter of exactly one node, daughters after their parent
    (final legs may be massive)"""
    nl, K = len(legs), len(tree)
    if not 1 <= K <= 16:
        raise ValueError("phase-space tree: 1..16 nodes")
    if not (window > 0 and math.isfinite(window)):
        raise ValueError("phase-space tree: window must be > 0")
    seen_legs, seen_nodes = [], []
    for k, (particle, mapping, d0, d1) in enumerate(tree):
        if k > 0 and (mapping not in (PS_FLAT, PS_BREIT_WIGNER) or not 0 <= particle < 5):
            raise ValueError(f"phase-space node {k}: bad mapping or particle")
        for d in (d0, d1):
            if d >= 0:
                if not 2 <= d < nl:
                    raise ValueError(f"phase-space node {k}: daughter {d} is not a final leg")
                seen_legs.append(d)
            else:
                j = -1 - d
                if not k < j < K:
                    raise ValueError(f"phase-space node {k}: daughter node {j} must come after it")
                seen_nodes.append(j)
    if sorted(seen_legs) != list(range(2, nl)) or sorted(seen_nodes) != list(range(1, K)):
        raise ValueError("phase-space tree: every final leg and node 1.. must be a daughter exactly once")


@dataclass
class Process:
    name: str
    legs: List[Leg]
    couplings: List[Coupling]
    calls: List[Call]
    n_amps: int
    n_flows: int
    jamp: List[List[Tuple[int, complex]]]       # per flow: (amp index, coefficient)
    colour: List[List[Fraction]]                # n_flows x n_flows
    helicities: List[Tuple[int, ...]]
    sqrt_s: float
    n_a_n_b: int
    symmetry: int
    cut_pt: float = 0.0
    cut_dr: float = 0.0
    cut_enabled: bool = False
    sm_overrides: dict = field(default_factory=dict)
    # Optional ordering table: when set, `calls` is a template over leg
    # *positions* 0..n_legs-1, evaluated once per ordering with position k
    # bound to external leg orderings[o][k]; flow o is the template's
    # amplitude combination jamp[o] for that ordering (all rows equal).
    orderings: Optional[List[Tuple[int, ...]]] = None
    # Optional flow map for ordering templates: flow f's jamp is
    # sum_o flow_map[f][o] * (ordering o's amplitude combination), small
    # integer coefficients; None means one flow per ordering.  With it the
    # colour matrix is n_flows x n_flows in the flows' basis.
    flow_map: Optional[List[List[int]]] = None
    # Optional resonance phase space (the paper's Appendix A at fixed sqrt_s):
    # nodes (particle, mapping, daughter0, daughter1); node 0 is the collision,
    # a daughter >= 0 is a final leg, -1 - k is node k (k > the parent's index).
    # None: RAMBO.  ps_window: the Breit-Wigner window factor (paper: 20).
    ps_tree: Optional[List[Tuple[int, int, int, int]]] = None
    ps_window: float = 20.0
    # Optional hadronic collision (the paper's Appendix A with parton densities
    # set to 1): (y_max, pt_min).  Node 0 of the tree is then a parton collision
    # at the hadronic sqrt_s, its two daughters generated in rapidity within
    # +-y_max, ln(m^2 + pT^2) from pt_min and azimuth; x_a, x_b follow.
    ps_hadronic: Optional[Tuple[float, float]] = None
    # Colour form of the code generator: "dense" (the colour matrix as it is) or
    # "compressed" (the paper's Sec. 5.4 decomposition: each row's entries
    # grouped by their distinct colour factors, one multiplication per factor
    # and row).  The compressed form runs on VALU with the flows' values in
    # registers: in FP32 always, in FP64 where they fit (bases below
    # MFMA_MIN_FLOWS flows; larger FP64 bases keep the dense MFMA form).
    colour_form: str = "dense"
    # Division of the amplitude program (the paper's Sec. 5.3): "fused" (one
    # kernel) or "split" (ordering templates: the orderings' amplitudes in one
    # kernel, written to device memory, the colour form in a second one,
    # launched one after the other per round of resident blocks).
    division: str = "fused"
    # Helicity combinations of the innermost helicity loops the kernel unrolls
    # (a code-generation setting, not part of the structure: unrolled loops
    # take table entries and the helicities of massless spinors as constants,
    # at the price of code size and registers)
    nest_unroll: int = 8
    # Waves per SIMD the kernel is compiled for (a code-generation setting: the
    # compiler keeps the registers within 512 / waves_per_simd per lane), and the
    # words per lane of the nest's LDS stash of event kinematics (with two waves
    # per SIMD two blocks must fit the CU's LDS)
    waves_per_simd: int = 1
    stash_words: int = 64
    # Waves per SIMD of the mixed-precision (FP32 chain) kernel when it differs
    # from the FP64 kernel's (0: the same); its registers are half as wide
    waves_per_simd_mixed: int = 0
    # Ordering templates: the number of innermost helicity loops of one
    # ordering's nest that the kernel unrolls (a code-generation setting)
    template_unroll: int = 0
    # Helicity schedule of the code generator (not part of the structure):
    # "nest" sums the full helicity product as a loop nest over the legs (each
    # call in the innermost loop its inputs need); "rows" evaluates the
    # helicity table row by row, every call in IR order with its momenta and
    # denominators formed where they are used and each amplitude added to its
    # flows at once, so that the live set follows the program (the paper's
    # recycling of temporaries, Sec. 5.5): for diagram sums too large for the
    # nest's registers.
    helicity_schedule: str = "nest"
    # Function division of the rows schedule (the paper's Sec. 5.3, a
    # code-generation setting): the amplitudes in this many groups, each
    # evaluated by a device function of its own (1: one piece)
    row_parts: int = 1
    # the same for the FP32 (mixed-precision) kernel; 0: as row_parts
    row_parts_mixed: int = 0

    def uses_colour_mfma(self):
        """The FP64 colour quadratic form runs on MFMA for ordering templates
        with at least MFMA_MIN_FLOWS flows; small colour bases stay on VALU."""
        return self.orderings is not None and self.n_flows >= MFMA_MIN_FLOWS

    def mixed_uses_mfma(self):
        """The FP32 (mixed-precision) colour form runs on MFMA: the dense form of
        an MFMA-sized basis; the compressed form never does."""
        return self.uses_colour_mfma() and self.colour_form == "dense"

    @property
    def n_legs(self):
        return len(self.legs)

    def n_slots(self):
        m = self.n_legs - 1
        for c in self.calls:
            if c.op not in AMP_OPS:
                m = max(m, c.out)
        return m + 1

    def colour_compression(self):
        """What the compressed colour form (Sec. 5.4) saves: the distinct
        factors it multiplies by (the non-zero entries on and above the
        diagonal, the off-diagonal ones doubled), the multiply-adds of the
        dense form (one per such entry) and the multiplications of the
        compressed one (one per distinct factor of each row)."""
        n = self.n_flows
        distinct, mults = set(), 0
        for f in range(n):
            vals = {Fraction(self.colour[f][g]) * (1 if g == f else 2) for g in range(f, n) if self.colour[f][g] != 0}
            distinct |= vals
            mults += len(vals)
        return {"flows": n, "distinct_factors": len(distinct), "dense_multiply_adds": n * (n + 1) // 2,
                "compressed_multiplications": mults}

    def colour_denominator(self):
        d = 1
        for row in self.colour:
            for x in row:
                d = d * Fraction(x).denominator // _gcd(d, Fraction(x).denominator)
        return d

    def validate(self):
        if self.colour_form not in COLOUR_FORMS:
            raise ValueError(f"unknown colour form {self.colour_form}")
        if self.division not in DIVISIONS:
            raise ValueError(f"unknown division {self.division}")
        if self.waves_per_simd not in (1, 2, 3, 4) or not 0 <= self.stash_words <= 64:
            raise ValueError("waves_per_simd in 1..4, stash_words in 0..64")
        if self.waves_per_simd_mixed not in (0, 1, 2, 3, 4):
            raise ValueError("waves_per_simd_mixed in 0..4")
        if self.row_parts < 1 or self.row_parts_mixed < 0:
            raise ValueError("row_parts >= 1, row_parts_mixed >= 0")
        if self.helicity_schedule not in ("nest", "rows"):
            raise ValueError(f"unknown helicity schedule {self.helicity_schedule}")
        if self.helicity_schedule == "rows" and self.orderings is not None:
            raise ValueError("the rows schedule applies to diagram call lists, not ordering templates")
        if self.division == "split" and self.orderings is None:
            raise ValueError("the split division applies to ordering templates")
        kinds = {i: leg.kind for i, leg in enumerate(self.legs)}
        amps = set()
        for k, c in enumerate(self.calls):
            if c.op not in OP:
                raise ValueError(f"call {k}: unknown op {c.op}")
            want = IN_KINDS[c.op]
            if len(c.ins) != len(want):
                raise ValueError(f"call {k}: {c.op} takes {len(want)} inputs")
            for s, w in zip(c.ins, want):
                if s not in kinds:
                    raise ValueError(f"call {k}: slot {s} used before it is defined")
                if kinds[s] != w:
                    raise ValueError(f"call {k}: slot {s} has the wrong kind for {c.op}")
            if c.op in AMP_OPS:
                if not (0 <= c.out < self.n_amps) or c.out in amps:
                    raise ValueError(f"call {k}: bad amplitude index {c.out}")
                amps.add(c.out)
            else:
                if c.out in kinds:
                    raise ValueError(f"call {k}: slot {c.out} defined twice")
                kinds[c.out] = OUT_KIND[c.op]
            if c.op in LINEAR_OPS:
                if c.cpl != -1:
                    raise ValueError(f"call {k}: {c.op} takes no coupling")
            elif not (0 <= c.cpl < len(self.couplings)):
                raise ValueError(f"call {k}: bad coupling index")
        if amps != set(range(self.n_amps)):
            raise ValueError("every amplitude index must be produced exactly once")
        n_rows = len(self.orderings) if self.orderings is not None else self.n_flows
        if len(self.jamp) != n_rows or len(self.colour) != self.n_flows:
            raise ValueError("jamp / colour sizes disagree with n_flows (jamp: one row per ordering "
                             "for templates)")
        for r in range(self.n_flows):
            for c in range(self.n_flows):
                if self.colour[r][c] != self.colour[c][r]:
                    raise ValueError("colour matrix must be symmetric")
        for h in self.helicities:
            if len(h) != self.n_legs:
                raise ValueError("helicity row length != number of legs")
        if self.flow_map is not None:
            if self.orderings is None:
                raise ValueError("a flow map needs an ordering table")
            if len(self.flow_map) != self.n_flows or any(len(r) != len(self.orderings) for r in self.flow_map):
                raise ValueError("flow map must be n_flows x n_orderings")
            for r in self.flow_map:
                if not any(r) or any(int(x) != x or not -127 <= x <= 127 for x in r):
                    raise ValueError("flow map rows: int8 coefficients, at least one non-zero")
        if self.orderings is not None:
            if self.flow_map is None and len(self.orderings) != self.n_flows:
                raise ValueError("one flow per ordering without a flow map")
            for o in self.orderings:
                if sorted(o) != list(range(self.n_legs)):
                    raise ValueError("orderings must be permutations of the legs")
            for row in self.jamp[1:]:
                if row != self.jamp[0]:
                    raise ValueError("ordering template: every jamp row is the same combination")
        if self.ps_tree is not None:
            validate_ps_tree(self.ps_tree, self.legs, self.ps_window)
        elif any(leg.particle != P_ZERO for leg in self.legs):
            raise ValueError("RAMBO phase space needs massless legs (give a resonance tree)")
        if self.ps_hadronic is not None:
            y_max, pt_min = self.ps_hadronic
            if self.ps_tree is None or not (y_max > 0 and math.isfinite(y_max)) or not pt_min >= 0:
                raise ValueError("hadronic collision: needs a tree, y_max > 0, pt_min >= 0")
            for d in self.ps_tree[0][2:4]:
                if d >= 0 and self.legs[d].particle == P_ZERO and not pt_min > 0:
                    raise ValueError("hadronic collision: a massless daughter of the collision needs pt_min > 0")
        return self

    # -------------------------------------------------------------- fingerprint
    def structure_bytes(self):
        """Canonical serialisation of the parts baked into the kernel: legs,
        couplings' kinds, calls, jamp coefficients, colour matrix, cut kind.
        Must match fingerprint() in the library (FNV-1a over the same bytes)."""
        b = bytearray()
        i32 = lambda x: b.extend(struct.pack("<i", int(x)))
        f64 = lambda x: b.extend(struct.pack("<d", float(x)))
        i32(self.n_legs)
        for leg in self.legs:
            for x in (leg.kind, int(leg.incoming), leg.flow, leg.particle, leg.colour):
                i32(x)
        i32(len(self.couplings))
        for c in self.couplings:
            i32(CPL[c.kind])
            f64(c.charge)
            f64(c.t3)
            i32(c.particle)
        i32(len(self.calls))
        for c in self.calls:
            i32(OP[c.op])
            ins = list(c.ins) + [-1] * (4 - len(c.ins))
            for x in ins:
                i32(x)
            for x in (c.out, c.cpl, c.prop):
                i32(x)
        i32(self.n_amps)
        i32(self.n_flows)
        for f, terms in enumerate(self.jamp):
            for a in range(self.n_amps):
                coef = 0j
                for (ai, cc) in terms:
                    if ai == a:
                        coef += cc
                f64(coef.real)
                f64(coef.imag)
        den = self.colour_denominator()
        for row in self.colour:
            for x in row:
                f64(float(Fraction(x) * den))
        f64(float(den))
        i32(int(self.cut_enabled))
        orders = self.orderings or []
        i32(len(orders))
        for o in orders:
            for x in o:
                i32(x)
        i32(0 if self.flow_map is None else 1)
        for r in self.flow_map or []:
            for x in r:
                i32(x)
        if self.ps_tree:
            i32(len(self.ps_tree))
            for node in self.ps_tree:
                for x in node:
                    i32(x)
            f64(self.ps_window)
        if self.ps_hadronic:
            i32(1)
            f64(self.ps_hadronic[0])
            f64(self.ps_hadronic[1])
        if self.colour_form != "dense" or self.division != "fused":
            i32(COLOUR_FORMS[self.colour_form])
            i32(DIVISIONS[self.division])
        return bytes(b)

    def fingerprint(self):
        h = 0xCBF29CE484222325
        for byte in self.structure_bytes():
            h ^= byte
            h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
        return h


def _gcd(a, b):
    while b:
        a, b = b, a % b
    return a


def all_helicities(legs, massive_vector_states=False):
    """All helicity combinations in lexicographic order, last leg fastest:
    fermions and massless vectors -1, +1; massive vectors -1, 0, +1; scalars 0."""
    choices = []
    for leg in legs:
        if leg.kind == S:
            choices.append((0,))
        elif leg.kind == V and leg.particle != P_ZERO:
            choices.append((-1, 0, 1))
        else:
            choices.append((-1, 1))
    out = [()]
    for ch in choices:
        out = [h + (c,) for h in out for c in ch]
    return out
