"""Algorithmic floating-point operation counts of the amplitude path.

Counted from the device functions as written (heget_device.hpp): a complex
multiply is 6 flops, a complex add 2, a real-times-complex product 2; square
roots, divisions and transcendentals are counted as one operation each.  Per
event, the helicity loop executes the external wavefunctions, every call of
the IR, the jamp sums and the colour form once per helicity combination; the
momenta, internal-line momenta and propagator denominators are formed once.
"""
from .ir import AMP_OPS, F, V, S, P_ZERO, P_W, P_Z

CMUL, CADD, RMUL = 6, 2, 2
DOT_CC = 4 * CMUL + 3 * CADD          # 30: complex four-vector dot
DOT_CR = 4 * RMUL + 3 * CADD          # 14: complex . real four-vector
WEYL_C = 4 + 2 * (2 + 2 * CMUL + CADD)  # 36: 2x2 sigma.V on a 2-spinor, V complex
WEYL_R = 2 * (1 + RMUL + CMUL + CADD)   # 22: the same with a real momentum
PROP_MASSLESS = 4 * CMUL              # 24: A / D
PROP_MASSIVE = DOT_CR + CMUL + 4 * (RMUL + CADD) + PROP_MASSLESS   # 60: unitary gauge

OP_FLOPS = {
    "iov": 2 * WEYL_C + 2 * (3 * CMUL + CADD) + CADD,           # 114
    "ffv_bra": 2 * WEYL_C + 4 * CMUL,                           # 96: <fo| Vslash (g0 P_L + g1 P_R)
    "spinor_dot": 4 * CMUL + 3 * CADD,                          # 30
    "vs_bra": 5 * CMUL,                                         # 30: (gc s) x v, four components
    "vec_dot": 4 * CMUL + 3 * CADD,                             # 30: Minkowski product
    "vvv_r3": 12 + DOT_CC + 2 * DOT_CR + 3 * RMUL + 4 * (RMUL + 2 * CMUL + 2 * CADD),   # 146
    "gggg_r4": 2 * DOT_CC + 2 * RMUL + 4 * (2 * CMUL + CADD),   # 120
    "gggg_r2": 2 * DOT_CC + 2 * RMUL + 4 * (2 * CMUL + CADD),   # 120
    "ffv_current": 8 * CMUL + 4 * (2 * CMUL + 3 * CADD),        # 120
    "fvi": 2 * WEYL_C + 4 * CMUL + 2 * WEYL_R + 2 + 4 * (2 * CMUL + CADD),   # 198
    "fvo": 2 * WEYL_C + 4 * CMUL + 2 * WEYL_R + 2 + 4 * (2 * CMUL + CADD),   # 198
    "ios": 2 * (2 * CMUL + CADD) + 2 * CMUL + CADD + CMUL,      # 48
    "hio": 2 * (2 * CMUL + CADD) + 2 * CMUL + CADD + CMUL,      # 48
    "fsi": 4 * CMUL + 2 * WEYL_R + CMUL + RMUL + 4 * (2 * CMUL + CADD),      # 134
    "fso": 4 * CMUL + 2 * WEYL_R + CMUL + RMUL + 4 * (2 * CMUL + CADD),      # 134
    "vvv": 12 + 3 * DOT_CC + 3 * DOT_CR + 3 * CMUL + 2 * CADD + RMUL,       # 168
    "jvv_vertex": 4 + 8 + 8 + DOT_CC + 2 * DOT_CR + 4 * (RMUL + 2 * CMUL + 2 * CADD + RMUL) + 4,  # 162
    "gggg": 4 * DOT_CC + 2 * CMUL + CADD + RMUL,                # 136
    "jggg_vertex": 2 * DOT_CC + 2 * RMUL + 4 * (2 * CMUL + CADD),            # 120
    "wwww": 2 * (4 * DOT_CC + 2 * CMUL + CADD + RMUL) + CADD,   # 274
    "jwww_vertex": 3 * DOT_CC + 4 * (4 * CMUL + 3 * CADD) + 4 * RMUL,        # 218
    "vvs": DOT_CC + 2 * CMUL,                                   # 42
    "jvs_vertex": CMUL + 4 * CMUL,                              # 30
    "hvv": DOT_CC + 2 * CMUL,                                   # 42
    "vvss": DOT_CC + 3 * CMUL,                                  # 48
    "jvss_vertex": 2 * CMUL + 4 * CMUL,                         # 36
    "hvvs": DOT_CC + 3 * CMUL,                                  # 48
    "sss": 3 * CMUL,                                            # 18
    "hss": 3 * CMUL,                                            # 18
    "ssss": 4 * CMUL,                                           # 24
    "hsss": 4 * CMUL,                                           # 24
    "vadd": 4 * CADD,                                           # 8
    "vsub": 4 * CADD,                                           # 8
}
EXTERNAL = {"f_massless": 6, "f_massive": 30, "v": 24, "s": 0}
MASSIVE = {P_W, P_Z}


def call_flops(c):
    op = c.op
    prop = PROP_MASSIVE if c.prop in MASSIVE else PROP_MASSLESS
    if op == "jio":
        return OP_FLOPS["ffv_current"] + prop
    if op in ("jvv", "jggg", "jwww", "jvs", "jvss"):
        return OP_FLOPS[op + "_vertex"] + prop
    return OP_FLOPS[op]


def per_helicity(proc):
    """flops of one helicity combination of one event"""
    n = 0
    for leg in proc.legs:
        if leg.kind == F:
            n += EXTERNAL["f_massless"] if leg.particle == P_ZERO else EXTERNAL["f_massive"]
        elif leg.kind == V:
            n += EXTERNAL["v"]
    reps = len(proc.orderings) if proc.orderings else 1             # ordering template
    n += reps * sum(call_flops(c) for c in proc.calls)
    if proc.orderings:
        n += reps * CADD * max(len(proc.jamp[0]) - 1, 0)
    else:
        n += sum(CADD * max(len(t) - 1, 0) for t in proc.jamp)      # jamp sums
    return n + colour_flops(proc)


def colour_flops(proc):
    """the colour quadratic form of one helicity of one event"""
    nf = proc.n_flows
    if proc.uses_colour_mfma():
        return colour_mfma_flops(proc)
    return nf * 4 + (nf * (nf - 1) // 2) * 4 + 2


def colour_mfma_flops(proc):
    """Algorithmic flops of the MFMA colour form for one helicity of one event:
    the flow-map sums (a complex add per term), the product of C with X^T over
    the upper triangle of 16 x 16 blocks (C is symmetric; the diagonal blocks
    whole), for the real and the imaginary parts, and the dot products (2 n_f
    each).  The zero padding of the last tiles is not counted."""
    nf = proc.n_flows
    terms = sum(sum(1 for x in row if x) for row in proc.flow_map) if proc.flow_map else nf
    nb = (nf + 15) // 16
    sizes = [min(16, nf - 16 * b) for b in range(nb)]
    pairs = sum(sizes[b] * sum(sizes[b:]) for b in range(nb))
    return CADD * terms + 2 * (2 * pairs) + 2 * (2 * nf)


def colour_mfma_flops_executed(proc):
    """flops the MFMA instructions execute per helicity and event, padding
    included: tile fo runs the k-steps s >= 4 fo"""
    nks, nfo = (proc.n_flows + 3) // 4, (proc.n_flows + 15) // 16
    steps = sum(nks - 4 * fo for fo in range(nfo))
    return 2 * (2 * 16 * 4 * steps)


def per_event(proc, n_hel=None):
    """flops of one event: the helicity sum plus the per-event denominators.
    With the full helicity product (n_hel None) a straight-line IR runs as the
    helicity loop nest (nest.schedule, less what its call tables save); a
    table of n_hel rows runs row by row."""
    n_cur = sum(1 for c in proc.calls if c.op not in AMP_OPS and c.op not in ("vadd", "vsub"))
    if n_hel is None and not proc.orderings:
        from . import nest
        sc = nest.schedule(proc)
        saved = sum(t[2] for t in nest.tables(proc, sc, nest.unrolled_levels(sc)).values())
        return sc.flops_per_event - saved + n_cur * (7 + 8)
    if n_hel is None:
        # ordering template: per ordering, the momenta and denominators once and
        # the helicity nest; per helicity, the colour form over all orderings
        from . import nest
        nh = len(proc.helicities)
        return (nest.template_schedule(proc).flops_per_event + len(proc.orderings) * n_cur * (7 + 8)
                + nh * colour_flops(proc))
    nh = len(proc.helicities) if n_hel is None else n_hel
    if proc.orderings:
        # per-ordering momenta and denominators are formed inside the helicity loop
        return nh * (per_helicity(proc) + len(proc.orderings) * n_cur * (7 + 8))
    return nh * per_helicity(proc) + n_cur * (7 + 8)
