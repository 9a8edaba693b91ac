"""Process IRs of the benchmark workloads.

Each builder returns an ``ir.Process``: the HEGET-style call list with its
colour decomposition, written out the way the paper's generated integrands
call the HEGET functions (Sec. 5.1) with the colour factors of Sec. 4.2:
quark-gluon vertex -T^a x (FFV output), triple-gluon vertex i f^abc x (VVV
output), four-gluon vertex f f x (VVVV output, three colour structures).

Leg order (the momentum layout of heget_eval):
  ee_mumu      e-(in, +z) e+(in, -z) mu- mu+
  gg_ttbar_6f  g g b e+ nu_e bbar mu- nu_mu~      (t -> b e+ nu_e, tbar -> bbar mu- nu_mu~)
  ud_udhh_4b   u d u d b bbar b bbar              (H -> b bbar twice)
  gg_4g        g g g g g g   (120 trace-basis flows; gg_4g_ddm: the 24 evaluated orderings as flows)
  uu_ttggg     u ubar t tbar g g g   (393 Feynman diagrams, 48 colour flows; uu_ttg, uu_ttgg: 1, 2 gluons)
"""
import copy
import dataclasses
import functools
from fractions import Fraction

from .. import ir
from ..ir import F, V, S, P_ZERO, P_W, P_Z, P_TOP, P_H, Leg, Call, Coupling, Process

Q_U, Q_D, Q_E = 2.0 / 3.0, -1.0 / 3.0, -1.0


def ee_mumu(sqrt_s=200.0):
    """e+ e- -> mu+ mu- via s-channel photon and Z (2 diagrams, 1 colour flow)."""
    legs = [Leg(F, True, +1, name="e-"), Leg(F, True, -1, name="e+"),
            Leg(F, False, +1, name="mu-"), Leg(F, False, -1, name="mu+")]
    cpl = [Coupling("gamma_ff", charge=Q_E), Coupling("z_ff", charge=Q_E, t3=-0.5)]
    calls = [
        Call("jio", (0, 1), 4, 0, P_ZERO),      # photon current from e- (|fi>) and e+ (<fo|)
        Call("iov", (3, 2, 4), 0, 0),           # <mu-| A |mu+>
        Call("jio", (0, 1), 5, 1, P_Z),         # Z current
        Call("iov", (3, 2, 5), 1, 1),
    ]
    # the whole 16-combination nest unrolled (8.8 -> 7.6 us per 65,536 events)
    return Process("ee_mumu", legs, cpl, calls, n_amps=2, n_flows=1,
                   jamp=[[(0, 1.0), (1, 1.0)]], colour=[[Fraction(1)]],
                   helicities=ir.all_helicities(legs), sqrt_s=sqrt_s, n_a_n_b=1, symmetry=1,
                   nest_unroll=16).validate()


def gg_ttbar_6f(sqrt_s=1000.0):
    """g g -> t tbar, t -> b e+ nu_e, tbar -> bbar mu- nu_mu~ with Breit-Wigner
    tops and W's: s-channel gluon, t- and u-channel top (3 diagrams).

    Colour: T = (T^a T^b)_ij (gluon 0 next to the top), U = (T^b T^a)_ij,
    S = (i f^abc)(-T^c) = -[T^a, T^b].  Flows are the two orderings
    {(T^a T^b)_ij, (T^b T^a)_ij}; colour matrix [[16/3, -2/3], [-2/3, 16/3]]."""
    legs = [Leg(V, True, colour=8, name="g"), Leg(V, True, colour=8, name="g"),
            Leg(F, False, +1, colour=3, name="b"), Leg(F, False, -1, name="e+"),
            Leg(F, False, +1, name="nu_e"), Leg(F, False, -1, colour=3, name="bbar"),
            Leg(F, False, +1, name="mu-"), Leg(F, False, -1, name="nu_mu~")]
    cpl = [Coupling("w_ff"), Coupling("g_qq"), Coupling("ggg")]
    W, GQ, GGG = 0, 1, 2
    calls = [
        Call("jio", (3, 4), 8, W, P_W),          # W+ -> e+ nu_e
        Call("jio", (7, 6), 9, W, P_W),          # W- -> mu- nu_mu~
        Call("fvo", (2, 8), 10, W, P_TOP),       # <t| from <b| and the W+
        Call("fvi", (5, 9), 11, W, P_TOP),       # |tbar> from |bbar> and the W-
        Call("jvv", (0, 1), 12, GGG, P_ZERO),    # s-channel gluon
        Call("iov", (11, 10, 12), 0, GQ),
        Call("fvo", (10, 0), 13, GQ, P_TOP),     # gluon 0 next to the top
        Call("iov", (11, 13, 1), 1, GQ),
        Call("fvo", (10, 1), 14, GQ, P_TOP),     # gluon 1 next to the top
        Call("iov", (11, 14, 0), 2, GQ),
    ]
    jamp = [[(1, 1.0), (0, -1.0)], [(2, 1.0), (0, 1.0)]]
    colour = [[Fraction(16, 3), Fraction(-2, 3)], [Fraction(-2, 3), Fraction(16, 3)]]
    # the whole helicity nest unrolled (256 combinations, every helicity a constant:
    # the compiler shares each current between the combinations that need it and
    # drops the arithmetic on the structural zeros), compiled for two waves per
    # SIMD; measured on MI355X per 2^20 events (FP64 / mixed): 32 combinations
    # 0.481 / 0.316 ms, 128 0.229 / 0.150 ms, 256 0.170 / 0.138 ms, 256 at two
    # waves per SIMD 0.142 / 0.138 ms; on the current kernels the FP32 kernel at
    # three waves (168 registers, 11 spilled) 0.1001 ms against 0.1024 at two
    return Process("gg_ttbar_6f", legs, cpl, calls, n_amps=3, n_flows=2, jamp=jamp, colour=colour,
                   helicities=ir.all_helicities(legs), sqrt_s=sqrt_s, n_a_n_b=64, symmetry=1,
                   nest_unroll=256, waves_per_simd=2, stash_words=36, waves_per_simd_mixed=3).validate()


def gg_ttbar_6f_bw(sqrt_s=1000.0):
    """The C1 process with the paper's resonance phase space (Appendix A) in
    place of RAMBO: g g -> t t~ at fixed sqrt_s, t -> b W+ (-> e+ nu_e),
    t~ -> b~ W- (-> mu- nu_mu~), each top and W mass Breit-Wigner mapped within
    min(20, m / Gamma) widths of its pole."""
    import dataclasses
    BW = ir.PS_BREIT_WIGNER
    tree = [(P_ZERO, ir.PS_FLAT, -2, -3),      # the collision -> t, t~
            (P_TOP, BW, 2, -4),                # t -> b W+
            (P_TOP, BW, 5, -5),                # t~ -> b~ W-
            (P_W, BW, 3, 4),                   # W+ -> e+ nu_e
            (P_W, BW, 6, 7)]                   # W- -> mu- nu_mu~
    # with the resonance tree's phase space in the kernel: the whole nest unrolled
    # at one wave per SIMD (per 2^20 events, FP64 / mixed: 0.189 / 0.148 ms; two
    # waves 0.201 / 0.148 ms)
    return dataclasses.replace(gg_ttbar_6f(sqrt_s), name="gg_ttbar_6f_bw", ps_tree=tree,
                               ps_window=20.0, nest_unroll=256, waves_per_simd=1, stash_words=64,
                               waves_per_simd_mixed=0).validate()


def ud_udhh_4b(sqrt_s=2000.0):
    """u d -> u d H H via W W and Z Z fusion, each H -> b bbar (16 diagrams).

    For each fusion class V in {Z Z, W W} and b pairing in {(b0 bbar1)(b2 bbar3),
    (b0 bbar3)(b2 bbar1)}: contact VVHH, s-channel H* -> H H, and t-/u-channel
    V exchange.  The W W class pairs the quark lines differently from Z Z and the
    second b pairing swaps two identical fermions: each carries a Fermi sign -1.
    Colour flows (quark pairing) x (b pairing), matrix [[9,3],[3,9]] (x) [[9,3],[3,9]]."""
    legs = [Leg(F, True, +1, colour=3, name="u"), Leg(F, True, +1, colour=3, name="d"),
            Leg(F, False, +1, colour=3, name="u"), Leg(F, False, +1, colour=3, name="d"),
            Leg(F, False, +1, colour=3, name="b"), Leg(F, False, -1, colour=3, name="bbar"),
            Leg(F, False, +1, colour=3, name="b"), Leg(F, False, -1, colour=3, name="bbar")]
    cpl = [Coupling("z_ff", charge=Q_U, t3=0.5), Coupling("z_ff", charge=Q_D, t3=-0.5),
           Coupling("w_ff"), Coupling("hbb"),
           Coupling("zzh"), Coupling("wwh"), Coupling("zzhh"), Coupling("wwhh"), Coupling("hhh")]
    ZU, ZD, W, HB, ZZH, WWH, ZZHH, WWHH, HHH = range(9)
    calls = []
    slot = [8]

    def cur(op, ins, cp, prop):
        s = slot[0]
        slot[0] += 1
        calls.append(Call(op, ins, s, cp, prop))
        return s
    # Higgs currents for both b pairings
    hA = (cur("hio", (5, 4), HB, P_H), cur("hio", (7, 6), HB, P_H))
    hB = (cur("hio", (7, 4), HB, P_H), cur("hio", (5, 6), HB, P_H))
    classes = [
        # (V1 current, V2 current, boson, vvh coupling, vvhh coupling, sign)
        (cur("jio", (0, 2), ZU, P_Z), cur("jio", (1, 3), ZD, P_Z), P_Z, ZZH, ZZHH, +1.0),
        (cur("jio", (0, 3), W, P_W), cur("jio", (1, 2), W, P_W), P_W, WWH, WWHH, -1.0),
    ]
    amp = 0
    jamp = [[] for _ in range(4)]
    for ci, (v1, v2, boson, c3, c4, sgn) in enumerate(classes):
        hs = cur("hvv", (v1, v2), c3, P_H)
        for pi, (h1, h2) in enumerate((hA, hB)):
            psign = sgn * (1.0 if pi == 0 else -1.0)
            flow = ci + 2 * pi
            calls.append(Call("vvss", (v1, v2, h1, h2), amp, c4)); jamp[flow].append((amp, psign)); amp += 1
            calls.append(Call("sss", (hs, h1, h2), amp, HHH)); jamp[flow].append((amp, psign)); amp += 1
            vt = cur("jvs", (v1, h1), c3, boson)
            calls.append(Call("vvs", (vt, v2, h2), amp, c3)); jamp[flow].append((amp, psign)); amp += 1
            vu = cur("jvs", (v1, h2), c3, boson)
            calls.append(Call("vvs", (vu, v2, h1), amp, c3)); jamp[flow].append((amp, psign)); amp += 1
    cq = [[9, 3], [3, 9]]
    colour = [[Fraction(cq[a % 2][b % 2] * cq[a // 2][b // 2]) for b in range(4)] for a in range(4)]
    # the whole helicity nest unrolled: per 2^21 events on MI355X (FP64 / mixed)
    # 64 combinations 0.712 / 0.435 ms, 128 0.609 / 0.373 ms, 256 0.438 / 0.328 ms
    return Process("ud_udhh_4b", legs, cpl, calls, n_amps=amp, n_flows=4, jamp=jamp, colour=colour,
                   helicities=ir.all_helicities(legs), sqrt_s=sqrt_s, n_a_n_b=9, symmetry=4,
                   sm_overrides={"complex_mass": 1}, nest_unroll=256).validate()


def ud_udhhh(sqrt_s=2000.0):
    """u d -> u d H H H via W W and Z Z fusion with external Higgs bosons (the
    paper's test of the quartic scalar vertex, Sec. 3.5 and 4.2.8): per fusion
    class, every tree of VVH, VVHH, HHH and HHHH that joins the two vector
    currents to the three Higgs bosons, 25 diagrams:

      one attachment   VVH -> H* -> H H H (quartic), VVH -> H* -> H H*(-> H H) (3),
                       VVHH(H, H*(-> H H)) (3);
      two attachments  VVH(H) then VVH(H* -> H H), VVH(H* -> H H) then VVH(H),
                       VVH(H) then VVHH(H H), VVHH(H H) then VVH(H) (3 each);
      three            VVH(H) VVH(H) VVH(H) in each order (6).

    The W W class pairs the quark lines differently from Z Z: Fermi sign -1.
    Colour flows: the two quark pairings, matrix [[9, 3], [3, 9]].  Phase
    space: a flat tree u (d (H (H H))) with the Higgs mass on the final legs."""
    legs = [Leg(F, True, +1, colour=3, name="u"), Leg(F, True, +1, colour=3, name="d"),
            Leg(F, False, +1, colour=3, name="u"), Leg(F, False, +1, colour=3, name="d"),
            Leg(S, False, particle=P_H, name="H"), Leg(S, False, particle=P_H, name="H"),
            Leg(S, False, particle=P_H, name="H")]
    cpl = [Coupling("z_ff", charge=Q_U, t3=0.5), Coupling("z_ff", charge=Q_D, t3=-0.5),
           Coupling("w_ff"), Coupling("zzh"), Coupling("wwh"), Coupling("zzhh"), Coupling("wwhh"),
           Coupling("hhh"), Coupling("hhhh")]
    ZU, ZD, W, ZZH, WWH, ZZHH, WWHH, HHH, HHHH = range(9)
    calls = []
    slot = [7]

    def cur(op, ins, cp, prop):
        s = slot[0]
        slot[0] += 1
        calls.append(Call(op, ins, s, cp, prop))
        return s
    splits = [(4, 5, 6), (5, 4, 6), (6, 4, 5)]          # Higgs i alone, pair (j, k)
    pair = {(j, k): cur("hss", (j, k), HHH, P_H) for _, j, k in splits}
    classes = [
        (cur("jio", (0, 2), ZU, P_Z), cur("jio", (1, 3), ZD, P_Z), P_Z, ZZH, ZZHH, +1.0),
        (cur("jio", (0, 3), W, P_W), cur("jio", (1, 2), W, P_W), P_W, WWH, WWHH, -1.0),
    ]
    amp = 0
    jamp = [[], []]

    def add(op, ins, cp, flow, sign):
        nonlocal amp
        calls.append(Call(op, ins, amp, cp))
        jamp[flow].append((amp, sign))
        amp += 1
    for flow, (v1, v2, boson, c3, c4, sgn) in enumerate(classes):
        hs = cur("hvv", (v1, v2), c3, P_H)
        add("ssss", (hs, 4, 5, 6), HHHH, flow, sgn)
        for i, j, k in splits:
            add("sss", (hs, i, pair[(j, k)]), HHH, flow, sgn)
            add("vvss", (v1, v2, i, pair[(j, k)]), c4, flow, sgn)
        # each vector current is used right after it is made (short live ranges)
        for i, j, k in splits:
            vt = cur("jvs", (v1, i), c3, boson)            # V1 emits Higgs i first
            add("vvs", (vt, v2, pair[(j, k)]), c3, flow, sgn)
            add("vvss", (vt, v2, j, k), c4, flow, sgn)
            for b, c in ((j, k), (k, j)):
                vtt = cur("jvs", (vt, b), c3, boson)
                add("vvs", (vtt, v2, c), c3, flow, sgn)
            vtp = cur("jvs", (v1, pair[(j, k)]), c3, boson)
            add("vvs", (vtp, v2, i), c3, flow, sgn)
            vss = cur("jvss", (v1, j, k), c4, boson)
            add("vvs", (vss, v2, i), c3, flow, sgn)
    assert amp == 50
    colour = [[Fraction(9), Fraction(3)], [Fraction(3), Fraction(9)]]
    tree = [(P_ZERO, ir.PS_FLAT, 2, -2), (P_ZERO, ir.PS_FLAT, 3, -3), (P_ZERO, ir.PS_FLAT, 4, -4),
            (P_ZERO, ir.PS_FLAT, 5, 6)]
    # the FP32 kernel at two waves per SIMD (per 2^20 events 0.182 ms against
    # 0.216 ms at one, where it kept 324 registers); FP64 at one
    return Process("ud_udhhh", legs, cpl, calls, n_amps=amp, n_flows=2, jamp=jamp, colour=colour,
                   helicities=ir.all_helicities(legs), sqrt_s=sqrt_s, n_a_n_b=9, symmetry=6,
                   sm_overrides={"complex_mass": 1}, ps_tree=tree, nest_unroll=64,
                   waves_per_simd_mixed=2).validate()


def ww_ww(sqrt_s=1000.0):
    """W- W+ -> W- W+ with on-shell external W bosons (massive external vector
    wavefunctions and the weak quartic vertex, Sec. 4.2.3-4.2.5): the W W W W
    contact, photon and Z exchange in the s and t channels through W W V, and
    Higgs exchange in both channels, 7 diagrams.  Arguments in the HELAS order:
    the first W of a vertex flows in as a W- (an incoming W- or an outgoing
    W+), the second as a W+.  Phase space: the two-body decay of the collision
    with the W mass on every leg."""
    legs = [Leg(V, True, particle=P_W, name="W-"), Leg(V, True, particle=P_W, name="W+"),
            Leg(V, False, particle=P_W, name="W-"), Leg(V, False, particle=P_W, name="W+")]
    cpl = [Coupling("wwa"), Coupling("wwz"), Coupling("wwww"), Coupling("wwh")]
    WWA, WWZ, WWWW, WWH = range(4)
    calls = [Call("wwww", (0, 1, 3, 2), 0, WWWW)]
    slot, amp = 4, 1
    # s channel: W-(0) W+(1) -> V* -> W-(2) W+(3); t channel: W-(0) -> W-(2) V*, V* W+(1) -> W+(3)
    for (a, b), (c, d) in (((0, 1), (3, 2)), ((0, 2), (3, 1))):
        for cp, prop in ((WWA, P_ZERO), (WWZ, P_Z)):
            calls.append(Call("jvv", (a, b), slot, cp, prop))
            calls.append(Call("vvv", (c, d, slot), amp, cp))
            slot += 1
            amp += 1
        calls.append(Call("hvv", (a, b), slot, WWH, P_H))
        calls.append(Call("vvs", (c, d, slot), amp, WWH))
        slot += 1
        amp += 1
    tree = [(P_ZERO, ir.PS_FLAT, 2, 3)]
    return Process("ww_ww", legs, cpl, calls, n_amps=amp, n_flows=1, jamp=[[(k, 1.0) for k in range(amp)]],
                   colour=[[Fraction(1)]], helicities=ir.all_helicities(legs), sqrt_s=sqrt_s, n_a_n_b=1,
                   symmetry=1, sm_overrides={"complex_mass": 1}, ps_tree=tree).validate()


@functools.lru_cache(maxsize=None)
def _gluons(n, basis):
    from .gluons import gg_ng
    return gg_ng(n, basis=basis)


def gg_ttbar_6f_had(sqrt_s=14000.0, y_max=2.5):
    """C1 at a hadron collider of energy sqrt_s (the paper's Appendix A): the
    top pair from a gluon-gluon collision with x_a, x_b from momentum
    conservation and parton densities set to 1 (CTEQ6L1 is absent), the tops
    in rapidity within +-y_max, ln(m_t^2 + pT^2) and azimuth, each decaying
    through the resonance tree of gg_ttbar_6f_bw.  sigma = integral dx_a dx_b
    sigma_hat(x_a x_b s) over |y_t| < y_max."""
    return dataclasses.replace(gg_ttbar_6f_bw(), name="gg_ttbar_6f_had", sqrt_s=sqrt_s,
                               ps_hadronic=(y_max, 0.0)).validate()


def by_name(name):
    gluon = {"gg_4g": (6, "trace"), "gg_4g_ddm": (6, "ddm"), "gg_5g_ddm": (7, "ddm")}
    if name in gluon:
        # the colour matrices of the larger bases take seconds to build: built once, copied out
        return copy.deepcopy(_gluons(*gluon[name]))
    # the same processes with the colour form compressed to its distinct colour
    # factors (Sec. 5.4): the FP32 kernels run it on VALU
    compressed = {"gg_4g_cf": "gg_4g", "gg_5g_cf": "gg_5g_ddm", "uu_ttggg_cf": "uu_ttggg"}
    if name in compressed:
        p = by_name(compressed[name])
        p.name, p.colour_form = name, "compressed"
        return p.validate()
    # the amplitude program divided into two kernels (Sec. 5.3): the orderings'
    # amplitudes, then the colour form
    split = {"gg_5g_split": "gg_5g_ddm"}
    if name in split:
        p = by_name(split[name])
        p.name, p.division = name, "split"
        return p.validate()
    # u ubar -> t tbar + n gluons: every Feynman diagram, its colour in a basis of flows
    quark_lines = {"uu_ttg": 1, "uu_ttgg": 2, "uu_ttggg": 3}
    if name in quark_lines:
        from .quark_lines import uu_ttbar_gluons
        return uu_ttbar_gluons(quark_lines[name])
    return {"ee_mumu": ee_mumu, "gg_ttbar_6f": gg_ttbar_6f, "gg_ttbar_6f_bw": gg_ttbar_6f_bw,
            "ud_udhh_4b": ud_udhh_4b, "ud_udhhh": ud_udhhh, "ww_ww": ww_ww,
            "gg_ttbar_6f_had": gg_ttbar_6f_had}[name]()
