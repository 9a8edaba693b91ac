"""Helicity loop nest for straight-line process IRs.

Summing |M|^2 over the full product of helicity states, a current or an
amplitude depends only on the helicities of the external legs that feed it.
Running the sum as nested loops, one per leg, and computing every external
wavefunction and every call in the innermost loop that fixes all of its legs'
helicities evaluates each distinct value once per combination of the legs it
depends on, instead of once per full helicity combination.  The terms summed
are the same products of the same factors, so |M|^2 is unchanged up to the
order of the final additions.

`plan` chooses the loop order (outermost first) that minimises the flop count
under the model of `flops.call_flops`, by exhaustive search over the orders of
the legs with more than one state (a greedy order beyond nine such legs).
"""
import itertools
from dataclasses import dataclass
from typing import Dict, List, Tuple

from . import flops
from .ir import AMP_OPS, OUT_KIND, F, V, S, P_ZERO


@dataclass
class Plan:
    order: List[int]               # legs, outermost loop first
    choices: List[Tuple[int, ...]]  # helicity states of every leg
    call_level: List[int]          # loop level (index into order) of every call
    leg_level: Dict[int, int]      # loop level of every leg's external wavefunction
    flops_per_event: int           # model flops of one event's helicity sum
    bra_level: List[object]        # FFV amplitudes split as <fo|V| . |fi>: level of the bra, else None


def leg_choices(leg):
    if leg.kind == S:
        return (0,)
    if leg.kind == V and leg.particle != P_ZERO:
        return (-1, 0, 1)
    return (-1, 1)


def _ext_flops(leg):
    if leg.kind == F:
        return flops.EXTERNAL["f_massless"] if leg.particle == P_ZERO else flops.EXTERNAL["f_massive"]
    return flops.EXTERNAL["v"] if leg.kind == V else flops.EXTERNAL["s"]


def call_dependencies(proc):
    """legs whose helicities each call's value depends on"""
    dep = {k: frozenset((k,)) for k in range(proc.n_legs)}
    out = []
    for c in proc.calls:
        d = frozenset().union(*(dep[x] for x in c.ins))
        out.append(d)
        if c.op not in AMP_OPS:
            dep[c.out] = d
    return out


def bra_dependencies(proc, deps):
    """legs the bra <fo| Vslash of each FFV amplitude depends on (None for other calls)"""
    dep = {k: frozenset((k,)) for k in range(proc.n_legs)}
    out = []
    for c, d in zip(proc.calls, deps):
        out.append(dep[c.ins[1]] | dep[c.ins[2]] if c.op == "iov" else None)
        if c.op not in AMP_OPS:
            dep[c.out] = d
    return out


def _levels(order, deps, bdeps):
    pos = {L: i for i, L in enumerate(order)}
    lvl = [max(pos[L] for L in d) for d in deps]
    blvl = [max(pos[L] for L in b) if b is not None else None for b in bdeps]
    # split an FFV amplitude only where its bra sits in an outer loop
    blvl = [b if b is not None and b < l else None for b, l in zip(blvl, lvl)]
    return pos, lvl, blvl


def _cost(order, choices, deps, bdeps, call_cost, ext_cost, tail_cost):
    pos, lvl, blvl = _levels(order, deps, bdeps)
    mult, m = [], 1
    for L in order:
        m *= len(choices[L])
        mult.append(m)
    c = sum(ext_cost[L] * mult[pos[L]] for L in order)
    for cc, l, b in zip(call_cost, lvl, blvl):
        if b is None:
            c += cc * mult[l]
        else:
            c += flops.OP_FLOPS["ffv_bra"] * mult[b] + flops.OP_FLOPS["spinor_dot"] * mult[l]
    return c + tail_cost * mult[-1]


def plan(proc):
    if proc.orderings is not None:
        raise ValueError("the helicity nest applies to straight-line IRs")
    nl = proc.n_legs
    choices = [leg_choices(leg) for leg in proc.legs]
    deps = call_dependencies(proc)
    bdeps = bra_dependencies(proc, deps)
    call_cost = [flops.call_flops(c) for c in proc.calls]
    ext_cost = [_ext_flops(leg) for leg in proc.legs]
    nf = proc.n_flows
    tail = sum(flops.CADD * max(len(t) - 1, 0) for t in proc.jamp) + nf * 4 + (nf * (nf - 1) // 2) * 4 + 2
    fixed = [L for L in range(nl) if len(choices[L]) == 1]
    free = [L for L in range(nl) if len(choices[L]) > 1]
    args = (choices, deps, bdeps, call_cost, ext_cost, tail)
    if len(free) <= 9:
        best = min(itertools.permutations(free), key=lambda perm: _cost(fixed + list(perm), *args))
        order = fixed + list(best)
    else:
        order = list(fixed)
        rest = list(free)
        while rest:
            # next loop: the leg whose addition keeps the remaining cost lowest
            L = min(rest, key=lambda x: _cost(order + [x] + [y for y in rest if y != x], *args))
            order.append(L)
            rest.remove(L)
    pos, call_level, bra_level = _levels(order, deps, bdeps)
    return Plan(order, choices, call_level, {L: pos[L] for L in range(nl)}, _cost(order, *args), bra_level)


# innermost loops unrolled up to this many helicity combinations, unless the
# process sets its own (ir.Process.nest_unroll)
UNROLL_INNER_COMBINATIONS = 8
# tables of calls: at most this many words per lane (in the arithmetic type)
TABLE_WORDS = 48

# ------------------------------------------------------------------ schedule
ONE = None   # an argument slot replaced by the scalar 1 (its value deferred as a factor)


@dataclass
class Item:
    kind: str          # "ext", "call", "mat", "bra", "dot", "vbra", "vdot", "ksum", "bsum", "bacc", "kdot", "jamp"
    level: int         # loop level (-1: before the loops)
    data: tuple
    flops: int


@dataclass
class Schedule:
    order: List[int]
    choices: List[Tuple[int, ...]]
    items: List[Item]          # in dependency order
    flops_per_event: int       # model flops of the loop nest, per event
    unroll: int = 8            # helicity combinations of the innermost loops the kernel unrolls


# each combined bra joins its jamp group's sum right after it is formed (bras
# of outer loops first, at the top of the sum's loop), so that the bras of a
# group do not all stay live until one sum takes them
EARLY_BRA_SUMS = True


def _early_bra_sums(items, proc):
    """the items with every bra sum ("bsum") replaced by a chain of partial sums
    ("bacc": jamp, group, amplitude, coefficient, position in the chain, last),
    each right after the bra it adds; the last one defines the group's sum"""
    out = [it for it in items if it.kind != "bsum"]
    bra_at = {proc.calls[it.data[0]].out: i for i, it in enumerate(out) if it.kind in ("bra", "vbra")}
    after = {}
    for it in items:
        if it.kind != "bsum":
            continue
        f, g, members = it.data
        chain = sorted(members, key=lambda m: (out[bra_at[m[0]]].level == it.level, bra_at[m[0]]))
        for j, (a, cc) in enumerate(chain):
            i = bra_at[a]
            anchor = i if out[i].level == it.level else -1
            after.setdefault(anchor, []).append(
                Item("bacc", it.level, (f, g, a, cc, j, j == len(chain) - 1), 0 if j == 0 else 4 * flops.CADD))
    res = list(after.get(-1, []))
    for i, it in enumerate(out):
        res.append(it)
        res.extend(after.get(i, []))
    return res


def schedule(proc):
    """What the loop nest evaluates where.

    Beyond placing each call in the innermost loop of its legs (plan):
      * a scalar input sitting in a deeper loop than the call's other inputs is
        deferred: the call runs with 1 in its place (every vertex and current
        is linear in each wavefunction input) and the scalar becomes a factor
        of the result, carried to the amplitudes;
      * an FFV amplitude whose |fi> sits deeper than <fo| and V is split into
        a bra formed in the outer loop and a spinor product (plan); a VVS or
        VVSS amplitude whose one vector sits deeper than all its other inputs
        likewise into the vector bra gc S V of the outer inputs and a
        Minkowski product with the deeper vector;
      * each jamp is sum_groups (product of the group's deferred factors) x
        (sum of the group's amplitude cores), the inner sums formed in the
        loop of their amplitudes.
    Sums (vadd / vsub) take their inputs with the factors multiplied in."""
    pl = plan(proc)
    nl = proc.n_legs
    pos = {L: i for i, L in enumerate(pl.order)}
    kind = {k: leg.kind for k, leg in enumerate(proc.legs)}
    clev = {k: pos[k] for k in range(nl)}
    fac = {k: () for k in range(nl)}          # ((slot, level), ...) deferred scalar factors
    items = [Item("ext", pos[L], (L,), _ext_flops(proc.legs[L])) for L in pl.order]
    amp_fac, amp_lev = {}, {}
    vcall = {}       # split VVS / VVSS amplitudes: the plain call, if their bra is not combined
    for k, c in enumerate(proc.calls):
        ins = list(c.ins)
        args, lv, f = [], -1, ()
        if c.op in ("vadd", "vsub"):
            for j, x in enumerate(ins):
                if fac[x]:
                    flv = max([clev[x]] + [l for _, l in fac[x]])
                    name = f"m{k}_{j}"
                    items.append(Item("mat", flv, (name, x, tuple(s for s, _ in fac[x])),
                                      len(fac[x]) * 4 * flops.CMUL))
                    args.append(("m", name))
                    lv = max(lv, flv)
                else:
                    args.append(("w", x))
                    lv = max(lv, clev[x])
        else:
            for x in ins:
                f += fac[x]
            scal = [x for x in ins if kind[x] == S]
            other = [clev[x] for x in ins if kind[x] != S]
            # an all-scalar call keeps its outermost scalar(s) as arguments
            keep_lev = max(other) if other else min(clev[x] for x in scal)
            for x in ins:
                if kind[x] == S and clev[x] > keep_lev:
                    f += ((x, clev[x]),)
                    args.append(ONE)
                else:
                    args.append(("w", x))
                    lv = max(lv, clev[x])
        if c.op in AMP_OPS:
            fi_lev = clev[ins[0]] if c.op == "iov" else None
            vdeep = None
            if c.op in ("vvs", "vvss"):
                # the deeper vector operand becomes the ket of a vector bra
                d = 0 if clev[ins[0]] > clev[ins[1]] else 1
                rest = [clev[ins[1 - d]]] + [clev[x] for x, a in zip(ins[2:], args[2:]) if a is not ONE]
                if clev[ins[d]] > max(rest):
                    vdeep = (d, max(rest))
            if c.op == "iov" and args[0] is not ONE and max(clev[ins[1]], clev[ins[2]]) < fi_lev:
                blev = max(clev[ins[1]], clev[ins[2]])
                items.append(Item("bra", blev, (k, args[1], args[2]), flops.OP_FLOPS["ffv_bra"]))
                items.append(Item("dot", fi_lev, (k, args[0]), flops.OP_FLOPS["spinor_dot"]))
                amp_lev[c.out] = fi_lev
            elif vdeep is not None:
                d, blev = vdeep
                items.append(Item("vbra", blev, (k, args[1 - d], tuple(args[2:])),
                                  flops.OP_FLOPS["vs_bra"] + flops.CMUL * (len(args) - 3)))
                items.append(Item("vdot", clev[ins[d]], (k, args[d]), flops.OP_FLOPS["vec_dot"]))
                amp_lev[c.out] = clev[ins[d]]
                vcall[c.out] = Item("call", clev[ins[d]], (k, tuple(args)), flops.call_flops(c))
            else:
                items.append(Item("call", lv, (k, tuple(args)), flops.call_flops(c)))
                amp_lev[c.out] = lv
            amp_fac[c.out] = tuple(sorted(f))
        else:
            items.append(Item("call", lv, (k, tuple(args)), flops.call_flops(c)))
            clev[c.out] = lv
            fac[c.out] = f
            kind[c.out] = OUT_KIND[c.op]
    inner = len(pl.order) - 1
    # split FFV amplitudes: bra level and ket argument, to combine bras before the product
    split = {}
    for it in items:
        if it.kind in ("bra", "vbra"):
            split[proc.calls[it.data[0]].out] = [it.level, None, it]
    for it in items:
        if it.kind in ("dot", "vdot"):
            split[proc.calls[it.data[0]].out][1] = it.data[1]
    combined = set()      # amplitudes whose every jamp term goes through a combined bra
    jamp_items = []
    for fl, terms in enumerate(proc.jamp):
        groups = {}
        for a, coef in terms:
            groups.setdefault(amp_fac[a], []).append((a, coef))
        parts = []
        for gi, (fk, members) in enumerate(sorted(groups.items())):
            kets = {split[a][1] if a in split else None for a, _ in members}
            if len(kets) == 1 and None not in kets and len(members) > 1:
                # sum_a c_a <bra_a|ket> = <sum_a c_a bra_a|ket>
                blev = max(split[a][0] for a, _ in members)
                ket = kets.pop()
                vector = split[members[0][0]][2].kind == "vbra"
                jamp_items.append(Item("bsum", blev, (fl, gi, tuple(members)), 4 * flops.CADD * (len(members) - 1)))
                jamp_items.append(Item("kdot", max(amp_lev[a] for a, _ in members), (fl, gi, ket, vector),
                                       flops.OP_FLOPS["vec_dot" if vector else "spinor_dot"]))
                combined.update(a for a, _ in members)
            else:
                klev = max(amp_lev[a] for a, _ in members)
                jamp_items.append(Item("ksum", klev, (fl, gi, tuple(members)), flops.CADD * max(len(members) - 1, 0)))
            parts.append((gi, tuple(s for s, _ in fk)))
        nmul = sum(len(fs) for _, fs in parts)
        jamp_items.append(Item("jamp", inner, (fl, tuple(parts)),
                               nmul * flops.CMUL + flops.CADD * max(len(parts) - 1, 0)))
    # the products of amplitudes used only through combined bras are not needed
    needed = {a for it in jamp_items if it.kind == "ksum" for a, _ in it.data[2]}
    items = [it for it in items
             if not (it.kind in ("dot", "vdot") and proc.calls[it.data[0]].out in combined
                     and proc.calls[it.data[0]].out not in needed)]
    # a vector bra pays only when it is summed with others: else the plain call
    out = []
    for it in items:
        a = proc.calls[it.data[0]].out if it.kind in ("vbra", "vdot") else None
        if a is not None and a not in combined:
            if it.kind == "vdot":
                out.append(vcall[a])
            continue
        out.append(it)
    items = out
    items += jamp_items
    if EARLY_BRA_SUMS:
        items = _early_bra_sums(items, proc)
    mult, m = {-1: 1}, 1
    for i, L in enumerate(pl.order):
        m *= len(pl.choices[L])
        mult[i] = m
    nf = proc.n_flows
    colour = nf * 4 + (nf * (nf - 1) // 2) * 4 + 2
    total = sum(it.flops * mult[it.level] for it in items) + colour * mult[inner]
    return Schedule(pl.order, pl.choices, items, total, proc.nest_unroll)


def unrolled_levels(sc):
    """the innermost loop levels, up to sc.unroll helicity combinations (the
    process's setting), that the kernel unrolls (constant helicities there)"""
    unrolled, combos = set(), 1
    for lvl in reversed(range(len(sc.order))):
        n = len(sc.choices[sc.order[lvl]])
        if combos * n > sc.unroll:
            break
        combos *= n
        unrolled.add(lvl)
    return unrolled


def tables(proc, sc, unrolled):
    """Calls evaluated in a real (not unrolled) helicity loop whose value does
    not vary with some loop between it and its inputs.  A call whose inputs
    are values of the loops down to level k plus external states of deeper
    legs is evaluated at level k for every combination of those legs'
    helicities (a table; k = -1 is before the loops) and picked by the loop
    counters where the nest needs it.  Tables are ranked by the flops they
    save, up to TABLE_WORDS words per lane.
    Returns {id(item): (k, legs outermost first, flops saved per event)}."""
    nl = proc.n_legs
    pos = {L: i for i, L in enumerate(sc.order)}
    real = {lvl for lvl, L in enumerate(sc.order) if len(sc.choices[L]) > 1 and lvl not in unrolled}
    mult, m = {-1: 1}, 1
    for lvl, L in enumerate(sc.order):
        m *= len(sc.choices[L])
        mult[lvl] = m
    slot_level = {L: pos[L] for L in range(nl)}
    for it in sc.items:
        if it.kind == "call" and proc.calls[it.data[0]].op not in AMP_OPS:
            slot_level[proc.calls[it.data[0]].out] = it.level
    cand = []
    for it in sc.items:
        if it.kind != "call" or it.level not in real:
            continue
        k, args = it.data
        if any(a is not ONE and a[0] != "w" for a in args):
            continue
        slots = [a[1] for a in args if a is not ONE]
        tlev = max((slot_level[x] for x in slots if x >= nl), default=-1)
        legs = sorted({x for x in slots if x < nl and pos[x] > tlev}, key=lambda L: pos[L])
        if not legs or any(pos[L] not in real or sc.choices[L] != (-1, 1) for L in legs):
            continue
        entries = 2 ** len(legs)
        saved = (mult[it.level] - mult[tlev] * entries) * it.flops
        if saved <= 0:
            continue
        words = entries * (2 if OUT_KIND[proc.calls[k].op] == S else 8)
        cand.append((saved, words, id(it), tlev, legs))
    out, used = {}, 0
    for saved, words, key, tlev, legs in sorted(cand, key=lambda c: -c[0]):
        if used + words <= TABLE_WORDS:
            out[key] = (tlev, legs, saved)
            used += words
    return out


# ------------------------------------------------- ordering templates (C2)
# amplitudes of a colour-ordered template are linear in the root position's
# vector (slot 0); the vertex vector of the other inputs is formed outside the
# root's loop: (op, index of the root input) -> device function
ROOT_SPLIT = {("vvv", 2): "vvv_r3", ("gggg", 3): "gggg_r4", ("gggg", 1): "gggg_r2"}


def template_plan(proc):
    """Loop order over the template's positions (root position 0 innermost
    when that is cheapest) and the root splits of the amplitude calls."""
    if proc.orderings is None:
        raise ValueError("not an ordering template")
    nl = proc.n_legs
    choices = []
    for k in range(nl):
        cand = {leg_choices(proc.legs[o[k]]) for o in proc.orderings}
        assert len(cand) == 1, "a position must hold one kind of particle"
        choices.append(cand.pop())
    deps = call_dependencies(proc)
    split = []
    for c in proc.calls:
        sp = None
        if c.op in AMP_OPS:
            for j, x in enumerate(c.ins):
                if x == 0 and (c.op, j) in ROOT_SPLIT:
                    sp = j
        split.append(sp)
    # the vertex vector of a split amplitude depends on the other inputs only
    odeps = []
    dep = {k: frozenset((k,)) for k in range(nl)}
    for c, d, sp in zip(proc.calls, deps, split):
        odeps.append(frozenset().union(*(dep[x] for j, x in enumerate(c.ins) if j != sp)) if sp is not None else d)
        if c.op not in AMP_OPS:
            dep[c.out] = d
    call_cost = [flops.call_flops(c) for c in proc.calls]
    ext_cost = [_ext_flops(proc.legs[proc.orderings[0][k]]) for k in range(nl)]

    def cost(order):
        pos = {L: i for i, L in enumerate(order)}
        mult, m = [], 1
        for L in order:
            m *= len(choices[L])
            mult.append(m)
        c = sum(ext_cost[L] * mult[pos[L]] for L in order)
        rl = []
        for cc, d, od, sp, call in zip(call_cost, deps, odeps, split, proc.calls):
            if sp is None:
                c += cc * mult[max(pos[L] for L in d)]
            else:
                lv = max(pos[L] for L in od)
                c += flops.OP_FLOPS[ROOT_SPLIT[(call.op, sp)]] * mult[lv]
                rl.append(lv)
        if rl:
            lv = max(rl)
            c += flops.CADD * 4 * (len(rl) - 1) * mult[lv] + flops.DOT_CC * mult[max(lv, pos[0])]
        return c

    free = [k for k in range(nl) if len(choices[k]) > 1]
    fixed = [k for k in range(nl) if len(choices[k]) == 1]
    if len(free) <= 8:
        best = min(itertools.permutations(free), key=lambda perm: cost(fixed + list(perm)))
        order = fixed + list(best)
    else:
        order = fixed + sorted(free, key=lambda k: k == 0)
    return order, choices, deps, odeps, split, cost(order)


def template_schedule(proc):
    """Items of one ordering's helicity loop nest over the template positions:
    externals, currents, the vertex vectors of the amplitudes with respect to
    the root (outside the root's loop), their jamp-weighted sum, and the
    ordering amplitude A = w_root . R innermost."""
    order, choices, deps, odeps, split, total = template_plan(proc)
    nl = proc.n_legs
    pos = {L: i for i, L in enumerate(order)}
    clev = {k: pos[k] for k in range(nl)}
    items = [Item("ext", pos[k], (k,), _ext_flops(proc.legs[proc.orderings[0][k]])) for k in order]
    coef = dict(proc.jamp[0])
    rterms = []
    for k, (c, od, sp) in enumerate(zip(proc.calls, odeps, split)):
        if c.op in AMP_OPS and sp is not None:
            lv = max(pos[L] for L in od)
            items.append(Item("rvec", lv, (k, sp), flops.OP_FLOPS[ROOT_SPLIT[(c.op, sp)]]))
            rterms.append((c.out, coef.get(c.out, 0.0), lv))
        else:
            lv = max(clev[x] for x in c.ins)
            items.append(Item("call", lv, (k, tuple(("w", x) for x in c.ins)), flops.call_flops(c)))
            if c.op not in AMP_OPS:
                clev[c.out] = lv
    amps_split = {a for a, _, _ in rterms}
    if amps_split != {a for a, _ in proc.jamp[0]} or len(amps_split) != proc.n_amps:
        raise NotImplementedError("every template amplitude must split on the root")
    rl = max(lv for _, _, lv in rterms)
    items.append(Item("rsum", rl, tuple((a, cf) for a, cf, _ in rterms), flops.CADD * 4 * (len(rterms) - 1)))
    items.append(Item("adot", max(rl, pos[0]), (), flops.DOT_CC))
    mult, m = {-1: 1}, 1
    for i, L in enumerate(order):
        m *= len(choices[L])
        mult[i] = m
    per_ordering = sum(it.flops * mult[it.level] for it in items)
    return Schedule(order, choices, items, per_ordering * len(proc.orderings))
