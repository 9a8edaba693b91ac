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
from .ir import AMP_OPS, F, V, S, P_ZERO


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
