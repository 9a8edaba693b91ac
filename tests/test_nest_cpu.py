"""Host-side checks of the helicity loop nest (no GPU): every call is
scheduled once, every item sits no deeper than needed and no shallower than
its inputs, and the nest does fewer flops than the row-by-row loop."""
import pytest

from paper_1305_0708_amd import flops, ir, nest, processes

NAMES = ["ee_mumu", "gg_ttbar_6f", "ud_udhh_4b"]


@pytest.mark.parametrize("name", NAMES)
def test_schedule_is_complete_and_ordered(name):
    p = processes.by_name(name)
    sc = nest.schedule(p)
    assert sorted(sc.order) == list(range(p.n_legs))
    pos = {L: i for i, L in enumerate(sc.order)}
    deps = nest.call_dependencies(p)
    seen_calls, seen_amps = [], []
    level_of = {k: pos[k] for k in range(p.n_legs)}      # slot -> level its core is ready
    for it in sc.items:
        if it.kind == "call":
            k, args = it.data
            seen_calls.append(k)
            for a in args:
                if a is not nest.ONE and a[0] == "w":
                    assert level_of[a[1]] <= it.level
            # never deeper than the legs the call depends on
            assert it.level <= max(pos[L] for L in deps[k])
            c = p.calls[k]
            if c.op in ir.AMP_OPS:
                seen_amps.append(c.out)
            else:
                level_of[c.out] = it.level
        elif it.kind == "bra":
            seen_calls.append(it.data[0])
        elif it.kind == "dot":
            k, fi = it.data
            seen_amps.append(p.calls[k].out)
            assert level_of[fi[1]] <= it.level
        elif it.kind == "bsum":
            seen_amps.extend(a for a, _ in it.data[2])      # products formed with the combined bra
    assert sorted(seen_calls) == list(range(len(p.calls)))
    assert set(seen_amps) == set(range(p.n_amps))
    ks = [it for it in sc.items if it.kind in ("ksum", "bsum")]
    used = sorted(a for it in ks for a, _ in it.data[2])
    assert used == sorted(a for terms in p.jamp for a, _ in terms)
    assert {it.data[0] for it in sc.items if it.kind == "jamp"} == set(range(p.n_flows))


@pytest.mark.parametrize("name", NAMES)
def test_nest_does_less_work(name):
    p = processes.by_name(name)
    assert flops.per_event(p) < flops.per_event(p, n_hel=len(p.helicities))


def test_ordering_templates_have_no_nest():
    with pytest.raises(ValueError):
        nest.plan(processes.by_name("gg_4g"))
