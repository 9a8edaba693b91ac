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
        elif it.kind == "bacc":
            seen_amps.append(it.data[2])                     # the same, one bra at a time
    assert sorted(seen_calls) == list(range(len(p.calls)))
    assert set(seen_amps) == set(range(p.n_amps))
    ks = [it for it in sc.items if it.kind in ("ksum", "bsum")]
    used = sorted([a for it in ks for a, _ in it.data[2]] + [it.data[2] for it in sc.items if it.kind == "bacc"])
    assert used == sorted(a for terms in p.jamp for a, _ in terms)
    assert {it.data[0] for it in sc.items if it.kind == "jamp"} == set(range(p.n_flows))


@pytest.mark.parametrize("name", NAMES)
def test_nest_does_less_work(name):
    p = processes.by_name(name)
    assert flops.per_event(p) < flops.per_event(p, n_hel=len(p.helicities))


def test_ordering_templates_have_no_nest():
    with pytest.raises(ValueError):
        nest.plan(processes.by_name("gg_4g"))


@pytest.mark.parametrize("name", NAMES)
def test_tables_are_valid(name):
    """A tabulated call: every input is an external state of a tabulated leg
    (deeper than the table's level, in a real two-state loop) or a value ready
    at the table's level; the call's own loop varies with something the table
    does not, so the table saves evaluations; the budget holds."""
    p = processes.by_name(name)
    sc = nest.schedule(p)
    un = nest.unrolled_levels(sc)
    pos = {L: i for i, L in enumerate(sc.order)}
    ready = {k: pos[k] for k in range(p.n_legs)}
    for it in sc.items:
        if it.kind == "call" and p.calls[it.data[0]].op not in ir.AMP_OPS:
            ready[p.calls[it.data[0]].out] = it.level
    items = {id(it): it for it in sc.items}
    words = 0
    for key, (tlev, legs, saved) in nest.tables(p, sc, un).items():
        it = items[key]
        assert it.kind == "call" and saved > 0
        assert tlev < it.level and it.level not in un
        for L in legs:
            assert tlev < pos[L] <= it.level and pos[L] not in un and sc.choices[L] == (-1, 1)
        for a in it.data[1]:
            if a is nest.ONE:
                continue
            assert a[1] in legs or ready[a[1]] <= tlev
        words += 2 ** len(legs) * 8
    assert words <= nest.TABLE_WORDS


def test_c1_tables_and_stash_in_the_generated_kernel():
    """C1 with its whole nest unrolled (its own setting, compiled for two
    waves per SIMD) needs no tables and no stash: every helicity is a constant
    of the unrolled code.  With five loops unrolled there are no tables either;
    with only the three fermion loops unrolled, the gg -> g* current is
    tabulated before the loops over both gluon helicities and the top current
    over gluon 1 inside the b-quark loop; the stash fits its budget and the
    flop model counts the tables."""
    import dataclasses
    from paper_1305_0708_amd import codegen
    c1 = processes.by_name("gg_ttbar_6f")
    sc1 = nest.schedule(c1)
    assert len(nest.unrolled_levels(sc1)) == 8
    src1 = codegen.Gen(c1).emit()
    assert "t12_" not in src1 and "stash_put(" not in src1
    # two waves per SIMD for the FP64 kernel, three for the FP32 one
    assert "__launch_bounds__(256, sizeof(T) == 8 ? 2 : 3) void amp_gg_ttbar_6f" in src1
    bw = codegen.Gen(processes.by_name("gg_ttbar_6f_bw")).emit()
    assert "__launch_bounds__(256) void amp_gg_ttbar_6f_bw" in bw
    c5 = dataclasses.replace(c1, nest_unroll=32)
    sc5 = nest.schedule(c5)
    assert len(nest.unrolled_levels(sc5)) == 5
    assert nest.tables(c5, sc5, nest.unrolled_levels(sc5)) == {}
    assert "t12_" not in codegen.Gen(c5).emit()
    p = dataclasses.replace(c1, nest_unroll=8)
    src = codegen.Gen(p).emit()
    assert "jvvxxx<T, false>(x0m, Qs0, x1m, Qs1" in src
    assert "(c0 ? (c1 ? t12_3 : t12_2) : (c1 ? t12_1 : t12_0))" in src
    assert "(c1 ? t14_1 : t14_0)" in src
    import re
    m = re.search(r"__shared__ T stash\[(\d+)\]\[256\]", src)
    assert m and int(m.group(1)) <= codegen.STASH_WORDS
    assert src.count("stash_get<") == src.count("stash_put(")
    sc = nest.schedule(p)
    assert flops.per_event(p) < sc.flops_per_event
