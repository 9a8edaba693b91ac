"""The n-gluon IR's colour algebra (product side, exact Fierz and
Kleiss-Kuijf) against the oracle's brute-force SU(3) colour matrix and its
independent Berends-Giele partial amplitudes."""
import itertools

import numpy as np
import pytest


@pytest.mark.parametrize("n", [4, 5, 6])
def test_trace_colour_matrix_matches_oracle(oracle, n):
    from paper_1305_0708_amd.processes import gluons
    C = np.array([[float(x) for x in row] for row in gluons.colour_matrix(n)])
    assert np.allclose(C, oracle.gluon_colour_matrix(n), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [5, 6])
def test_kleiss_kuijf_reproduces_all_orderings(oracle, n):
    from paper_1305_0708_amd.processes import gluons
    K = np.array(gluons.kk_matrix(n), dtype=float)
    orders = gluons.trace_orderings(n)
    ddm = gluons.ddm_orderings(n)
    mom = oracle.generate(31, 1, n - 2, 1000.0)[0]
    # helicities with at least two of each sign after crossing the incoming legs
    # (amplitudes with at most one helicity of either sign vanish identically)
    hels = {5: [(1, -1, 1, -1, 1), (-1, 1, -1, 1, 1), (1, -1, -1, 1, 1)],
            6: [(1, -1, 1, -1, 1, -1), (-1, 1, 1, -1, -1, 1), (1, 1, 1, 1, -1, -1)]}[n]
    errs, scale = [], 0.0
    for hel in hels:
        A = np.array([oracle.gluon_partial(mom, hel, o) for o in orders])
        D = np.array([oracle.gluon_partial(mom, hel, o) for o in ddm])
        errs.append(np.max(np.abs(K @ D - A)))
        scale = max(scale, np.max(np.abs(A)))
    # rounding is relative to the event's amplitude scale: a helicity whose
    # partial amplitudes are small because two legs are nearly collinear
    # carries the absolute error of the larger terms it is built from
    assert max(errs) < 1e-13 * scale


def test_ddm_colour_form_equals_trace_form(oracle):
    from paper_1305_0708_amd.processes import gluons
    n = 6
    C = np.array([[float(x) for x in row] for row in gluons.colour_matrix(n)])
    CD = np.array([[float(x) for x in row] for row in gluons.ddm_colour_matrix(n)])
    K = np.array(gluons.kk_matrix(n), dtype=float)
    assert np.allclose(K.T @ C @ K, CD, atol=1e-9)
    mom = oracle.generate(32, 1, n - 2, 1000.0)[0]
    hel = (-1, 1, -1, 1, 1, -1)
    D = np.array([oracle.gluon_partial(mom, hel, o) for o in gluons.ddm_orderings(n)])
    A = K @ D
    assert np.real(np.conj(D) @ CD @ D) == pytest.approx(np.real(np.conj(A) @ C @ A), rel=1e-12)


def test_gluon_ir_shape():
    from paper_1305_0708_amd.processes import gluons
    for basis, nf in (("trace", 120), ("ddm", 24)):
        p = gluons.gg_ng(6, basis=basis)
        assert p.n_flows == nf and len(p.orderings) == 24 and len(p.colour) == nf
        assert all(o[0] == 0 and o[-1] == 5 for o in p.orderings)
        assert p.symmetry == 24 and p.n_a_n_b == 64 and p.cut_enabled
        assert p.uses_colour_mfma() == (basis == "trace")
    # trace basis: flow f is the Kleiss-Kuijf row of ordering f, with 1, 4, 6, 4, 1 terms as the
    # last gluon sits at the end, one, two, three or four places before it
    p = gluons.gg_ng(6)
    counts = sorted(sum(1 for x in r if x) for r in p.flow_map)
    assert counts == sorted([1] * 24 + [4] * 24 + [6] * 24 + [4] * 24 + [1] * 24)
    ddm = {o: k for k, o in enumerate(p.orderings)}
    for f, t in enumerate(gluons.trace_orderings(6)):
        if t[-1] == 5:
            assert p.flow_map[f] == [1 if k == ddm[t] else 0 for k in range(24)]
