"""Pins of the oracle's u ubar -> t tbar + n gluons (oracle/quark_lines.cpp):
every tree diagram with explicit Dirac matrices and SU(3) colour sums.

* n = 0 through the same diagram code equals the textbook q qbar -> Q Qbar
  spin- and colour-summed |M|^2 (normalisation of the quark-gluon vertex, the
  colour sum Tr(T^a T^b) Tr(T^a T^b) = 2, the external spinors).
* Ward identity: with one gluon's polarisation replaced by its momentum the
  sum over diagrams vanishes, for every gluon and n = 1, 2, 3 (zero top width:
  a fixed-width propagator breaks it at O(Gamma / m)).  It ties the normalisation
  and sign of the triple- and four-gluon vertices and their colour structures to
  the quark-gluon vertex, and it fails when a diagram is missing.  Planted in a
  copy of the oracle, each of these mistakes leaves ratios of 1e-4 or more:
  the sign of the triple-gluon vertex flipped, one colour structure of the
  four-gluon vertex dropped or given another's colour factor, the momenta of
  the triple-gluon vertex swapped, the gluon propagator's 1/k^2 replaced by
  1/(2 k^2).
* Lorentz invariance (momentum routing of the propagators) and Bose symmetry
  under permutations of the gluons (the diagram set and the colour sum).
"""
import itertools
import math

import numpy as np
import pytest

import fp64_bounds as B

GS2 = 4 * math.pi * 0.118
MT = 175.0
IDS = {1: "UU_TTG", 2: "UU_TTGG", 3: "UU_TTGGG"}


def events(oracle, ng, n, seed):
    from oracle import phase_space_tree as T
    mom, w = T.generate(seed, n, 1000.0, B._tt_gluons_tree(ng), 4 + ng, leg_mass=[0, 0, MT, MT] + [0] * ng)
    return mom[w > 0]


def boost(mom, b):
    b = np.asarray(b, dtype=float)
    bb = b @ b
    g = 1.0 / math.sqrt(1.0 - bb)
    flat = mom.reshape(-1, 4)
    out = flat.copy()
    E, bp = flat[:, 0], flat[:, 1:] @ b
    out[:, 0] = g * (E + bp)
    out[:, 1:] = flat[:, 1:] + (((g - 1.0) * bp / bb + g * E)[:, None]) * b[None, :]
    return out.reshape(mom.shape)


def test_no_gluon_is_the_textbook_formula(oracle):
    # (1/36) sum |M|^2 = (4/9) g^4 (tau1^2 + tau2^2 + rho/2), tau_i = 2 p_i.p_3 / s, rho = 4 m^2 / s
    rng = np.random.default_rng(17)
    for _ in range(4):
        c, phi = rng.uniform(-1, 1), rng.uniform(0, 2 * math.pi)
        E = 400.0
        p = math.sqrt(E * E - MT * MT)
        st = math.sqrt(1 - c * c)
        m = np.array([[[E, 0, 0, E], [E, 0, 0, -E], [E, p * st * math.cos(phi), p * st * math.sin(phi), p * c],
                       [E, -p * st * math.cos(phi), -p * st * math.sin(phi), -p * c]]])
        s = (2 * E) ** 2
        dot = lambda a, b: a[0] * b[0] - a[1:] @ b[1:]
        t1, t2, rho = 2 * dot(m[0, 0], m[0, 2]) / s, 2 * dot(m[0, 1], m[0, 2]) / s, 4 * MT * MT / s
        cf = 36 * (4 / 9) * GS2 ** 2 * (t1 ** 2 + t2 ** 2 + rho / 2)
        assert oracle.me2(oracle.UU_TT_DIAG, m)[0] / cf - 1 == pytest.approx(0, abs=1e-13)


def test_diagram_counts(oracle):
    """1, 5, 38, 393 tree diagrams (the four-gluon vertex once per colour
    structure); 5 for one gluon is the textbook count"""
    assert [oracle.uu_tt_gluons_diagrams(n) for n in range(4)] == [1, 5, 38, 393]


@pytest.mark.parametrize("ng", [1, 2, 3])
def test_ward_identity(oracle, ng):
    mom = events(oracle, ng, 6 if ng == 3 else 12, 0x57415244 + ng)
    pid = getattr(oracle, IDS[ng])
    f = oracle.me2(pid, mom, oracle.params(wt=0.0))
    assert np.all(f > 0)
    for g in range(4, 4 + ng):
        fw = oracle.me2(pid, mom, oracle.params(wt=0.0, gauge_leg=g))
        assert np.max(np.abs(fw / f)) < 1e-12, (g, np.max(np.abs(fw / f)))


def test_lorentz_invariance(oracle):
    """at zero top width: with a fixed width the sum over the gluons' physical
    polarisations (transverse in the event's frame) depends on the frame at the
    level of the gauge violation, 1e-5 here"""
    prm = oracle.params(wt=0.0)
    mom = events(oracle, 3, 4, 0x4C4F5245)
    f = oracle.me2(oracle.UU_TTGGG, mom, prm)
    for b in ([0.3, 0.2, -0.5], [0.0, 0.0, 0.9]):
        assert np.max(np.abs(oracle.me2(oracle.UU_TTGGG, boost(mom, b), prm) / f - 1)) < 1e-11


@pytest.mark.parametrize("ng", [2, 3])
def test_bose_symmetry(oracle, ng):
    mom = events(oracle, ng, 4, 0x424F5345 + ng)
    pid = getattr(oracle, IDS[ng])
    f = oracle.me2(pid, mom)
    for perm in itertools.permutations(range(4, 4 + ng)):
        moved = mom.copy()
        moved[:, 4:] = mom[:, list(perm)]
        assert np.max(np.abs(oracle.me2(pid, moved) / f - 1)) < 1e-12
