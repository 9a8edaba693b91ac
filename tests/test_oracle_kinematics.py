"""Pins of the oracle's random numbers, RAMBO phase space and generation cut.

These check the oracle against facts fixed outside it: Philox4x32-10 known
answers from its defining publication, the closed-form massless n-body phase
space volume (paper Eq. for dPhi_n, Sec. 2), momentum conservation and mass
shells, and the isotropy of RAMBO's single-particle distributions.
"""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(oracle):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, expect in rows:
        assert oracle.philox4x32_10(ctr, key) == expect


def test_uniform_mapping_is_open_interval(oracle):
    # the uniform built from words (w0, w1) is (floor((w0 2^32 + w1) / 2^12) + 1/2) 2^-52
    seed, ev = 0x1234567890ABCDEF, 77
    words = oracle.philox4x32_10([ev & 0xFFFFFFFF, ev >> 32, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
    u = oracle.uniforms(seed, ev, 2)
    x0 = (words[0] << 32) | words[1]
    x1 = (words[2] << 32) | words[3]
    assert u[0] == ((x0 >> 12) + 0.5) * 2.0 ** -52
    assert u[1] == ((x1 >> 12) + 0.5) * 2.0 ** -52
    # extreme words stay strictly inside (0, 1); with 53 bits the top value would
    # round to exactly 1.0
    assert (0 + 0.5) * 2.0 ** -52 > 0.0
    assert ((2 ** 52 - 1) + 0.5) * 2.0 ** -52 < 1.0
    assert ((2 ** 53 - 1) + 0.5) * 2.0 ** -53 == 1.0
    many = np.concatenate([oracle.uniforms(3, i, 24) for i in range(2000)])
    assert many.min() > 0.0 and many.max() < 1.0
    assert abs(many.mean() - 0.5) < 0.01


@pytest.mark.parametrize("n,rs,expect", [
    (2, 200.0, 1.0 / (8.0 * math.pi)),
    # (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!) evaluated by hand
    (4, 1000.0, (2 * math.pi) ** -8 * (math.pi / 2) ** 3 * 1e12 / (6 * 2)),
    (6, 1000.0, (2 * math.pi) ** -14 * (math.pi / 2) ** 5 * 1e24 / (120 * 24)),
    (6, 2000.0, (2 * math.pi) ** -14 * (math.pi / 2) ** 5 * 4.0 ** 4 * 1e24 / (120 * 24)),
])
def test_phase_space_volume(oracle, n, rs, expect):
    assert oracle.phase_space_volume(rs, n) == pytest.approx(expect, rel=1e-14)


def test_phase_space_volume_printed_values(oracle):
    # magnitudes quoted for the benchmark workloads
    assert oracle.phase_space_volume(200.0, 2) == pytest.approx(3.978874e-2, rel=1e-6)
    assert oracle.phase_space_volume(1000.0, 4) == pytest.approx(1.329656e5, rel=1e-6)
    assert oracle.phase_space_volume(1000.0, 6) == pytest.approx(2.221717e10, rel=1e-6)
    assert oracle.phase_space_volume(2000.0, 6) == pytest.approx(5.687596e12, rel=1e-6)


def test_phase_space_two_body_integral(oracle):
    # Phi_2 = integral of |p| / (16 pi^2 sqrt s) dOmega = 1 / (8 pi) for massless particles
    assert 4 * math.pi * (100.0 / (16 * math.pi ** 2 * 200.0)) == pytest.approx(1 / (8 * math.pi), rel=1e-14)


@pytest.mark.parametrize("n_out,rs", [(2, 200.0), (4, 1000.0), (6, 1000.0), (6, 2000.0)])
def test_rambo_conservation_and_shells(oracle, n_out, rs):
    # for n = 2 the conformal boost is large when the two seed vectors are nearly
    # collinear (gamma = Q0 / M), which amplifies rounding: allow 1e-10 there
    tol = 1e-10 if n_out == 2 else 1e-13
    mom = oracle.generate(0x48454746, 500, n_out, rs)
    tot = mom[:, 2:, :].sum(axis=1)
    assert np.allclose(tot[:, 0], rs, rtol=0, atol=tol * rs)
    assert np.abs(tot[:, 1:]).max() < tol * rs
    m2 = mom[:, :, 0] ** 2 - (mom[:, :, 1:] ** 2).sum(axis=2)
    assert np.abs(m2).max() < tol * rs * rs
    assert (mom[:, 2:, 0] > 0).all()


def test_rambo_weight_is_constant_volume(oracle):
    u = oracle.uniforms(5, 9, 24)
    p, w = oracle.rambo(1000.0, u)
    assert w == oracle.phase_space_volume(1000.0, 6)


def test_rambo_isotropy(oracle):
    # single-particle cos(theta) and phi are uniform (Kolmogorov-Smirnov)
    from scipy import stats
    mom = oracle.generate(99, 4000, 4, 1000.0)
    p = mom[:, 2, :]
    c = p[:, 3] / np.linalg.norm(p[:, 1:], axis=1)
    ph = np.arctan2(p[:, 2], p[:, 1])
    assert stats.kstest(c, "uniform", args=(-1, 2)).pvalue > 1e-3
    assert stats.kstest(ph, "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-3


def test_rambo_matches_flat_two_body(oracle):
    # for n = 2 RAMBO is back-to-back with |p| = sqrt(s)/2
    mom = oracle.generate(1, 50, 2, 200.0)
    assert np.allclose(mom[:, 2, 0], 100.0, rtol=1e-14)
    assert np.allclose(mom[:, 2, 1:], -mom[:, 3, 1:], atol=1e-12)


def test_gluon_cut_hand_cases(oracle):
    def ev(pts, etas, phis):
        m = np.zeros((6, 4))
        m[0] = [500, 0, 0, 500]
        m[1] = [500, 0, 0, -500]
        for k, (pt, eta, phi) in enumerate(zip(pts, etas, phis)):
            m[2 + k] = [pt * math.cosh(eta), pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta)]
        return m
    good = ev([100, 100, 100, 100], [0, 0, 1, -1], [0, 2, 0, 4])
    low_pt = ev([100, 19.9, 100, 100], [0, 0, 1, -1], [0, 2, 0, 4])
    close = ev([100, 100, 100, 100], [0, 0.3, 1, -1], [0, 0.2, 0, 4])     # dR = 0.36
    wrap = ev([100, 100, 100, 100], [0, 0, 1, -1], [3.1, -3.1, 1.0, 4.5])  # dphi wraps to 0.083
    far = ev([100, 100, 100, 100], [0, 0.3, 1, -1], [0, 0.3, 0, 4])      # dR = 0.424
    res = oracle.cut_gluons(np.stack([good, low_pt, close, wrap, far]))
    assert list(res) == [1, 0, 0, 0, 1]


@pytest.mark.parametrize("n_out", [3, 4, 6])
def test_rambo_energy_fraction_is_beta_2_n_minus_2(oracle, n_out):
    """The flat massless n-body density (Sec. 2, Eq. of dPhi_n) fixes the energy
    of any one particle: dPhi_n = d^3p/(2E) Phi_{n-1}((P - p)^2) with
    Phi_{n-1}(s') proportional to s'^(n-3) and s' = s (1 - x), x = 2E/sqrt(s), so
    x follows x (1 - x)^(n-3), the Beta(2, n - 2) law.  Conservation, mass
    shells, isotropy and a constant weight hold for any energy law; this does
    not (an exponential instead of a Gamma(2) seed energy fails it by far)."""
    from scipy import stats
    N = 20000
    mom = oracle.generate(0x52414D42, N, n_out, 1000.0)
    idx = 2 + np.arange(N) % n_out        # one particle per event: independent samples
    x = 2.0 * mom[np.arange(N), idx, 0] / 1000.0
    assert stats.kstest(x, stats.beta(2, n_out - 2).cdf).pvalue > 1e-3
    # second moment 6 / (n (n + 1)) within five standard errors
    m2 = 6.0 / (n_out * (n_out + 1))
    assert abs(np.mean(x * x) - m2) < 5 * np.std(x * x) / math.sqrt(N)


def test_rambo_three_body_dalitz_moments(oracle):
    """Three massless bodies: the Dalitz plot is flat, so (s12, s13, s23)/s is
    uniform on the simplex (a Dirichlet(1, 1, 1) law): <s12> = s/3,
    <s12^2> = s^2/6, <s12 s23> = s^2/12."""
    N = 200000
    mom = oracle.generate(0x44414C49, N, 3, 1000.0)
    p = mom[:, 2:, :]

    def inv(a, b):
        q = p[:, a] + p[:, b]
        return (q[:, 0] ** 2 - (q[:, 1:] ** 2).sum(axis=1)) / 1e6
    y12, y23 = inv(0, 1), inv(1, 2)
    for v, expect in ((y12, 1 / 3), (y12 * y12, 1 / 6), (y12 * y23, 1 / 12)):
        assert abs(v.mean() - expect) < 5 * v.std() / math.sqrt(N)


def test_rambo_matches_the_flat_tree(oracle):
    """For 4 and 6 bodies the pair mass s12 / s and the single energy E / sqrt(s)
    of RAMBO events (constant weight) have the means of the flat resonance tree,
    whose weights carry the density event by event (the tree's volume is pinned
    to the closed form in test_oracle_phase_space_tree)."""
    from oracle import phase_space_tree as T
    for n_out in (4, 6):
        N = 40000
        mom = oracle.generate(0x464C4154 + n_out, N, n_out, 1000.0)
        nodes = [(0.0, 0.0, None, 2, -2, None)] + \
            [(0.0, 0.0, "flat", 2 + k, -(k + 2), None) for k in range(1, n_out - 1)]
        nodes[-1] = (0.0, 0.0, "flat", n_out, n_out + 1, None)
        tmom, w = T.generate(0x54524545 + n_out, N, 1000.0, nodes, n_out + 2)

        def obs(m):
            q = m[:, 2] + m[:, 3]
            return np.stack([(q[:, 0] ** 2 - (q[:, 1:] ** 2).sum(axis=1)) / 1e6, m[:, 2, 0] / 1000.0,
                             m[:, 5, 0] / 1000.0], axis=1)
        a, b = obs(mom), obs(tmom)
        for k in range(a.shape[1]):
            ma, sa = a[:, k].mean(), a[:, k].std() / math.sqrt(N)
            mb = np.sum(w * b[:, k]) / np.sum(w)
            sb = math.sqrt(np.sum((w * (b[:, k] - mb)) ** 2)) / np.sum(w)
            assert abs(ma - mb) < 5 * math.hypot(sa, sb), (n_out, k, ma, mb)
