"""Pins of the oracle's resonance phase space (the paper's Appendix A at a fixed
collision energy) against what the mathematics fixes: momentum conservation
and mass shells, the closed-form n-body volume that every parametrisation of
the same phase space must reproduce, the Breit-Wigner Jacobian per event, and
two mappings of the same windowed region agreeing."""
import math

import numpy as np
import pytest

MT, WT, MW, WW = 175.0, 1.55, 80.4, 2.085
ROOTS = 1000.0


def c1_tree(mapping="bw", window=20.0):
    """g g -> t t~, t -> b W+ (-> e+ nu), t~ -> b~ W- (-> mu- nu~); legs as in the C1 process"""
    return [(0.0, 0.0, None, -2, -3, None),
            (MT, WT, mapping, 2, -4, window),
            (MT, WT, mapping, 5, -5, window),
            (MW, WW, mapping, 3, 4, window),
            (MW, WW, mapping, 6, 7, window)]


def flat_tree_c1():
    return [(0.0, 0.0, None, -2, -3, None),
            (0.0, 0.0, "flat", 2, -4, None),
            (0.0, 0.0, "flat", 5, -5, None),
            (0.0, 0.0, "flat", 3, 4, None),
            (0.0, 0.0, "flat", 6, 7, None)]


def msq(p):
    return p[..., 0] ** 2 - (p[..., 1:] ** 2).sum(-1)


@pytest.fixture(scope="module")
def T(oracle):
    from oracle import phase_space_tree
    return phase_space_tree


def test_uniform_count(T):
    assert T.n_uniforms(c1_tree()) == 14


def test_conservation_shells_and_windows(T):
    mom, w = T.generate(7, 20000, ROOTS, c1_tree(), 8)
    assert np.abs(mom[:, 2:].sum(1) - [ROOTS, 0, 0, 0]).max() < 1e-11 * ROOTS
    assert np.abs(msq(mom[:, 2:])).max() < 1e-12 * ROOTS ** 2
    assert np.all(w > 0)
    for legs, m, g in (((2, 3, 4), MT, WT), ((5, 6, 7), MT, WT), ((3, 4), MW, WW), ((6, 7), MW, WW)):
        s = msq(mom[:, list(legs)].sum(1))
        assert np.all(np.abs(s - m * m) <= 20.0 * m * g * (1 + 1e-12))


def test_two_body_weight_is_exact(T):
    """one decay of the collision into two massless particles: dPhi_2 = 1/(8 pi) per event"""
    mom, w = T.generate(3, 1000, ROOTS, [(0.0, 0.0, None, 2, 3, None)], 4)
    assert np.allclose(w, 1.0 / (8.0 * math.pi), rtol=1e-15, atol=0)
    assert np.abs(mom[:, 2, 1:] + mom[:, 3, 1:]).max() < 1e-12 * ROOTS


@pytest.mark.parametrize("tree,n", [
    ([(0.0, 0.0, None, 2, -2, None), (0.0, 0.0, "flat", 3, 4, None)], 3),
    ([(0.0, 0.0, None, -2, -3, None), (0.0, 0.0, "flat", 2, 3, None), (0.0, 0.0, "flat", 4, 5, None)], 4),
    ([(0.0, 0.0, None, 2, -2, None), (0.0, 0.0, "flat", 3, -3, None), (0.0, 0.0, "flat", 4, 5, None)], 4),
    (flat_tree_c1(), 6),
])
def test_flat_tree_reproduces_the_n_body_volume(oracle, T, tree, n):
    """any factorisation of the massless n-body phase space has the volume
    (2 pi)^(4 - 3n) (pi / 2)^(n - 1) s^(n - 2) / ((n - 1)! (n - 2)!)"""
    N = 300000
    _, w = T.generate(0x5EED + n, N, ROOTS, tree, n + 2)
    mean, err = w.mean(), w.std() / math.sqrt(N)
    ref = oracle.phase_space_volume(ROOTS, n)
    assert abs(mean - ref) < 4.0 * err, (mean, err, ref)
    assert err < 0.02 * ref


def test_breit_wigner_jacobian_per_event(T):
    """root -> (2, R), R -> (3, 4) with the Breit-Wigner mapping: per event
    w * 2 pi / (dPhi_2(root) dPhi_2(R)) / [(s - m^2)^2 + (m Gamma)^2] = (t_hi - t_lo) / (m Gamma)"""
    m, g, win = MW, WW, 20.0
    tree = [(0.0, 0.0, None, 2, -2, None), (m, g, "bw", 3, 4, win)]
    mom, w = T.generate(5, 5000, ROOTS, tree, 5)
    s = msq(mom[:, 3] + mom[:, 4])
    S = ROOTS ** 2
    dphi_root = (S - s) / (8.0 * math.pi * S)          # lambda^(1/2)(S, 0, s) / (8 pi S)
    dphi_r = 1.0 / (8.0 * math.pi)
    lo, hi = max(0.0, m * m - win * m * g), min(S, m * m + win * m * g)
    span = (math.atan((hi - m * m) / (m * g)) - math.atan((lo - m * m) / (m * g))) / (m * g)
    got = w * 2.0 * math.pi / (dphi_root * dphi_r) / ((s - m * m) ** 2 + (m * g) ** 2)
    assert np.allclose(got, span, rtol=1e-9, atol=0)


def test_mappings_of_one_window_agree(T):
    """the Breit-Wigner and the flat mapping of the same windowed region
    estimate the same volume"""
    N = 200000
    _, wb = T.generate(21, N, ROOTS, c1_tree("bw"), 8)
    _, wf = T.generate(22, N, ROOTS, c1_tree("flat"), 8)
    eb, ef = wb.std() / math.sqrt(N), wf.std() / math.sqrt(N)
    assert abs(wb.mean() - wf.mean()) < 4.0 * math.hypot(eb, ef), (wb.mean(), eb, wf.mean(), ef)


MH = 125.0


def lam(a, b, c):
    return a * a + b * b + c * c - 2 * a * b - 2 * a * c - 2 * b * c


def test_massive_two_body_weight_is_exact(T):
    """collision into two massive particles: dPhi_2 = lambda^(1/2)(s, m1^2, m2^2) / (8 pi s)"""
    m1, m2 = 125.0, 91.1876
    mom, w = T.generate(4, 500, ROOTS, [(0.0, 0.0, None, 2, 3, None)], 4, leg_mass=[0, 0, m1, m2])
    s = ROOTS ** 2
    assert np.allclose(w, math.sqrt(lam(s, m1 * m1, m2 * m2)) / (8 * math.pi * s), rtol=1e-14, atol=0)
    assert np.abs(msq(mom[:, 2]) - m1 * m1).max() < 1e-12 * s
    assert np.abs(msq(mom[:, 3]) - m2 * m2).max() < 1e-12 * s


HHH_MASSES = [0, 0, 0, 0, MH, MH, MH]


def test_massive_legs_conservation_and_shells(T):
    tree = [(0.0, 0.0, None, 2, -2, None), (0.0, 0.0, "flat", 3, -3, None),
            (0.0, 0.0, "flat", 4, -4, None), (0.0, 0.0, "flat", 5, 6, None)]
    mom, w = T.generate(8, 5000, ROOTS, tree, 7, leg_mass=HHH_MASSES)
    assert np.all(w > 0)
    assert np.abs(mom[:, 2:].sum(1) - [ROOTS, 0, 0, 0]).max() < 1e-11 * ROOTS
    m2 = np.array(HHH_MASSES[2:]) ** 2
    assert np.abs(msq(mom[:, 2:]) - m2).max() < 1e-10 * ROOTS ** 2


def test_massive_volume_does_not_depend_on_the_tree(T):
    """the volume of the u d H H H final state (two massless, three of 125 GeV)
    from two different factorisations agrees within the Monte Carlo errors (a
    wrong two-body weight or daughter energy with masses changes one of them;
    a range too wide leaves events of zero weight, which the conservation test
    rejects)"""
    trees = ([(0.0, 0.0, None, 2, -2, None), (0.0, 0.0, "flat", 3, -3, None),
              (0.0, 0.0, "flat", 4, -4, None), (0.0, 0.0, "flat", 5, 6, None)],
             [(0.0, 0.0, None, -2, -3, None), (0.0, 0.0, "flat", 2, 3, None),
              (0.0, 0.0, "flat", 4, -4, None), (0.0, 0.0, "flat", 5, 6, None)])
    est = []
    for k, tree in enumerate(trees):
        _, w = T.generate(11 + k, 200000, 700.0, tree, 7, leg_mass=HHH_MASSES)
        est.append((w.mean(), w.std() / math.sqrt(w.size)))
    (a, ea), (b, eb) = est
    assert abs(a - b) < 4 * math.hypot(ea, eb)
    assert ea < 0.01 * a and eb < 0.01 * b


# ------------------------------------------------------------ hadronic collision (Appendix A, densities 1)
def test_hadronic_two_body_volume_matches_quadrature(T):
    """t tbar at a 2 TeV hadron collider with the rapidity range covering every
    kinematically allowed top (|y| <= ln(sqrt_S / m_t) < 2.5): the Monte Carlo
    mean of dSigma_2 g(s_hat) (the weight times 2 s_hat) equals the integral
    over dx_a dx_b of Phi_2(s_hat; m_t, m_t) g(s_hat), here with g = S / s_hat,
    by two-dimensional quadrature in x_a, x_b"""
    from scipy import integrate
    m, rs = 175.0, 2000.0
    S = rs * rs
    mom, w = T.generate(5, 400000, rs, [(0.0, 0.0, None, 2, 3, None)], 4, leg_mass=[0, 0, m, m],
                        hadronic=(2.5, 0.0))
    P = mom[:, 0] + mom[:, 1]
    sh = P[:, 0] ** 2 - (P[:, 1:] ** 2).sum(1)
    val = w * 2.0 * sh * (S / sh)
    est, err = val.mean(), val.std() / math.sqrt(val.size)

    def phi2_g(xb, xa):
        s = xa * xb * S
        return math.sqrt(max((s - 4 * m * m) * s, 0.0)) / (8 * math.pi * s) * (S / s) if s > 4 * m * m else 0.0
    ref, _ = integrate.dblquad(phi2_g, 4 * m * m / S, 1.0, lambda xa: 4 * m * m / (S * xa), 1.0,
                               epsabs=1e-12, epsrel=1e-9)
    assert abs(est - ref) < 4 * err
    assert err < 0.01 * ref


def test_hadronic_tree_conservation_and_beams(T):
    """C1 from a gluon-gluon collision at 14 TeV: the incoming partons along +-z
    with x_a, x_b < 1 carry the final state's four-momentum; the tops sit in
    |y| < 2.5; an event outside x < 1 has weight 0"""
    tree = [(0.0, 0.0, None, -2, -3, None), (MT, WT, "bw", 2, -4, 20.0), (MT, WT, "bw", 5, -5, 20.0),
            (MW, WW, "bw", 3, 4, 20.0), (MW, WW, "bw", 6, 7, 20.0)]
    rs = 14000.0
    assert T.n_uniforms(tree, (2.5, 0.0)) == 16
    mom, w = T.generate(9, 20000, rs, tree, 8, hadronic=(2.5, 0.0))
    ok = w > 0
    assert 0.1 < ok.mean() < 1.0
    xa, xb = 2 * mom[:, 0, 0] / rs, 2 * mom[:, 1, 0] / rs
    assert np.all(xa[ok] < 1) and np.all(xb[ok] < 1) and np.all((xa >= 1) | (xb >= 1) | ok)
    assert np.abs(mom[:, 0, 1:3]).max() == 0 and np.abs(mom[:, 1, 1:3]).max() == 0
    bal = mom[:, 0] + mom[:, 1] - mom[:, 2:].sum(1)
    assert np.abs(bal[ok]).max() < 1e-10 * rs
    assert np.abs(msq(mom[ok][:, 2:])).max() < 1e-10 * rs ** 2
    top = mom[:, 2:5].sum(1)
    y = 0.5 * np.log((top[:, 0] + top[:, 3]) / (top[:, 0] - top[:, 3]))
    assert np.abs(y).max() < 2.5 + 1e-9
