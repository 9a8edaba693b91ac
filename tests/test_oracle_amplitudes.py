"""Pins of the oracle's squared matrix elements against physics that fixes them
independently of the oracle: closed forms, Ward identities, Lorentz
invariance, spin sums by Dirac traces, Parke-Taylor magnitudes, exact zeros,
Bose/Fermi symmetry and tree-level unitarity.
"""
import itertools
import math

import numpy as np
import pytest

GS2 = 4 * math.pi * 0.118


def boost(mom, b):
    b = np.asarray(b, dtype=float)
    bb = b @ b
    g = 1.0 / math.sqrt(1.0 - bb)
    flat = mom.reshape(-1, 4)
    out = flat.copy()
    E = flat[:, 0]
    bp = flat[:, 1:] @ b
    out[:, 0] = g * (E + bp)
    out[:, 1:] = flat[:, 1:] + (((g - 1.0) * bp / bb + g * E)[:, None]) * b[None, :]
    return out.reshape(mom.shape)


def rotate(mom, axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    R = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    out = mom.copy()
    out[..., 1:] = mom[..., 1:] @ R.T
    return out


def two_to_two_massive(rs, m, c, phi):
    E = rs / 2
    p = math.sqrt(E * E - m * m)
    s = math.sqrt(1 - c * c)
    return np.array([[E, 0, 0, E], [E, 0, 0, -E],
                     [E, p * s * math.cos(phi), p * s * math.sin(phi), p * c],
                     [E, -p * s * math.cos(phi), -p * s * math.sin(phi), -p * c]])


# ------------------------------------------------------------------ C0 closed form
def ee_closed_form(p, prm_alpha=1 / 128, sw2=0.2222, mz=91.1876, wz=2.4952):
    """sum_spins |M|^2 for e+e- -> mu+mu- via gamma and Z from helicity amplitudes:
    s^2 [(|A_LL|^2 + |A_RR|^2)(1+c)^2 + (|A_LR|^2 + |A_RL|^2)(1-c)^2],
    A_ij = sum_V g_i^e g_j^mu / (s - M_V^2 + i M_V Gamma_V), c = cos angle(e-, mu-)."""
    e = math.sqrt(4 * math.pi * prm_alpha)
    sw, cw = math.sqrt(sw2), math.sqrt(1 - sw2)
    gz = e / (sw * cw)
    g = {"L": (e, -gz * (-0.5 + sw2)), "R": (e, -gz * sw2)}   # (photon, Z) for Q = -1
    s = (p[0, 0] + p[1, 0]) ** 2
    dz = s - mz * mz + 1j * mz * wz
    A = {i + j: g[i][0] * g[j][0] / s + g[i][1] * g[j][1] / dz for i in "LR" for j in "LR"}
    # 1 + c = 4 p_e-.p_mu+ / s and 1 - c = 4 p_e-.p_mu- / s (massless), free of cancellation
    def dot(a, b):
        return a[0] * b[0] - a[1:] @ b[1:]
    opc, omc = 4 * dot(p[0], p[3]) / s, 4 * dot(p[0], p[2]) / s
    return s * s * ((abs(A["LL"]) ** 2 + abs(A["RR"]) ** 2) * opc ** 2
                    + (abs(A["LR"]) ** 2 + abs(A["RL"]) ** 2) * omc ** 2)


def test_ee_mumu_closed_form(oracle):
    # momenta built exactly from (cos theta, phi) so that the kinematics is
    # massless and back-to-back to the last bit (RAMBO output is so only to ~1e-13)
    rng = np.random.default_rng(0x48454745)
    mom = np.array([two_to_two_massive(200.0, 0.0, c, ph)
                    for c, ph in zip(rng.uniform(-1, 1, 256), rng.uniform(0, 2 * math.pi, 256))])
    f = oracle.me2(oracle.EE_MUMU, mom)
    cf = np.array([ee_closed_form(m) for m in mom])
    assert np.max(np.abs(f / cf - 1)) < 1e-13


def test_ee_mumu_qed_limit(oracle):
    # far below the Z pole with the Z decoupled: (1/4) sum |M|^2 = e^4 (1 + cos^2)
    prm = oracle.params(mz=1e7, wz=0.0)
    mom = oracle.generate(4, 64, 2, 10.0)
    f = oracle.me2(oracle.EE_MUMU, mom, prm)
    e2 = 4 * math.pi / 128
    c = mom[:, 2, 3] / mom[:, 2, 0]
    assert np.max(np.abs(0.25 * f / (e2 * e2 * (1 + c * c)) - 1)) < 1e-9


def test_ee_dsigma_dcos(oracle):
    # d sigma / d cos = (1/4 sum|M|^2) / (32 pi s): flat-phase-space estimate of the
    # forward-backward-integrated sigma agrees with the analytic integral
    s = 200.0 ** 2
    cs = np.linspace(-1, 1, 2001)
    vals = []
    for c in cs:
        p = np.array([[100, 0, 0, 100], [100, 0, 0, -100],
                      [100, 100 * math.sqrt(1 - c * c), 0, 100 * c],
                      [100, -100 * math.sqrt(1 - c * c), 0, -100 * c]])
        vals.append(oracle.me2(oracle.EE_MUMU, p)[0])
    sigma_analytic = np.trapezoid(0.25 * np.array(vals) / (32 * math.pi * s), cs)
    mom = oracle.generate(0x48454745, 20000, 2, 200.0)
    f = oracle.me2(oracle.EE_MUMU, mom)
    sig, err, _, _ = oracle.cross_section(f, oracle.phase_space_volume(200.0, 2), 200.0, 1, 1)
    assert abs(sig - sigma_analytic) < 5 * err + 1e-6 * sigma_analytic


# ------------------------------------------------------------------ gluons
def mandelstam(p):
    s = (p[0, 0] + p[1, 0]) ** 2
    q = p[0] - p[2]
    t = q[0] ** 2 - q[1:] @ q[1:]
    return s, t, -s - t


def test_gg_gg_closed_form(oracle):
    mom = oracle.generate(7, 32, 2, 1000.0)
    f = oracle.me2(oracle.GG_GG, mom)
    for k in range(mom.shape[0]):
        s, t, u = mandelstam(mom[k])
        cf = 256 * 4.5 * GS2 ** 2 * (3 - t * u / s ** 2 - s * u / t ** 2 - s * t / u ** 2)
        assert f[k] / cf - 1 == pytest.approx(0, abs=1e-12)


def _pt_case(oracle, n, seed, n_orders):
    mom = oracle.generate(seed, 1, n - 2, 1000.0)[0]
    P = mom.copy()
    P[:2] *= -1.0   # all-outgoing momenta

    def sij(i, j):
        q = P[i] + P[j]
        return q[0] ** 2 - q[1:] @ q[1:]
    gs = math.sqrt(GS2)
    worst_pt, worst_zero, scale = 0.0, 0.0, 0.0
    orders = list(itertools.permutations(range(1, n)))[::max(1, math.factorial(n - 1) // n_orders)]
    for hel in itertools.product((-1, 1), repeat=n):
        out = [-h if k < 2 else h for k, h in enumerate(hel)]   # crossing flips incoming helicities
        neg = [k for k in range(n) if out[k] < 0]
        pos = [k for k in range(n) if out[k] > 0]
        for perm in orders:
            order = [0] + list(perm)
            A = oracle.gluon_partial(mom, hel, order)
            if len(neg) == 2 or len(pos) == 2:
                i, j = neg if len(neg) == 2 else pos
                den = 1.0
                for k in range(n):
                    den *= math.sqrt(abs(sij(order[k], order[(k + 1) % n])))
                # |A| = g^(n-2) 2^(n/2) s_ij^2 / prod |<k k+1>|  for Tr(T^a T^b) = delta/2
                pt = gs ** (n - 2) * 2 ** (n / 2) * sij(i, j) ** 2 / den
                worst_pt = max(worst_pt, abs(abs(A) / pt - 1))
                scale = max(scale, abs(A))
            elif len(neg) <= 1 or len(pos) <= 1:
                worst_zero = max(worst_zero, abs(A))
    return worst_pt, worst_zero, scale


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_gluon_parke_taylor_and_zeros(oracle, n):
    worst_pt, worst_zero, scale = _pt_case(oracle, n, 21 + n, 12)
    assert worst_pt < 1e-11
    assert worst_zero < 1e-12 * scale


@pytest.mark.parametrize("proc,n", [("GG_GG", 4), ("GG_GGG", 5), ("GG_4G", 6), ("GG_5G", 7)])
def test_gluon_ward_identity(oracle, proc, n):
    pid = getattr(oracle, proc)
    mom = oracle.generate(13, 3 if n < 7 else 1, n - 2, 1000.0)
    base = oracle.me2(pid, mom)
    for leg in range(n):
        w = oracle.me2(pid, mom, oracle.params(gauge_leg=leg))
        assert np.all(np.sqrt(np.abs(w) / base) < 1e-12)


def test_gluon_lorentz_invariance(oracle):
    mom = oracle.generate(17, 3, 4, 1000.0)
    base = oracle.me2(oracle.GG_4G, mom)
    moved = rotate(boost(mom, [0.3, -0.5, 0.6]), [1, 2, 3], 0.7)
    assert np.max(np.abs(oracle.me2(oracle.GG_4G, moved) / base - 1)) < 1e-11


def test_gluon_bose_symmetry(oracle):
    mom = oracle.generate(19, 2, 4, 1000.0)
    base = oracle.me2(oracle.GG_4G, mom)
    perm = mom[:, [0, 1, 4, 2, 5, 3], :]
    assert np.max(np.abs(oracle.me2(oracle.GG_4G, perm) / base - 1)) < 1e-12
    swap_in = mom[:, [1, 0, 2, 3, 4, 5], :]
    assert np.max(np.abs(oracle.me2(oracle.GG_4G, swap_in) / base - 1)) < 1e-12


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_fierz_colour_matrix_equals_the_explicit_sum(oracle, n):
    """the oracle's 7-gluon colour matrix comes from Fierz expansion with loop
    counting; for up to 6 gluons it equals the brute-force sum over 8^n colours"""
    A, B = oracle.gluon_colour_matrix(n), oracle.gluon_colour_matrix_fierz(n)
    assert np.abs(A - B).max() < 1e-12 * np.abs(A).max()


def test_seven_gluon_bose_symmetry(oracle):
    mom = oracle.generate(29, 1, 5, 1000.0)
    base = oracle.me2(oracle.GG_5G, mom)
    perm = mom[:, [0, 1, 5, 2, 6, 4, 3], :]
    assert np.max(np.abs(oracle.me2(oracle.GG_5G, perm) / base - 1)) < 1e-12


def fierz_trace_product(traces, N=3):
    """Exact sum over gluon labels of a product of fundamental traces, each label
    occurring twice, by the SU(N) Fierz identity
    sum_a T^a_ij T^a_kl = (delta_il delta_kj - delta_ij delta_kl / N) / 2.
    Returns a Fraction (N = 3)."""
    from fractions import Fraction
    terms = [(Fraction(1), [list(t) for t in traces])]
    total = Fraction(0)
    while terms:
        c, trs = terms.pop()
        label = None
        for t in trs:
            if t:
                label = t[0]
                break
        if label is None:
            total += c * Fraction(N) ** len(trs)
            continue
        loc = [(i, j) for i, t in enumerate(trs) for j, x in enumerate(t) if x == label]
        (i1, j1), (i2, j2) = loc
        if i1 == i2:
            t = trs[i1]
            A, B = t[:j1] + t[j2 + 1:], t[j1 + 1:j2]     # Tr(A' a B a) with A = cyclic remainder
            rest = [x for k, x in enumerate(trs) if k != i1]
            terms.append((c / 2, rest + [A, B]))
            terms.append((-c / (2 * N), rest + [A + B]))
        else:
            t1 = trs[i1][j1 + 1:] + trs[i1][:j1]          # Tr(a X) -> X
            t2 = trs[i2][j2 + 1:] + trs[i2][:j2]          # Tr(a Y) -> Y
            rest = [x for k, x in enumerate(trs) if k not in (i1, i2)]
            terms.append((c / 2, rest + [t1 + t2]))
            terms.append((-c / (2 * N), rest + [t1, t2]))
    return total


def test_gluon_colour_matrix_four(oracle):
    C = oracle.gluon_colour_matrix(4)
    orders = [(0,) + p for p in itertools.permutations(range(1, 4))]
    for x, sx in enumerate(orders):
        for y, sy in enumerate(orders):
            exact = fierz_trace_product([list(sx), list(reversed(sy))])
            assert C[x, y] == pytest.approx(float(exact), abs=1e-13)
    # the diagonal by hand: (1/2)[C_F^3 N - (1/N)(1/2)(C_F^2 N - (N^2-1)/(4N))] = 19/6
    assert C[0, 0] == pytest.approx(19 / 6, abs=1e-13)


def test_gluon_colour_matrix_six(oracle):
    C = oracle.gluon_colour_matrix(6)
    assert C.shape == (120, 120)
    assert np.allclose(C, C.T, atol=1e-12)
    orders = [(0,) + p for p in itertools.permutations(range(1, 6))]
    rng = np.random.default_rng(2)
    picks = [(0, y) for y in range(120)] + [tuple(rng.integers(0, 120, 2)) for _ in range(30)]
    for x, y in picks:
        exact = fierz_trace_product([list(orders[x]), list(reversed(orders[y]))])
        assert C[x, y] == pytest.approx(float(exact), abs=1e-12)
    assert np.linalg.eigvalsh(C).min() > -1e-9


# ------------------------------------------------------------------ tops
@pytest.mark.parametrize("proc", ["UU_TT", "GG_TT"])
def test_helicity_sum_equals_trace(oracle, proc):
    pid = getattr(oracle, proc)
    rng = np.random.default_rng(3)
    for _ in range(4):
        m = two_to_two_massive(1000.0, 175.0, rng.uniform(-1, 1), rng.uniform(0, 2 * math.pi))
        a = oracle.me2(pid, m)[0]
        b = oracle.trace_me2(pid, m)
        assert a / b - 1 == pytest.approx(0, abs=1e-13)


def test_uu_tt_closed_form(oracle):
    # textbook q qbar -> Q Qbar: (1/36) sum |M|^2 = (4/9) g^4 (tau1^2 + tau2^2 + rho/2),
    # tau1 = 2 p1.p3 / s, tau2 = 2 p2.p3 / s, rho = 4 m^2 / s
    rng = np.random.default_rng(5)
    for _ in range(4):
        m = two_to_two_massive(800.0, 175.0, rng.uniform(-1, 1), rng.uniform(0, 2 * math.pi))
        s = 800.0 ** 2

        def dot(a, b):
            return a[0] * b[0] - a[1:] @ b[1:]
        t1, t2, rho = 2 * dot(m[0], m[2]) / s, 2 * dot(m[1], m[2]) / s, 4 * 175.0 ** 2 / s
        cf = 36 * (4 / 9) * GS2 ** 2 * (t1 ** 2 + t2 ** 2 + rho / 2)
        assert oracle.me2(oracle.UU_TT, m)[0] / cf - 1 == pytest.approx(0, abs=1e-13)


def test_gg_tt_ward_identity_per_colour(oracle):
    m = two_to_two_massive(1000.0, 175.0, 0.3, 0.4)
    prm0, big, worst = oracle.params(wt=0.0), 0.0, 0.0
    cols = [(a, b, i, j) for a in range(8) for b in range(8) for i in range(3) for j in range(3)][::5]
    for leg in (0, 1):
        prmw = oracle.params(wt=0.0, gauge_leg=leg)
        for hel in itertools.product((-1, 1), repeat=4):
            for col in cols:
                big = max(big, abs(oracle.amp_colour(oracle.GG_TT, m, hel, col, prm0)))
                worst = max(worst, abs(oracle.amp_colour(oracle.GG_TT, m, hel, col, prmw)))
    assert worst < 1e-13 * big


def test_top_pair_colour_matrix(oracle):
    # diagram colour factors (T^a T^b)_ij, (T^b T^a)_ij, f^abc T^c_ij:
    # C_F^2 N = 16/3, -C_F/(2N)... = -2/3, C_A (N^2-1)/2 = 12, and the f-row 6 / -6
    from oracle import lib  # noqa: F401
    m = two_to_two_massive(1000.0, 175.0, 0.1, 0.2)
    hel = [1, -1, 1, 1]
    cols = [(a, b, i, j) for a in range(8) for b in range(8) for i in range(3) for j in range(3)]
    # recover the colour matrix from amplitudes: sum_col |sum_d c_d M_d|^2 = me2_hel
    tot = sum(abs(oracle.amp_colour(oracle.GG_TT, m, hel, c)) ** 2 for c in cols)
    assert tot / oracle.me2_hel(oracle.GG_TT, m, hel) - 1 == pytest.approx(0, abs=1e-12)


def test_c1_helicity_selection(oracle):
    # V-A decays: only b(-) e+(+) nu(-) bbar(+) mu-(-) nu~(+) survive; 4 of 256
    mom = oracle.generate(3, 2, 6, 1000.0)
    H = oracle.helicities(oracle.GG_TT_6F)
    for m in mom:
        ph = oracle.me2_per_helicity(oracle.GG_TT_6F, m)
        tot = ph.sum()
        keep = [k for k in range(len(ph)) if ph[k] > 1e-20 * tot]
        assert len(keep) == 4
        for k in keep:
            assert list(H[k][2:]) == [-1, 1, -1, 1, -1, 1]


def test_c1_covariant_lorentz_invariance(oracle):
    # sum_{alpha beta} g^aa g^bb sum_ferm |M(e_alpha, e_beta)|^2 is a Lorentz scalar
    m = oracle.generate(8, 1, 6, 1000.0)[0]
    ferm = [-1, 1, -1, 1, -1, 1]

    def cov(mm):
        tot = 0.0
        for a in range(4):
            for b in range(4):
                g = (1 if a == 0 else -1) * (1 if b == 0 else -1)
                tot += g * oracle.me2_hel(oracle.GG_TT_6F, mm, [10 + a, 10 + b] + ferm)
        return tot
    base = cov(m)
    moved = rotate(boost(m, [0.2, 0.4, -0.3]), [0.3, 1, 0.2], 1.1)
    assert cov(moved) / base - 1 == pytest.approx(0, abs=1e-10)


# ------------------------------------------------------------------ Higgs pair
def test_c3_lorentz_invariance(oracle):
    mom = oracle.generate(5, 3, 6, 2000.0)
    prm = oracle.params(cms=1)
    f = oracle.me2(oracle.UD_UDHH_4B, mom, prm)
    for b in ([0.3, 0.2, -0.5], [0.0, 0.0, 0.9]):
        g = oracle.me2(oracle.UD_UDHH_4B, boost(mom, b), prm)
        assert np.max(np.abs(g / f - 1)) < 1e-10


@pytest.mark.parametrize("proc,legs", [("UD_UDHH_4B", (4, 6)), ("UD_UDHH_4B", (5, 7)), ("UU_UUHH_4B", (2, 3))])
def test_fermi_antisymmetry(oracle, proc, legs):
    pid = getattr(oracle, proc)
    prm = oracle.params(cms=1)
    mom = oracle.generate(5, 2, 6, 2000.0)
    i, j = legs
    for ev in mom:
        for hel, col in (([-1, -1, -1, -1, 1, 1, -1, -1], [0, 1, 0, 1, 2, 2, 1, 1]),
                         ([-1, -1, -1, -1, -1, -1, -1, -1], [0, 1, 1, 0, 2, 2, 0, 0])):
            A = oracle.amp_colour(pid, ev, hel, col, prm)
            ev2 = ev.copy()
            ev2[[i, j]] = ev[[j, i]]
            h2, c2 = list(hel), list(col)
            h2[i], h2[j] = hel[j], hel[i]
            c2[i], c2[j] = col[j], col[i]
            B = oracle.amp_colour(pid, ev2, h2, c2, prm)
            assert abs(A) > 0
            assert abs(A + B) < 1e-13 * abs(A)


@pytest.mark.parametrize("proc,mass", [("WW_HH", 91.1876 * math.sqrt(1 - 0.2222)), ("ZZ_HH", 91.1876)])
def test_longitudinal_vv_hh_unitarity(oracle, proc, mass):
    # V_L V_L -> H H stops growing like s / m_V^2 once contact, s-, t- and
    # u-channel pieces carry the right relative couplings
    pid = getattr(oracle, proc)
    prm = oracle.params(cms=1, wz=0.0, wh=0.0)
    H = oracle.helicities(pid)
    k00 = [k for k, h in enumerate(H) if h[0] == 0 and h[1] == 0][0]
    amps = []
    for rs in (2000.0, 20000.0):
        E = rs / 2
        pv, ph = math.sqrt(E * E - mass * mass), math.sqrt(E * E - 125.0 ** 2)
        c, s = 0.4, math.sqrt(1 - 0.16)
        m = np.array([[E, 0, 0, pv], [E, 0, 0, -pv], [E, ph * s, 0, ph * c], [E, -ph * s, 0, -ph * c]])
        amps.append(math.sqrt(oracle.me2_per_helicity(pid, m, prm)[k00]))
    # a s/m^2 growth would scale by 100 between the two energies
    assert amps[1] / amps[0] < 1.05
    assert amps[1] > 0.1


def test_c3_helicity_selection(oracle):
    # vector couplings conserve quark helicity; the scalar Yukawa gives b and bbar
    # equal helicities: 4 quark patterns x 6 b patterns = 24 of 256 survive
    mom = oracle.generate(9, 1, 6, 2000.0)[0]
    ph = oracle.me2_per_helicity(oracle.UD_UDHH_4B, mom, oracle.params(cms=1))
    assert np.sum(ph > 1e-20 * ph.sum()) == 24


def test_spinor_identities(oracle):
    rng = np.random.default_rng(11)
    for m in (0.0, 4.7, 175.0):
        for _ in range(10):
            p3 = rng.normal(size=3) * 300
            p = np.array([math.sqrt(p3 @ p3 + m * m), *p3])
            assert oracle.selfcheck_spinors(p, m) < 1e-13
    # directions along -z and +z
    for p in ([100.0, 0, 0, -100.0], [100.0, 0, 0, 100.0]):
        assert oracle.selfcheck_spinors(np.array(p), 0.0) < 1e-13


# ------------------------------------------------------------------ Higgs triple (SSSS)
MH = 125.0


def hhh_tree():
    """u d -> u d H H H by successive two-body splittings, all flat: (u (d (H (H H))))"""
    return [(0.0, 0.0, None, 2, -2, None), (0.0, 0.0, "flat", 3, -3, None),
            (0.0, 0.0, "flat", 4, -4, None), (0.0, 0.0, "flat", 5, 6, None)]


def hhh_events(seed, n, rs):
    from oracle import phase_space_tree as T
    mom, w = T.generate(seed, n, rs, hhh_tree(), 7, leg_mass=[0, 0, 0, 0, MH, MH, MH])
    assert np.all(w > 0)
    return mom


@pytest.mark.parametrize("proc,mass", [("WW_HHH", 91.1876 * math.sqrt(1 - 0.2222)), ("ZZ_HHH", 91.1876)])
def test_longitudinal_vv_hhh_unitarity(oracle, proc, mass):
    """V_L V_L -> H H H: single diagrams grow with the energy relative to the sum;
    with every tree of VVH, VVHH, HHH and HHHH at its coupling the sum falls like
    1/E^2 (|M| drops to ~0.02 from 2 to 20 TeV at fixed decay angles).  Leaving
    out the quartic scalar diagram, flipping the sign of a VVHH diagram, dropping
    the triple vector-exchange diagrams or giving a propagator the wrong momentum
    leaves ratios of 0.77 or more"""
    from oracle import phase_space_tree as T
    pid = getattr(oracle, proc)
    prm = oracle.params(cms=1, wz=0.0, wh=0.0)
    H = oracle.helicities(pid)
    k00 = [k for k, h in enumerate(H) if h[0] == 0 and h[1] == 0][0]
    tree = [(0.0, 0.0, None, 2, -2, None), (0.0, 0.0, "flat", 3, 4, None)]
    u = np.array([[0.4, 0.3, 0.7, 0.55, 0.2]])
    amps = []
    for rs in (2000.0, 20000.0):
        mom, _ = T.generate_from(u, rs, tree, 5, leg_mass=[0, 0, MH, MH, MH])
        E = rs / 2
        pv = math.sqrt(E * E - mass * mass)
        mom[0, 0] = [E, 0, 0, pv]
        mom[0, 1] = [E, 0, 0, -pv]
        amps.append(math.sqrt(oracle.me2_per_helicity(pid, mom[0], prm)[k00]))
    assert amps[0] > 0
    assert amps[1] / amps[0] < 0.05


def test_hhh_bose_symmetry(oracle):
    mom = hhh_events(21, 6, 2000.0)
    prm = oracle.params(cms=1)
    f = oracle.me2(oracle.UD_UDHHH, mom, prm)
    for perm in itertools.permutations((4, 5, 6)):
        moved = mom.copy()
        moved[:, [4, 5, 6]] = mom[:, list(perm)]
        assert np.max(np.abs(oracle.me2(oracle.UD_UDHHH, moved, prm) / f - 1)) < 1e-12


def test_hhh_lorentz_invariance(oracle):
    mom = hhh_events(22, 4, 2000.0)
    prm = oracle.params(cms=1)
    f = oracle.me2(oracle.UD_UDHHH, mom, prm)
    for b in ([0.3, 0.2, -0.5], [0.0, 0.0, 0.9]):
        g = oracle.me2(oracle.UD_UDHHH, boost(mom, b), prm)
        assert np.max(np.abs(g / f - 1)) < 1e-10
    g = oracle.me2(oracle.UD_UDHHH, rotate(mom, [1, 2, 3], 0.7), prm)
    assert np.max(np.abs(g / f - 1)) < 1e-10


def test_hhh_helicity_selection(oracle):
    # vector couplings of massless quarks conserve helicity along each line:
    # 4 of the 16 quark helicity patterns survive (the W W class only for left-handed)
    mom = hhh_events(23, 1, 2000.0)[0]
    ph = oracle.me2_per_helicity(oracle.UD_UDHHH, mom, oracle.params(cms=1))
    assert np.sum(ph > 1e-20 * ph.sum()) == 4


# ------------------------------------------------------------------ W W -> W W (EW VVVV, massive externals)
def ww_event(rs, mw, c, phi=0.4):
    E = rs / 2
    p = math.sqrt(E * E - mw * mw)
    s = math.sqrt(1 - c * c)
    return np.array([[E, 0, 0, p], [E, 0, 0, -p], [E, p * s * math.cos(phi), p * s * math.sin(phi), p * c],
                     [E, -p * s * math.cos(phi), -p * s * math.sin(phi), -p * c]])


def longitudinal(oracle, mom, prm):
    H = oracle.helicities(oracle.WW_WW)
    k = [i for i, h in enumerate(H) if all(x == 0 for x in h)][0]
    return math.sqrt(oracle.me2_per_helicity(oracle.WW_WW, mom, prm)[k])


def test_longitudinal_ww_ww_unitarity(oracle):
    """W_L W_L -> W_L W_L: single diagrams grow like E^4 / m_W^4; the quartic
    contact with photon and Z exchange cancels that to E^2, Higgs exchange the
    rest, and |M| stays flat (ratio 0.98 from 2 to 20 TeV).  Leaving out the
    Higgs, the Z or one term of the W W V vertex, or flipping the quartic sign,
    gives ratios of 99 to 1e6 (checked by planting each in a copy of the oracle)"""
    mw = 91.1876 * math.sqrt(1 - 0.2222)
    prm = oracle.params(cms=1, wz=0.0, wh=0.0)
    a = [longitudinal(oracle, ww_event(rs, mw, 0.3), prm) for rs in (2000.0, 20000.0)]
    assert 0.5 < a[1] / a[0] < 2.0


def test_ww_ww_goldstone_limit(oracle):
    """equivalence theorem in the gaugeless limit (g -> 0 at fixed v, so m_W ->
    0): the longitudinal amplitude becomes the Goldstone-boson one,
    -(m_H^2 / v^2) [s / (s - m_H^2) + t / (t - m_H^2)], up to O(g^2) and
    O(m_W^2 / s) (1e-4 to 1.5e-3 at these points)"""
    sw2, mh, v, alpha = 0.2222, 125.0, 246.22, 1e-6
    e = math.sqrt(4 * math.pi * alpha)
    gw = e / math.sqrt(sw2)
    mw = gw * v / 2
    prm = oracle.params(cms=1, wz=0.0, wh=0.0, alpha=alpha, mz=mw / math.sqrt(1 - sw2), sw2=sw2)

    def mdot(a, b):
        return a[0] * b[0] - a[1:] @ b[1:]
    for rs, c in ((300.0, 0.3), (1000.0, -0.5), (3000.0, 0.7)):
        m = ww_event(rs, mw, c)
        s, t = mdot(m[0] + m[1], m[0] + m[1]), mdot(m[0] - m[2], m[0] - m[2])
        gold = (mh * mh / (v * v)) * (s / (s - mh * mh) + t / (t - mh * mh))
        assert abs(longitudinal(oracle, m, prm) / abs(gold) - 1) < 5e-3


def test_ww_ww_lorentz_invariance(oracle):
    """the longitudinal diagrams cancel from E^4 / m_W^4 ~ 1.5e3 at 1 TeV, which
    the FP64 rounding of a changed frame carries: 1e-9 (measured 1.7e-10)"""
    prm = oracle.params(cms=1)
    mw = 91.1876 * math.sqrt(1 - 0.2222)
    mom = np.array([ww_event(1000.0, mw, c, phi) for c, phi in ((0.3, 0.4), (-0.7, 2.0), (0.95, 5.0))])
    f = oracle.me2(oracle.WW_WW, mom, prm)
    for b in ([0.3, 0.2, -0.5], [0.0, 0.0, 0.9]):
        g = oracle.me2(oracle.WW_WW, boost(mom, b), prm)
        assert np.max(np.abs(g / f - 1)) < 1e-9


def test_w_fermion_coupling_by_the_w_width(oracle):
    """The normalisation of the W-fermion vertex (Sec. 4.2.1, the FFV vertex with
    the W couplings; -g_W/sqrt2 for left-handed doublets) fixes the W width:
    Gamma(W -> e nu) = g_W^2 m_W / (48 pi) at tree level with massless leptons.
    The oracle's own vertex, spinors and massive polarisation vectors, summed
    over spins, must give it; a missing 1/sqrt2 doubles it."""
    e = math.sqrt(4 * math.pi / 128.0)
    gw = e / math.sqrt(0.2222)
    assert oracle.decay_width(0) == pytest.approx(gw * gw * 80.4 / (48 * math.pi), rel=1e-13)
    # the value the workload's inputs give (alpha = 1/128, sin^2 theta_W = 0.2222, m_W = 80.4)
    assert oracle.decay_width(0) == pytest.approx(0.235570432, rel=1e-8)


def test_w_fermion_coupling_by_the_top_width(oracle):
    """Gamma(t -> b W) = g_W^2 m_t^3 / (64 pi m_W^2) (1 - r)^2 (1 + 2 r), r =
    m_W^2 / m_t^2, at tree level with a massless b: the same vertex between a
    massive top spinor and a massive external W (all three polarisations)."""
    e = math.sqrt(4 * math.pi / 128.0)
    gw = e / math.sqrt(0.2222)
    for mt, mw in ((175.0, 80.4), (250.0, 91.0)):
        r = mw * mw / (mt * mt)
        expect = gw * gw * mt ** 3 / (64 * math.pi * mw * mw) * (1 - r) ** 2 * (1 + 2 * r)
        assert oracle.decay_width(1, oracle.params(mt=mt, mw=mw)) == pytest.approx(expect, rel=1e-13)
