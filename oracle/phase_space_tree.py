"""Oracle (test infrastructure only): the resonance phase space of the paper's
Appendix A (Eq. ps2-resonance and the Breit-Wigner mapping of Sec. B of the
appendix) at a fixed collision energy.

The collision system (mass sqrt_s, at rest) and every resonance decay into two
daughters, each a final massless particle or another resonance:

    dPhi_n = dPhi_2(root) * prod_k [ds_k / (2 pi)] dPhi_2(R_k -> its daughters at s_k),

with dPhi_2(M; m1, m2) = lambda^(1/2)(M^2, m1^2, m2^2) / (8 pi M^2) for isotropic
decay angles in the parent's rest frame.  A resonance's invariant mass follows
either the Breit-Wigner mapping

    s_k = m^2 + m Gamma tan(theta),  ds_k = [(s_k - m^2)^2 + (m Gamma)^2] / (m Gamma) dtheta,

with theta uniform over the window |s_k - m^2| / (m Gamma) < min(window, m / Gamma)
intersected with the kinematic range, or a flat distribution over the range
(optionally windowed the same way).  Final particles have fixed masses (zero
unless given); the minimal mass of a resonance is the sum of the masses of the
final particles below it.  Kinematic range of the first daughter of a node of
mass M: [its minimal mass^2, (M - minimal mass of the second)^2]; of the
second: [its minimal mass^2, (M - mass of the first)^2].

Uniforms: the same Philox4x32-10 stream as RAMBO (two per counter block, the
event index in the counter); per node in index order, first one uniform for the
invariant mass of each daughter that is a resonance (first daughter first),
then cos(theta) = 2u - 1 and phi = 2 pi u' of the node's decay.

Written with numpy over events; no code shared with the library.
"""
import math

import numpy as np

from . import uniforms_bulk


def n_uniforms(nodes, hadronic=None):
    return sum(sum(1 for d in nd[3:5] if d < 0) + 2 for nd in nodes) + (2 if hadronic else 0)


def _sample_s(u, lo, hi, m, g, mapping, window):
    """invariant mass s in [lo, hi] (arrays) by the node's mapping; returns (s,
    ds / (2 pi) weight, valid)"""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if mapping == "bw" or (mapping == "flat" and window is not None and g > 0):
        w = min(window, m / g) if window is not None else m / g
        lo = np.maximum(lo, m * m - w * m * g)
        hi = np.minimum(hi, m * m + w * m * g)
    valid = hi > lo
    if mapping == "bw":
        mg = m * g
        t_lo = np.arctan((lo - m * m) / mg)
        t_hi = np.arctan((hi - m * m) / mg)
        t = t_lo + u * (t_hi - t_lo)
        s = m * m + mg * np.tan(t)
        jac = (t_hi - t_lo) * ((s - m * m) ** 2 + mg * mg) / mg
    else:
        s = lo + u * (hi - lo)
        jac = hi - lo
    s = np.where(valid, s, np.maximum(lo, 0.0))
    return s, np.where(valid, jac / (2.0 * math.pi), 0.0), valid


def _boost(P, M, q):
    """q (rest frame of P, of mass M) to the frame where P is given; arrays [n,4]"""
    E = P[:, 0]
    pq = P[:, 1] * q[:, 1] + P[:, 2] * q[:, 2] + P[:, 3] * q[:, 3]
    q0 = (E * q[:, 0] + pq) / M
    f = (q[:, 0] + q0) / (E + M)
    out = np.empty_like(q)
    out[:, 0] = q0
    out[:, 1:] = q[:, 1:] + f[:, None] * P[:, 1:]
    return out


def generate(seed, n_events, sqrt_s, nodes, n_legs, counter_offset=0, leg_mass=None, hadronic=None):
    """nodes[k] = (mass, width, mapping, d0, d1, window): node 0 is the collision
    (mass and width ignored), d >= 0 a final leg, d < 0 node -1 - d; mapping
    "bw" or "flat", window None (flat over the kinematic range) or the factor
    of min(window, m / Gamma).  Returns momenta [n][n_legs][4] (legs 0, 1 the
    beams along +-z) and the phase-space weight [n] (0 where a window is empty)."""
    u = uniforms_bulk(seed, n_events, n_uniforms(nodes, hadronic), counter_offset)
    return generate_from(u, sqrt_s, nodes, n_legs, leg_mass, hadronic)


def _min_mass(nodes, leg_mass, d):
    """minimal invariant mass of daughter d (a final leg d >= 0, or node -1 - d)"""
    if d >= 0:
        return leg_mass[d]
    node = nodes[-1 - d]
    return _min_mass(nodes, leg_mass, node[3]) + _min_mass(nodes, leg_mass, node[4])


def _hadronic_pair(u, sqrt_s, m0, m1, y_max, pt_min):
    """the paper's Appendix A at a hadron collider of energy sqrt_s with parton
    densities set to 1: rapidities y0, y1 flat in [-y_max, y_max], the first
    daughter's ln(m0^2 + pT^2) flat up to the kinematic limit, its azimuth
    flat; the second balances pT; x_a, x_b from momentum conservation.

        d Sigma_2 = dx_a dx_b dPhi_2 = (2 pi / S) dy_1 dy_0 dpT^2 / (4 pi)^2 dphi / (2 pi)

    Returns the daughters' lab momenta, the beams', and the weight
    dSigma_2 / (2 s_hat) (the partonic flux per event), 0 unless x_a, x_b < 1."""
    S = sqrt_s * sqrt_s
    y0 = -y_max + 2.0 * y_max * u[:, 0]
    y1 = -y_max + 2.0 * y_max * u[:, 3]
    lam = np.maximum((S - (m0 + m1) ** 2) * (S - (m0 - m1) ** 2), 0.0)
    pt2max = lam / (4.0 * S)
    llo = np.log(m0 * m0 + pt_min * pt_min)
    lhi = np.log(m0 * m0 + pt2max)
    L = llo + u[:, 1] * (lhi - llo)
    mt0sq = np.exp(L)
    pt = np.sqrt(np.maximum(mt0sq - m0 * m0, 0.0))
    phi = 2.0 * math.pi * u[:, 2]
    px, py = pt * np.cos(phi), pt * np.sin(phi)
    mt0 = np.sqrt(mt0sq)
    mt1 = np.sqrt(m1 * m1 + pt * pt)
    e0, z0 = mt0 * np.cosh(y0), mt0 * np.sinh(y0)
    e1, z1 = mt1 * np.cosh(y1), mt1 * np.sinh(y1)
    xa = (e0 + z0 + e1 + z1) / sqrt_s
    xb = (e0 - z0 + e1 - z1) / sqrt_s
    ok = (lhi > llo) & (xa < 1.0) & (xb < 1.0)
    sh = xa * xb * S
    w = (2.0 * math.pi / S) * (2.0 * y_max) * (2.0 * y_max) * mt0sq * (lhi - llo) / (16.0 * math.pi * math.pi)
    w = np.where(ok, w / (2.0 * sh), 0.0)
    n = u.shape[0]
    q0 = np.stack([e0, px, py, z0], axis=1)
    q1 = np.stack([e1, -px, -py, z1], axis=1)
    h = 0.5 * sqrt_s
    pa = np.stack([xa * h, np.zeros(n), np.zeros(n), xa * h], axis=1)
    pb = np.stack([xb * h, np.zeros(n), np.zeros(n), -xb * h], axis=1)
    return q0, q1, pa, pb, w


def generate_from(u, sqrt_s, nodes, n_legs, leg_mass=None, hadronic=None):
    """the same from given uniforms u[n][n_uniforms(nodes, hadronic)]; leg_mass[k]
    the mass of leg k (default all zero; legs 0 and 1 the beams).  hadronic =
    (y_max, pt_min): node 0 is a parton collision at a hadron collider of
    energy sqrt_s (parton densities 1, the partonic flux in the weight), its
    two daughters generated in rapidity, ln(m^2 + pT^2) and azimuth."""
    K = len(nodes)
    n = u.shape[0]
    leg_mass = [0.0] * n_legs if leg_mass is None else [float(x) for x in leg_mass]
    mom = np.zeros((n, n_legs, 4))
    ma, mb = leg_mass[0], leg_mass[1]
    if ma == 0.0 and mb == 0.0:
        h = 0.5 * sqrt_s
        mom[:, 0] = [h, 0.0, 0.0, h]
        mom[:, 1] = [h, 0.0, 0.0, -h]
    else:
        # beams of masses m_a, m_b along +-z in the collision frame
        s0 = sqrt_s * sqrt_s
        pz = math.sqrt(max((s0 - (ma + mb) * (ma + mb)) * (s0 - (ma - mb) * (ma - mb)), 0.0)) / (2.0 * sqrt_s)
        mom[:, 0] = [(s0 + ma * ma - mb * mb) / (2.0 * sqrt_s), 0.0, 0.0, pz]
        mom[:, 1] = [(s0 + mb * mb - ma * ma) / (2.0 * sqrt_s), 0.0, 0.0, -pz]
    weight = np.ones(n)
    mass = {0: np.full(n, float(sqrt_s))}            # node -> invariant mass sqrt(s)
    lab = {0: np.tile([sqrt_s, 0.0, 0.0, 0.0], (n, 1))}
    iu = 0
    for k in range(K):
        m_k, g_k, mp_k, d0, d1, win_k = nodes[k]
        M = mass[k]
        dm = {}
        # invariant masses of resonant daughters: first, then second
        for j, d in enumerate((d0, d1)):
            if d >= 0:
                dm[j] = np.full(n, leg_mass[d])
                continue
            other_mass = dm[0] if j == 1 else np.full(n, _min_mass(nodes, leg_mass, d1))
            hi = (M - other_mass) ** 2
            lo = np.full(n, _min_mass(nodes, leg_mass, d) ** 2)
            node = nodes[-1 - d]
            s, wj, valid = _sample_s(u[:, iu], lo, hi, node[0], node[1], node[2], node[5])
            iu += 1
            weight *= wj
            dm[j] = np.sqrt(s)
            mass[-1 - d] = dm[j]
        m0, m1 = dm[0], dm[1]
        if k == 0 and hadronic is not None:
            q0, q1, mom[:, 0], mom[:, 1], wh = _hadronic_pair(u[:, iu:iu + 4], sqrt_s, m0, m1, *hadronic)
            iu += 4
            weight *= wh
            for d, q in ((d0, q0), (d1, q1)):
                if d >= 0:
                    mom[:, d] = q
                else:
                    lab[-1 - d] = q
            continue
        lam = (M * M - (m0 + m1) ** 2) * (M * M - (m0 - m1) ** 2)
        lam = np.maximum(lam, 0.0)
        pst = np.sqrt(lam) / (2.0 * M)
        weight *= np.sqrt(lam) / (8.0 * math.pi * M * M)
        ct = 2.0 * u[:, iu] - 1.0
        phi = 2.0 * math.pi * u[:, iu + 1]
        iu += 2
        st = np.sqrt(1.0 - ct * ct)
        nvec = np.stack([st * np.cos(phi), st * np.sin(phi), ct], axis=1)
        e0 = (M * M + m0 * m0 - m1 * m1) / (2.0 * M)
        e1 = (M * M + m1 * m1 - m0 * m0) / (2.0 * M)
        q0 = np.concatenate([e0[:, None], pst[:, None] * nvec], axis=1)
        q1 = np.concatenate([e1[:, None], -pst[:, None] * nvec], axis=1)
        for d, q in ((d0, q0), (d1, q1)):
            ql = _boost(lab[k], M, q) if k > 0 else q
            if d >= 0:
                mom[:, d] = ql
            else:
                lab[-1 - d] = ql
    return mom, weight
