"""FP64 CPU oracle for the per-event amplitude path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this package.  It loads ``oracle/_build/liboracle.so`` (built by
``oracle/build.py``) and shares no code with the product library.

Every function here is a thin ctypes wrapper over ``oracle.h``; the physics
lives in the C++ sources next to this file:

* ``kinematics.cpp`` -- Philox4x32-10 uniforms, RAMBO, the gluon cut.
* ``processes.cpp``  -- Feynman-diagram sums for C0/C1/C3 and 2->2 checks,
  written from the Lagrangians of the paper's Sec. 4.2 (FFV, FFS, VVS, VVSS, SSS)
  with explicit Dirac matrices and brute-force SU(3) colour sums.
* ``gluons.cpp``     -- colour-ordered Berends-Giele recursion for n gluons and
  the trace-basis colour matrix by brute force.
* ``quark_lines.cpp`` -- u ubar -> t tbar + n gluons (n <= 3): every tree
  diagram with explicit Dirac matrices, colour summed over explicit SU(3)
  indices through the diagrams' colour matrix.
* ``phase_space_tree.py`` -- (numpy) the resonance phase space of the paper's
  Appendix A at a fixed collision energy: nested two-body decays with
  Breit-Wigner mapped invariant masses.
* ``vegas.py`` -- (numpy) adaptive importance sampling of the phase-space
  uniforms (VEGAS grids, Lepage's refinement), the BASES role.

Parity unpinned: the size of the H^3 contribution in u d -> u d H H and the
Yukawa normalisation are definitional (same written convention on both sides);
every other piece is pinned by tests in ``tests/test_oracle_*.py``.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
# the same sources built with long double arithmetic: the extended-precision
# reference that bounds the rounding of an FP64 evaluation (oracle/build.py)
_LIB_LD_PATH = os.path.join(_HERE, "_build", "liboracle_ld.so")

EE_MUMU, GG_TT_6F, GG_4G, UD_UDHH_4B = 0, 1, 2, 3
GG_GG, GG_GGG, UU_TT, GG_TT, UU_UUHH_4B, WW_HH, ZZ_HH = 10, 11, 12, 13, 14, 16, 17
UD_UDHHH, WW_HHH, ZZ_HHH, WW_WW, GG_5G = 4, 18, 19, 20, 21
# u ubar -> t tbar + 1, 2, 3 gluons by Feynman diagrams (quark_lines.cpp); UU_TT_DIAG: no gluon
UU_TTG, UU_TTGG, UU_TTGGG, UU_TT_DIAG = 22, 23, 24, 25


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("sw2", ctypes.c_double),
                ("mz", ctypes.c_double), ("wz", ctypes.c_double),
                ("mw", ctypes.c_double), ("ww", ctypes.c_double),
                ("mt", ctypes.c_double), ("wt", ctypes.c_double),
                ("mh", ctypes.c_double), ("wh", ctypes.c_double),
                ("alpha_s", ctypes.c_double), ("mb_yuk", ctypes.c_double),
                ("cms", ctypes.c_int), ("gauge_leg", ctypes.c_int)]


def params(**kw):
    """SM inputs of the benchmark configurations, overridable by keyword."""
    d = dict(alpha=1.0 / 128.0, sw2=0.2222, mz=91.1876, wz=2.4952, mw=80.4, ww=2.085,
             mt=175.0, wt=1.55, mh=125.0, wh=0.00407, alpha_s=0.118, mb_yuk=4.7,
             cms=0, gauge_leg=-1)
    d.update(kw)
    return Params(**d)


_libs = {}


def lib(extended=False):
    """the FP64 oracle library, or with extended=True its long-double build"""
    path = _LIB_LD_PATH if extended else _LIB_PATH
    if path not in _libs:
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        dp, ip = P(ctypes.c_double), P(ctypes.c_int)
        L.or_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.or_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, dp]
        L.or_uniforms_bulk.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, dp]
        L.or_rambo.argtypes = [ctypes.c_double, ctypes.c_int, dp, dp]
        L.or_rambo.restype = ctypes.c_double
        L.or_phase_space_volume.argtypes = [ctypes.c_double, ctypes.c_int]
        L.or_phase_space_volume.restype = ctypes.c_double
        L.or_generate.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                  ctypes.c_double, dp]
        L.or_cut_gluons.argtypes = [ctypes.c_int64, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                                    P(ctypes.c_int32)]
        L.or_eval.argtypes = [ctypes.c_int, P(Params), ctypes.c_int64, dp, dp, ctypes.c_int]
        L.or_amp_colour.argtypes = [ctypes.c_int, P(Params), dp, ip, ip, dp]
        L.or_me2_per_helicity.argtypes = [ctypes.c_int, P(Params), dp, dp]
        L.or_helicities.argtypes = [ctypes.c_int, ip]
        L.or_me2_hel.argtypes = [ctypes.c_int, P(Params), dp, ip, dp]
        L.or_gluon_partial.argtypes = [ctypes.c_int, P(Params), dp, ip, ip, dp]
        L.or_gluon_colour_matrix.argtypes = [ctypes.c_int, dp]
        L.or_gluon_colour_matrix_fierz.argtypes = [ctypes.c_int, dp]
        L.or_trace_me2.argtypes = [ctypes.c_int, P(Params), dp, dp]
        L.or_nlegs.argtypes = [ctypes.c_int]
        L.or_uu_tt_gluons_diagrams.argtypes = [ctypes.c_int]
        L.or_selfcheck_spinors.argtypes = [dp, ctypes.c_double]
        L.or_selfcheck_spinors.restype = ctypes.c_double
        L.or_decay_width.argtypes = [ctypes.c_int, P(Params), dp]
        L.or_condition.argtypes = [ctypes.c_int, P(Params), ctypes.c_int64, dp, dp, ctypes.c_int]
        _libs[path] = L
    return _libs[path]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return list(o)


def uniforms(seed, event, n):
    u = np.zeros(n)
    lib().or_uniforms(seed, event, n, _dp(u))
    return u


def uniforms_bulk(seed, n_events, n, counter_offset=0):
    """u[i][k]: the first n uniforms of events counter_offset + i"""
    u = np.zeros((n_events, n))
    lib().or_uniforms_bulk(seed, counter_offset, n_events, n, _dp(u))
    return u


def rambo(sqrt_s, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = u.size // 4
    p = np.zeros((n, 4))
    w = lib().or_rambo(sqrt_s, n, _dp(u), _dp(p))
    return p, w


def phase_space_volume(sqrt_s, n):
    return lib().or_phase_space_volume(sqrt_s, n)


def generate(seed, n_events, n_out, sqrt_s, counter_offset=0):
    """Momenta [n_events][2 + n_out][4]: beams along +-z, RAMBO final state."""
    mom = np.zeros((n_events, n_out + 2, 4))
    lib().or_generate(seed, counter_offset, n_events, n_out, sqrt_s, _dp(mom))
    return mom


def cut_gluons(mom, pt_min=20.0, dr_min=0.4):
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    out = np.zeros(mom.shape[0], dtype=np.int32)
    lib().or_cut_gluons(mom.shape[0], mom.shape[1], _dp(mom), pt_min, dr_min,
                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return out


def nlegs(proc):
    return lib().or_nlegs(proc)


def uu_tt_gluons_diagrams(n_gluons):
    """the number of tree diagrams u ubar -> t tbar + n gluons sums (a four-gluon
    vertex counted once per colour structure)"""
    return lib().or_uu_tt_gluons_diagrams(n_gluons)


def me2(proc, mom, prm=None, threads=0, extended=False):
    """Helicity- and colour-summed |M|^2 per event (no averaging).  With
    extended=True the long-double build evaluates it on the same (FP64)
    momenta and parameters and the result is rounded to FP64 once."""
    prm = prm or params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    if mom.ndim == 2:
        mom = mom[None]
    out = np.zeros(mom.shape[0])
    rc = lib(extended).or_eval(proc, ctypes.byref(prm), mom.shape[0], _dp(mom), _dp(out), threads)
    if rc != 0:
        raise ValueError(f"oracle: unknown process {proc}")
    return out


def condition(proc, mom, prm=None, threads=0):
    """Per-event conditioning kappa of the diagram sum (see oracle.h)."""
    prm = prm or params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    if mom.ndim == 2:
        mom = mom[None]
    out = np.zeros(mom.shape[0])
    if lib().or_condition(proc, ctypes.byref(prm), mom.shape[0], _dp(mom), _dp(out), threads) != 0:
        raise ValueError(f"oracle: no diagram list for process {proc}")
    return out


def amp_colour(proc, mom, hel, col, prm=None):
    prm = prm or params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    out = np.zeros(2)
    if lib().or_amp_colour(proc, ctypes.byref(prm), _dp(mom), _ip(h), _ip(c), _dp(out)) != 0:
        raise ValueError(proc)
    return complex(out[0], out[1])


def helicities(proc):
    n = lib().or_helicities(proc, None)
    t = np.zeros((n, nlegs(proc)), dtype=np.int32)
    lib().or_helicities(proc, _ip(t))
    return t


def me2_per_helicity(proc, mom, prm=None):
    prm = prm or params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    n = lib().or_helicities(proc, None)
    out = np.zeros(n)
    lib().or_me2_per_helicity(proc, ctypes.byref(prm), _dp(mom), _dp(out))
    return out


def me2_hel(proc, mom, hel, prm=None):
    """Colour-summed |M|^2 for one explicit helicity vector."""
    prm = prm or params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    out = np.zeros(1)
    if lib().or_me2_hel(proc, ctypes.byref(prm), _dp(mom), _ip(h), _dp(out)) != 0:
        raise ValueError(proc)
    return out[0]


def gluon_partial(mom, hel, order, prm=None):
    prm = prm or params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    n = mom.shape[0]
    out = np.zeros(2)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    o = np.ascontiguousarray(order, dtype=np.int32)
    if lib().or_gluon_partial(n, ctypes.byref(prm), _dp(mom), _ip(h), _ip(o), _dp(out)) != 0:
        raise ValueError(n)
    return complex(out[0], out[1])


def gluon_colour_matrix(n):
    k = math.factorial(n - 1)
    C = np.zeros((k, k))
    lib().or_gluon_colour_matrix(n, _dp(C))
    return C


def gluon_colour_matrix_fierz(n):
    k = math.factorial(n - 1)
    C = np.zeros((k, k))
    if lib().or_gluon_colour_matrix_fierz(n, _dp(C)) != 0:
        raise ValueError(n)
    return C


def trace_me2(proc, mom, prm=None):
    prm = prm or params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    out = np.zeros(1)
    if lib().or_trace_me2(proc, ctypes.byref(prm), _dp(mom), _dp(out)) != 0:
        raise ValueError(proc)
    return out[0]


def decay_width(which, prm=None, extended=False):
    """tree-level width (GeV) of W+ -> e+ nu_e (which 0) or t -> b W+ (which 1)
    from the oracle's own vertex, spinors and polarisation vectors"""
    prm = prm or params()
    out = np.zeros(1)
    if lib(extended).or_decay_width(which, ctypes.byref(prm), _dp(out)) != 0:
        raise ValueError(which)
    return out[0]


def selfcheck_spinors(p, m):
    p = np.ascontiguousarray(p, dtype=np.float64)
    return lib().or_selfcheck_spinors(_dp(p), m)


HBARC2_PB = 0.3893793721e9  # (hbar c)^2 in pb GeV^2 (PDG)


def cross_section(me2_values, phase_space_weight, sqrt_s, n_a_n_b, symmetry, passed=None, beam_mass=(0.0, 0.0),
                  spin_states=4, flux_in_weight=False):
    """sigma = (1/N) sum_i w_i with w_i = Phi_n * pass_i * F_i / (2 F spins n_a n_b S),
    the flux F = lambda^(1/2)(s, m_a^2, m_b^2) (s for massless beams) and spins
    the polarisation states of the two incoming particles (4 for fermions and
    gluons, 9 for two massive vector bosons), summed exactly (math.fsum).  With
    flux_in_weight the weights already hold 1 / (2 F) (hadronic collisions,
    s_hat per event).
    Returns (sigma_GeV^-2, err_GeV^-2, sum_w, sum_w2)."""
    s = sqrt_s * sqrt_s
    ma, mb = beam_mass
    flux = s if ma == 0.0 and mb == 0.0 else math.sqrt(max((s - (ma + mb) ** 2) * (s - (ma - mb) ** 2), 0.0))
    f = (1.0 if flux_in_weight else 1.0 / (2.0 * flux)) / spin_states / n_a_n_b / symmetry
    w = phase_space_weight * f * np.asarray(me2_values, dtype=np.float64)
    if passed is not None:
        w = np.where(np.asarray(passed) != 0, w, 0.0)
    n = w.size
    sw = math.fsum(w.tolist())
    sw2 = math.fsum((w * w).tolist())
    sigma = sw / n
    var = max(sw2 / n - sigma * sigma, 0.0)
    err = math.sqrt(var / max(n - 1, 1))
    return sigma, err, sw, sw2
