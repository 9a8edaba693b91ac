"""The extended-precision oracle: the same oracle sources built with long
double arithmetic (64-bit significand) give the reference against which the
FP64 path's per-event error is bounded (tests/fp64_bounds.py).

Checks, on the CPU:
* the long-double build reproduces the closed forms the FP64 oracle is pinned
  to (C0's helicity amplitudes, the W and top widths), at its own precision;
* on every parity event set, the FP64 oracle's own error against it is at most
  the tabulated X, and the GPU bound B follows from X by the stated rule (so
  the bound is one an FP64 evaluation can meet);
* the two builds agree to the FP64 rounding level on well-conditioned events
  (they evaluate the same rules).
"""
import math

import numpy as np
import pytest

import fp64_bounds as B


def test_extended_build_meets_the_closed_forms(oracle):
    from test_oracle_amplitudes import ee_closed_form, two_to_two_massive
    rng = np.random.default_rng(11)
    mom = np.array([two_to_two_massive(200.0, 0.0, c, ph)
                    for c, ph in zip(rng.uniform(-1, 1, 64), rng.uniform(0, 2 * math.pi, 64))])
    got = oracle.me2(oracle.EE_MUMU, mom, extended=True)
    cf = np.array([ee_closed_form(m) for m in mom])
    assert np.max(np.abs(got / cf - 1)) < 2e-15
    e = math.sqrt(4 * math.pi / 128.0)
    gw = e / math.sqrt(0.2222)
    assert oracle.decay_width(0, extended=True) == pytest.approx(gw * gw * 80.4 / (48 * math.pi), rel=2e-15)


def test_bounds_follow_the_rule():
    for name, x in B.X_ORACLE.items():
        b = B.BOUND[name]
        if x <= 5e-13:
            assert b == 1e-12
        else:
            assert 4 * x * (1 - 1e-12) <= b <= 10 * x
    # the configured FP64 workloads keep the 1e-12 bar
    assert B.BOUND["ee_mumu"] == B.BOUND["gg_ttbar_6f"] == B.BOUND["gg_4g"] == 1e-12


@pytest.mark.parametrize("name", ["ee_mumu", "gg_ttbar_6f", "ud_udhh_4b", "gg_4g"])
def test_fp64_oracle_within_x_on_rambo_parity_events(oracle, name):
    mom = B.rambo_events(oracle, name)
    ext = B.reference(oracle, name, mom)
    f64 = B.reference(oracle, name, mom, extended=False)
    nz = ext != 0
    assert np.array_equal(f64 == 0, ext == 0)
    err = np.abs(f64[nz] / ext[nz] - 1)
    print(f"{name}: FP64 oracle vs long double max {err.max():.2e}, median {np.median(err):.2e}")
    assert err.max() <= B.X_ORACLE[name]
    assert np.median(err) < 1e-13


@pytest.mark.parametrize("name", ["ud_udhhh", "ww_ww", "gg_ttbar_6f_had", "gg_ttbar_6f_bw"])
def test_fp64_oracle_within_x_on_tree_parity_events(oracle, name):
    worst = 0.0
    for mom in B.tree_events(oracle, name):
        ext = B.reference(oracle, name, mom)
        f64 = B.reference(oracle, name, mom, extended=False)
        err = np.abs(f64 / ext - 1)
        worst = max(worst, err.max())
    print(f"{name}: FP64 oracle vs long double max {worst:.2e}")
    assert worst <= B.X_ORACLE[name]
