"""Pins of the oracle's adaptive importance sampling (VEGAS-style grids over the
phase-space uniforms): the map is the identity on a uniform grid and keeps the
measure on any grid, refinement leaves a flat integrand's grid alone and moves
bins onto a peak, and the adaptive integral of a known function converges to
its exact value faster than plain sampling."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def V(oracle):
    from oracle import vegas
    return vegas


def test_uniform_grid_is_the_identity(oracle, V):
    r = oracle.uniforms_bulk(3, 5000, 4)
    x, jac, bins = V.map_uniforms(r, V.uniform_grid(4, 32))
    assert np.abs(x - r).max() < 1e-15
    assert np.abs(jac - 1).max() < 1e-14
    assert np.array_equal(bins, np.minimum((r * 32).astype(int), 31))


def test_any_grid_keeps_the_measure(oracle, V):
    """x(r) is monotone and continuous, maps 0 -> 0 and 1 -> 1, and its Jacobian
    integrates to 1 (midpoint rule within each bin is exact: J is constant there)"""
    rng = np.random.default_rng(4)
    B = 16
    edges = np.concatenate([[0.0], np.sort(rng.uniform(0, 1, B - 1)), [1.0]])[None, :]
    r = np.linspace(1e-9, 1 - 1e-9, 20001)[:, None]
    x, jac, _ = V.map_uniforms(r, edges)
    assert np.all(np.diff(x[:, 0]) > 0)
    assert abs(x[0, 0]) < 1e-8 and abs(x[-1, 0] - 1) < 1e-8
    mid = ((np.arange(B) + 0.5) / B)[:, None]
    _, jm, _ = V.map_uniforms(mid, edges)
    assert abs(jm.sum() / B - 1.0) < 1e-14


def test_flat_integrand_keeps_the_grid(V):
    g = V.uniform_grid(3, 20)
    assert np.abs(V.refine(g, np.ones((3, 20))) - g).max() < 1e-14


def test_peak_draws_the_bins(V):
    B = 20
    d = np.zeros((1, B))
    d[0, 7] = 5.0
    new = V.refine(V.uniform_grid(1, B), d)[0]
    assert np.all(np.diff(new) > 0)
    inside = np.sum((new > 6 / B) & (new < 9 / B))        # smoothing spreads the peak over bins 6..8
    assert inside >= B - 3


def test_adaptive_integral_of_a_peaked_function(V):
    """prod_d g(x_d) with g a normalised Gaussian of width 0.05 at 0.3: exact
    integral 1; the adapted iterations' errors are far below plain sampling's"""
    a, c, D = 0.05, 0.3, 3
    norm = a * math.sqrt(math.pi) / 2 * (math.erf((1 - c) / a) + math.erf(c / a))

    def f(x):
        return np.prod(np.exp(-((x - c) / a) ** 2) / norm, axis=1)

    per, (mean, err, chi2), _ = V.integrate(f, 77, 20000, 6, D, 32)
    assert abs(mean - 1.0) < 4 * err
    assert per[-1][1] < per[0][1] / 4          # the first iteration is plain sampling
    assert chi2 < 5
