"""GPU parity of the adaptive integration (VEGAS grids over the uniforms of the
resonance-tree phase space, the role of the paper's BASES integrator in
Sec. 1 and 6): every pass's cross section and error, the combination and the
final grid of heget_integrate_adaptive against the oracle's adaptive integrator
driven by the oracle's tree generator and |M|^2."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NAME = "gg_ttbar_6f_bw"
ROOTS = 1000.0
SEED = 0x56454741
MT, WT, MW, WW = 175.0, 1.55, 80.4, 2.085


def oracle_tree():
    return [(0.0, 0.0, None, -2, -3, None),
            (MT, WT, "bw", 2, -4, 20.0),
            (MT, WT, "bw", 5, -5, 20.0),
            (MW, WW, "bw", 3, 4, 20.0),
            (MW, WW, "bw", 6, 7, 20.0)]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def proc(torch):
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    return H.Process(processes.by_name(NAME))


def oracle_integrand(oracle, proc):
    from oracle import phase_space_tree as T
    flux = 1.0 / (2.0 * ROOTS * ROOTS) / 4.0 / proc.ir.n_a_n_b / proc.ir.symmetry

    def f(x):
        mom, psw = T.generate_from(x, ROOTS, oracle_tree(), 8)
        return oracle.me2(oracle.GG_TT_6F, mom, oracle.params()) * psw * flux
    return f


def test_grid_dims(proc):
    assert proc.grid_dims == 14          # 4 resonance masses + 5 decays x (cos theta, phi)


def test_passes_and_grid_match_oracle(torch, oracle, proc):
    """4 passes of 8192 events, 16 bins.  Pass 0 runs on the uniform grid (the
    events of heget_integrate up to the map's rounding) and meets 1e-12 in sigma;
    later passes run on grids refined from device and oracle bin sums that agree
    to ~1e-15, so their events differ by that much more, which a Breit-Wigner
    pole amplifies by up to 1 / Gamma-widths: 1e-11 in sigma, 1e-9 in its error"""
    from oracle import vegas
    n, iters, B = 8192, 4, 16
    per, comb, chi2, grid = proc.integrate_adaptive(n, iterations=iters, bins=B, seed=SEED, sqrt_s=ROOTS)
    ref_per, (ref_mean, ref_err, ref_chi2), ref_grid = vegas.integrate(
        oracle_integrand(oracle, proc), SEED, n, iters, proc.grid_dims, B)
    for k, (r, (s, e)) in enumerate(zip(per, ref_per)):
        print(f"pass {k}: GPU {r['sigma_gev2']:.15e} +- {r['err_gev2']:.3e}  oracle {s:.15e} +- {e:.3e}"
              f"  rel {r['sigma_gev2'] / s - 1:.2e}")
        assert r["n_generated"] == n and r["n_accepted"] == n
        assert abs(r["sigma_gev2"] / s - 1) <= (1e-12 if k == 0 else 1e-11)
        assert abs(r["err_gev2"] / e - 1) <= 1e-9
    assert abs(comb["sigma_gev2"] / ref_mean - 1) <= 1e-11
    assert abs(comb["err_gev2"] / ref_err - 1) <= 1e-9
    assert abs(chi2 - ref_chi2) <= 1e-6 * max(1.0, ref_chi2)
    assert comb["n_generated"] == iters * n
    assert abs(comb["sigma_pb"] / (comb["sigma_gev2"] * 0.3893793721e9) - 1) < 1e-15
    print(f"final grid: max |GPU - oracle| {np.abs(grid - ref_grid).max():.2e}")
    assert np.abs(grid - ref_grid).max() < 1e-12
    assert np.all(np.diff(grid, axis=1) > 0)
    assert np.all(grid[:, 0] == 0.0) and np.all(grid[:, -1] == 1.0)


def test_one_pass_is_plain_integration(torch, proc):
    """on the uniform starting grid the map is the identity up to rounding: one
    pass gives heget_integrate's cross section"""
    n = 1 << 14
    per, comb, chi2, _ = proc.integrate_adaptive(n, iterations=1, bins=8, seed=SEED, sqrt_s=ROOTS)
    r = proc.integrate(n, seed=SEED, sqrt_s=ROOTS)
    assert abs(per[0]["sigma_gev2"] / r["sigma_gev2"] - 1) < 1e-12
    assert abs(comb["sigma_gev2"] / r["sigma_gev2"] - 1) < 1e-12
    assert abs(comb["err_gev2"] / r["err_gev2"] - 1) < 1e-9
    assert chi2 == 0.0


def test_adaptation_reduces_the_error(torch, proc):
    """the grid learns what the Breit-Wigner mapping leaves (the angular and
    off-peak structure): the last pass's error over 2^18 events is below the
    first's, and the passes agree (chi^2 per degree of freedom small)"""
    n = 1 << 18
    per, comb, chi2, _ = proc.integrate_adaptive(n, iterations=6, bins=32, seed=SEED + 7, sqrt_s=ROOTS)
    rel = [p["err_gev2"] / p["sigma_gev2"] for p in per]
    print("relative error per pass:", " ".join(f"{x:.2e}" for x in rel), f"chi2/dof {chi2:.2f}")
    assert rel[-1] < 0.8 * rel[0]
    assert chi2 < 5.0
    assert comb["err_gev2"] < min(p["err_gev2"] for p in per)


def test_argument_errors(torch, proc):
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import _lib, processes
    for bins in (1, 33):
        with pytest.raises(RuntimeError):
            proc.integrate_adaptive(1024, iterations=2, bins=bins, seed=1, sqrt_s=ROOTS)
    with pytest.raises(RuntimeError):
        proc.integrate_adaptive(1024, iterations=0, bins=8, seed=1, sqrt_s=ROOTS)
    rambo = H.Process(processes.by_name("gg_ttbar_6f"))
    assert rambo.grid_dims == 0
    L = _lib.load()
    comb = _lib.heget_result()
    rc = L.heget_integrate_adaptive(rambo._h, 1024, 2, 8, ROOTS, 1, None, comb, None, None, None)
    assert rc == _lib.HEGET_E_UNSUPPORTED
    assert math.isfinite(proc.integrate(256, seed=1, sqrt_s=ROOTS)["sigma_gev2"])


def test_repeated_calls_give_the_same_bits(torch, proc):
    """the handle's buffers grow for a larger n and are reused for a smaller
    one; a call's results depend only on its arguments"""
    args = dict(iterations=3, bins=12, seed=SEED + 3, sqrt_s=ROOTS)
    first = proc.integrate_adaptive(3000, **args)
    proc.integrate_adaptive(9001, **args)
    again = proc.integrate_adaptive(3000, **args)
    assert first[0] == again[0] and first[1] == again[1] and first[2] == again[2]
    assert np.array_equal(first[3], again[3])
