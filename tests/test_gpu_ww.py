"""GPU parity of W- W+ -> W- W+ (massive external vector wavefunctions, the
weak quartic vertex wwwwxx, W W V vertices vvvxxx / jvvxxx and Higgs exchange;
the paper's Sec. 4.2.3-4.2.5) against the oracle's Feynman-diagram sum: |M|^2
on the oracle's events, the generated momenta and weights of its massive-beam
phase space, and the cross section with the massive-beam flux and the 1/9
spin average."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NAME = "ww_ww"
ROOTS = 1000.0
SEED = 0x57575757
MW = 91.1876 * math.sqrt(1 - 0.2222)      # the complex-mass relation m_W = c_W m_Z (widths aside)
LEG_MASS = [MW, MW, MW, MW]
TREE = [(0.0, 0.0, None, 2, 3, None)]


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


def to_aos(t):
    return np.ascontiguousarray(np.transpose(t.cpu().numpy(), (2, 0, 1)))


def to_soa(torch, mom):
    return torch.from_numpy(np.ascontiguousarray(np.transpose(mom, (1, 2, 0)))).cuda()


def test_me2_matches_oracle(torch, oracle, proc):
    """momenta in (the oracle's events, 3,000 and a ragged 41): every event
    within the process's bound of the extended-precision oracle (5e-12, 99 %
    within 1e-12): the longitudinal diagrams cancel from E^4 / m_W^4 ~ 1.5e3 at
    1 TeV, and the FP64 oracle is off by up to 6.6e-13 on these events"""
    import fp64_bounds as B
    for mom in B.tree_events(oracle, NAME):
        me2 = proc.eval(momenta=to_soa(torch, mom)).cpu().numpy()
        B.check(oracle, NAME, mom, me2)


def test_mixed_precision_error(torch, oracle):
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    from oracle import phase_space_tree as T
    mixed = H.Process(processes.by_name(NAME), precision="mixed")
    mom, _ = T.generate(SEED + 1, 4096, ROOTS, TREE, 4, leg_mass=LEG_MASS)
    me2 = mixed.eval(momenta=to_soa(torch, mom)).cpu().numpy()
    ref = oracle.me2(oracle.WW_WW, mom, oracle.params(cms=1))
    err = np.abs(me2 - ref) / np.abs(ref)
    print(f"WW->WW mixed: max rel err {err.max():.2e}, median {np.median(err):.2e}")
    assert np.median(err) < 1e-2


@pytest.mark.parametrize("n,offset", [(1000, 0), (4099, 321)])
def test_momenta_and_weights_match_oracle(torch, oracle, proc, n, offset):
    from oracle import phase_space_tree as T
    mom, w = proc.generate(n, seed=SEED, counter_offset=offset, sqrt_s=ROOTS, want_weights=True)
    torch.cuda.synchronize()
    ref_mom, ref_w = T.generate(SEED, n, ROOTS, TREE, 4, counter_offset=offset, leg_mass=LEG_MASS)
    got = to_aos(mom)
    assert np.abs(got - ref_mom).max() < 1e-12 * ROOTS
    msq = got[..., 0] ** 2 - (got[..., 1:] ** 2).sum(-1)
    assert np.abs(msq - MW * MW).max() < 1e-9 * ROOTS ** 2
    assert np.abs(w.cpu().numpy() / ref_w - 1).max() < 1e-12


def test_integrate_matches_oracle(torch, oracle, proc):
    """sigma with the flux lambda^(1/2)(s, m_W^2, m_W^2) and the 1/9 average over
    the two W's polarisations"""
    from oracle import phase_space_tree as T
    n = 1 << 12
    r = proc.integrate(n, seed=SEED, sqrt_s=ROOTS)
    mom, w = T.generate(SEED, n, ROOTS, TREE, 4, leg_mass=LEG_MASS)
    f = oracle.me2(oracle.WW_WW, mom, oracle.params(cms=1))
    sig, err, _, _ = oracle.cross_section(f, w, ROOTS, proc.ir.n_a_n_b, proc.ir.symmetry,
                                          beam_mass=(MW, MW), spin_states=9)
    print(f"WW->WW sigma: GPU {r['sigma_gev2']:.15e} oracle {sig:.15e} rel {r['sigma_gev2'] / sig - 1:.2e}")
    assert abs(r["sigma_gev2"] / sig - 1) <= 1e-12
    assert abs(r["err_gev2"] / err - 1) <= 1e-9
