"""GPU parity of the resonance phase space (the paper's Appendix A at fixed
collision energy) for the C1 process: momenta and per-event weights of
heget_generate against the oracle's tree generator, |M|^2 of the generated
events, and the cross section of heget_integrate against the oracle's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NAME = "gg_ttbar_6f_bw"
ROOTS = 1000.0
SEED = 0x4845474B
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


def to_aos(t):
    return np.ascontiguousarray(np.transpose(t.cpu().numpy(), (2, 0, 1)))


def to_soa(torch, mom):
    return torch.from_numpy(np.ascontiguousarray(np.transpose(mom, (1, 2, 0)))).cuda()


@pytest.mark.parametrize("n,offset", [(1000, 0), (4099, 12345)])
def test_momenta_and_weights_match_oracle(torch, oracle, proc, n, offset):
    from oracle import phase_space_tree as T
    mom, w = proc.generate(n, seed=SEED, counter_offset=offset, sqrt_s=ROOTS, want_weights=True)
    torch.cuda.synchronize()
    ref_mom, ref_w = T.generate(SEED, n, ROOTS, oracle_tree(), 8, counter_offset=offset)
    got = to_aos(mom)
    assert np.abs(got - ref_mom).max() < 1e-12 * ROOTS
    w = w.cpu().numpy()
    assert np.all(ref_w > 0)
    assert np.abs(w / ref_w - 1).max() < 1e-12


def test_eval_generates_the_same_events(torch, proc):
    n = 3000
    _, mom_eval = proc.eval(n=n, seed=SEED, counter_offset=5, sqrt_s=ROOTS, want_momenta=True)
    mom_gen = proc.generate(n, seed=SEED, counter_offset=5, sqrt_s=ROOTS)
    torch.cuda.synchronize()
    assert torch.equal(mom_eval, mom_gen)


def test_me2_of_tree_events_matches_oracle(torch, oracle, proc):
    """F on the tree's events (on the top and W peaks, where the RAMBO events
    rarely land), momenta-in: the oracle's momenta fed to both sides, every
    event within the process's bound of the extended-precision oracle.  On the
    poles the denominators q^2 - m^2 come from cancelling momentum sums: the
    FP64 oracle is off by up to 7.3e-13 there, by 1.1e-13 at the median.  The
    median is held to twice that of the FP64 oracle on the same events: no FP64
    evaluation is expected to beat an independent one by more than the change
    of operation order allows."""
    import fp64_bounds as B
    (mom,) = B.tree_events(oracle, NAME)
    me2 = proc.eval(momenta=to_soa(torch, mom)).cpu().numpy()
    err = B.check(oracle, NAME, mom, me2)
    ref = B.reference(oracle, NAME, mom)
    x = np.abs(B.reference(oracle, NAME, mom, extended=False) - ref) / np.abs(ref)
    print(f"median: GPU {np.median(err):.3e}, FP64 oracle {np.median(x):.3e}")
    assert np.median(err) <= 2.0 * np.median(x)


def test_integrate_matches_oracle(torch, oracle, proc):
    """sigma from the GPU's own events against the oracle's own: the two
    generators agree to ~1e-13 in the momenta, which near a Breit-Wigner pole
    moves F by up to ds / (m Gamma) (~1e-11 for the top) per event; these
    differences average out in the sum, which meets the 1e-12 bar of sigma"""
    from oracle import phase_space_tree as T
    n = 1 << 13
    r = proc.integrate(n, seed=SEED, sqrt_s=ROOTS)
    mom, w = T.generate(SEED, n, ROOTS, oracle_tree(), 8)
    f = oracle.me2(oracle.GG_TT_6F, mom, oracle.params())
    sig, err, _, _ = oracle.cross_section(f, w, ROOTS, proc.ir.n_a_n_b, proc.ir.symmetry)
    print(f"tree sigma: GPU {r['sigma_gev2']:.15e} oracle {sig:.15e} rel {r['sigma_gev2'] / sig - 1:.2e}")
    assert r["n_generated"] == n and r["n_accepted"] == n
    assert abs(r["sigma_gev2"] / sig - 1) <= 1e-12
    assert abs(r["err_gev2"] / err - 1) <= 1e-9


def test_resonance_mapping_error_is_small(torch):
    """with the resonances mapped onto their poles the Monte Carlo error of
    sigma over 2^18 events is below 1 % (flat RAMBO events leave it above 50 %
    for this process)"""
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    r = H.Process(processes.by_name(NAME)).integrate(1 << 18, seed=SEED + 1, sqrt_s=ROOTS)
    assert r["err_gev2"] / r["sigma_gev2"] < 0.01
