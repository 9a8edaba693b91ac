"""GPU parity of the HIP path against the oracle, through the C ABI.

FP64 path: every event within the per-process bound of fp64_bounds.py of the
oracle's extended-precision (long double) F -- 1e-12 for the configured
workloads C0, C1 and C2, and for u d -> u d H H (C3), whose gauge cancellations
already take an independent FP64 evaluation (the FP64 oracle) to 4.9e-12 of
the exact value, 2e-11 with 98 % of the events within 1e-12.  Mixed path: max
and median relative error against the same reference are reported; the test
only guards against gross failure (max < 1e-2).  Sizes: a few thousand events
(several 256-lane blocks plus a ragged tail) compared element by element, and
the full workload sizes in the benchmark's launch configuration compared on
sampled events.
"""
import math

import numpy as np
import pytest

import fp64_bounds as B

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12

# name -> (oracle process id, final-state multiplicity, sqrt_s, oracle params, seed, full-size N)
CASES = {
    "ee_mumu": ("EE_MUMU", 2, 200.0, {}, 0x48454745, 65536),
    "gg_ttbar_6f": ("GG_TT_6F", 6, 1000.0, {}, 0x48454746, 1 << 20),
    "ud_udhh_4b": ("UD_UDHH_4B", 6, 2000.0, {"cms": 1}, 0x48454748, 1 << 21),
    "gg_4g": ("GG_4G", 4, 1000.0, {}, 0x48454747, 1 << 20),        # 120 trace flows, MFMA colour form
    "gg_4g_ddm": ("GG_4G", 4, 1000.0, {}, 0x48454747, 1 << 20),    # 24 DDM flows, VALU colour form
    # 120 trace flows, colour form compressed to its distinct factors: FP32 on VALU, FP64 on MFMA
    "gg_4g_cf": ("GG_4G", 4, 1000.0, {}, 0x48454747, 1 << 20),
}
CUT = {"gg_4g": (20.0, 0.4), "gg_4g_ddm": (20.0, 0.4), "gg_4g_cf": (20.0, 0.4)}   # generation cut: failing events have |M|^2 = 0


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def to_soa(torch, mom):
    """oracle layout [n][legs][4] -> device SoA [legs][4][n]"""
    return torch.from_numpy(np.ascontiguousarray(np.transpose(mom, (1, 2, 0)))).cuda()


def to_aos(t):
    return np.ascontiguousarray(np.transpose(t.cpu().numpy(), (2, 0, 1)))


def make(name, precision="fp64"):
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    return H.Process(processes.by_name(name), precision=precision)


def oracle_me2(oracle, name, mom, cut=True, extended=False):
    pid, _, _, kw, _, _ = CASES[name]
    f = oracle.me2(getattr(oracle, pid), mom, oracle.params(**kw), extended=extended)
    if cut and name in CUT:
        f = f * oracle.cut_gluons(mom, *CUT[name])
    return f


def rel_err(a, b):
    return np.abs(a - b) / np.abs(b)


def random_rotation(mom, seed):
    """rotate every three-momentum by one random rotation (unit quaternion)"""
    a, b, c, d = (lambda q: q / np.linalg.norm(q))(np.random.default_rng(seed).normal(size=4))
    R = np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                  [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                  [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])
    out = mom.copy()
    out[..., 1:] = mom[..., 1:] @ R.T
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_generated_momenta_match_oracle(torch, oracle, name):
    _, nout, rs, _, seed, _ = CASES[name]
    p = make(name)
    n = 1000
    me2, mom = p.eval(n=n, seed=seed, counter_offset=7, sqrt_s=rs, want_momenta=True)
    torch.cuda.synchronize()
    got = to_aos(mom)
    ref = oracle.generate(seed, n, nout, rs, counter_offset=7)
    # RAMBO's conformal boost amplifies rounding when the seed vectors are nearly
    # collinear (n = 2); elsewhere the momenta agree to a few ulp
    tol = 1e-10 if nout == 2 else 1e-13
    assert np.max(np.abs(got - ref)) < tol * rs


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_parity_momenta_in(torch, oracle, name):
    """the parity events (several blocks and a ragged tail), momenta in: every
    event within the process's bound of the extended-precision oracle"""
    mom = B.rambo_events(oracle, name)
    p = make(name)
    got = p.eval(momenta=to_soa(torch, mom)).cpu().numpy()
    B.check(oracle, name, mom, got)


# The mixed-precision 120-flow MFMA colour form faulted on the GPU in a variant
# that staged its FP32 colour fragments in LDS; that variant is taken out and,
# its cause not yet shown, the case stays off the GPU for now.
MIXED_MFMA_OFF = "mixed gg_4g (FP32 MFMA colour form) kept off the GPU until a GPU fault's cause is shown"


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_error_report(torch, oracle, name):
    if name == "gg_4g":
        pytest.skip(MIXED_MFMA_OFF)
    _, nout, rs, _, seed, _ = CASES[name]
    n = 2048
    mom = oracle.generate(seed ^ 0x66, n, nout, rs)
    ref = oracle_me2(oracle, name, mom, extended=True)
    p = make(name, "mixed")
    got = p.eval(momenta=to_soa(torch, mom)).cpu().numpy()
    nz = ref != 0
    assert np.all(got[~nz] == 0.0)
    err = rel_err(got[nz], ref[nz])
    print(f"{name} mixed: max rel err {err.max():.3e}, median {np.median(err):.3e}")
    assert np.all(np.isfinite(got))
    assert err.max() < 1e-2


@pytest.mark.parametrize("name", list(CASES))
def test_full_size_sampled(torch, oracle, name):
    """Full workload size in seed mode (the benchmark's launch), checked on
    sampled events: their momenta against the oracle's generator and their
    |M|^2 against the oracle evaluated on those momenta."""
    _, nout, rs, _, seed, N = CASES[name]
    p = make(name)
    me2, mom = p.eval(n=N, seed=seed, sqrt_s=rs, want_momenta=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([[0, 255, 256, N - 1], rng.integers(0, N, 200)]))
    sel = torch.from_numpy(idx).cuda()
    got_mom = to_aos(mom[:, :, sel].contiguous())
    got_me2 = me2[sel].cpu().numpy()
    for k, i in enumerate(idx[:20]):
        ref = oracle.generate(seed, 1, nout, rs, counter_offset=int(i))[0]
        assert np.max(np.abs(got_mom[k] - ref)) < (1e-10 if nout == 2 else 1e-13) * rs
    B.check(oracle, name, got_mom, got_me2, share=0.95)


@pytest.mark.parametrize("name", list(CASES))
def test_integrate_matches_oracle(torch, oracle, name):
    """sigma against the oracle's on the same events, F in extended precision:
    with every weight >= 0, sigma's relative error is at most the largest
    per-event one, so the per-event bound holds for it"""
    pid, nout, rs, kw, seed, _ = CASES[name]
    n = 1 << 13
    p = make(name)
    r = p.integrate(n, seed=seed, sqrt_s=rs)
    mom = oracle.generate(seed, n, nout, rs)
    f = oracle_me2(oracle, name, mom, extended=True)
    proc = p.ir
    sig, err, sw, sw2 = oracle.cross_section(f, oracle.phase_space_volume(rs, nout), rs, proc.n_a_n_b,
                                             proc.symmetry)
    assert r["n_generated"] == n and r["n_accepted"] == int(np.sum(f != 0))
    tol = B.BOUND[name]
    print(f"{name} sigma: rel diff {r['sigma_gev2'] / sig - 1:.2e} (bound {tol:.0e})")
    assert abs(r["sigma_gev2"] / sig - 1) <= tol
    if name != "gg_4g":   # mixed: see MIXED_MFMA_OFF
        rm = make(name, "mixed").integrate(n, seed=seed, sqrt_s=rs)
        print(f"{name} mixed sigma: rel diff {rm['sigma_gev2'] / sig - 1:.2e}")
        assert rm["n_accepted"] == r["n_accepted"]
        assert abs(rm["sigma_gev2"] / sig - 1) < 1e-4
    assert abs(r["err_gev2"] / err - 1) <= 1e-9
    assert abs(r["sigma_pb"] / (sig * oracle.HBARC2_PB) - 1) <= tol


@pytest.mark.parametrize("name,expect", [("ee_mumu", 4), ("gg_ttbar_6f", 4), ("ud_udhh_4b", 24)])
def test_helicity_filter_keeps_result(torch, oracle, name, expect):
    _, nout, rs, _, seed, _ = CASES[name]
    mom = to_soa(torch, oracle.generate(seed ^ 0x77, 1500, nout, rs))
    p = make(name)
    full = p.eval(momenta=mom).cpu().numpy()
    kept = p.filter_helicities(n_probe=64, seed=99, sqrt_s=rs, rel_threshold=1e-20)
    assert kept == expect == p.n_helicities
    filt = p.eval(momenta=mom).cpu().numpy()
    assert rel_err(filt, full).max() <= 1e-13


@pytest.mark.parametrize("leg", range(6))
def test_gluon_ward_identity_on_gpu(torch, oracle, leg):
    """g g -> g g g g: replacing one gluon's polarisation by k/k^0 (helicity
    code 4) makes every colour-ordered amplitude vanish; |M|^2 drops to the
    rounding level of the physical |M|^2."""
    import itertools
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    proc = processes.by_name("gg_4g")
    hels = [tuple(4 if k == leg else h[k - (k > leg)] for k in range(6))
            for h in itertools.product((-1, 1), repeat=5)]
    mom = oracle.generate(0x57A4D, 512, 4, 1000.0)
    t = to_soa(torch, mom)
    full = H.Process(proc).eval(momenta=t).cpu().numpy()
    gauge = H.Process(proc, helicities=hels).eval(momenta=t).cpu().numpy()
    nz = full > 0
    assert nz.sum() > 100
    ratio = np.sqrt(gauge[nz] / full[nz])
    print(f"leg {leg}: max amplitude ratio {ratio.max():.2e}")
    assert ratio.max() < 1e-12


def test_edge_cases(torch, oracle):
    import paper_1305_0708_amd as H
    p = make("gg_ttbar_6f")
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    assert p.eval(n=0, me2_out=empty).numel() == 0
    for n in (1, 63, 65, 257):
        mom = oracle.generate(5, n, 6, 1000.0)
        got = p.eval(momenta=to_soa(torch, mom)).cpu().numpy()
        B.check(oracle, "gg_ttbar_6f", mom, got, share=0.0)
    with pytest.raises(H.HegetError) as e:
        p.eval(n=-1)
    assert e.value.status == -1
    with pytest.raises(H.HegetError):
        p.eval(n=10, sqrt_s=0.0)
    with pytest.raises(H.HegetError):
        p.integrate(1)


def test_bitwise_deterministic(torch):
    p = make("ud_udhh_4b")
    a = p.eval(n=5000, seed=3, sqrt_s=2000.0)
    b = p.eval(n=5000, seed=3, sqrt_s=2000.0)
    assert torch.equal(a, b)
    r1 = p.integrate(4096, seed=1)
    r2 = p.integrate(4096, seed=1)
    assert r1 == r2


def test_c0_closed_form_on_gpu(torch):
    """e+e- -> mu+mu-: the GPU result equals the analytic helicity-amplitude
    formula on exactly massless 2 -> 2 momenta."""
    from test_oracle_amplitudes import ee_closed_form, two_to_two_massive
    rng = np.random.default_rng(3)
    mom = np.array([two_to_two_massive(200.0, 0.0, c, ph)
                    for c, ph in zip(rng.uniform(-1, 1, 500), rng.uniform(0, 2 * math.pi, 500))])
    got = make("ee_mumu").eval(momenta=to_soa(torch, mom)).cpu().numpy()
    cf = np.array([ee_closed_form(m) for m in mom])
    assert rel_err(got, cf).max() < 1e-13


def test_colour_bases_agree(torch, oracle):
    """The 120-flow trace basis and the 24-flow DDM basis on VALU give the same
    |M|^2 (the colour sum is basis independent): in FP64 with the trace basis's
    dense form on MFMA, and, within the mixed path's precision, in FP32 with its
    form compressed to the distinct colour factors on VALU."""
    mom = oracle.generate(0xC0105, 2000, 4, 1000.0)
    t = to_soa(torch, mom)
    for prec, name, tol in (("fp64", "gg_4g", 1e-12), ("mixed", "gg_4g_cf", 1e-4)):   # mixed gg_4g: MIXED_MFMA_OFF
        a = make(name, prec).eval(momenta=t).cpu().numpy()
        b = make("gg_4g_ddm", prec).eval(momenta=t).cpu().numpy()
        assert np.array_equal(a == 0, b == 0)
        nz = b != 0
        err = rel_err(a[nz], b[nz])
        print(f"{prec}: trace basis ({name}) vs DDM basis max rel diff {err.max():.3e}, median {np.median(err):.3e}")
        assert err.max() < tol


@pytest.mark.parametrize("name", ["ee_mumu", "gg_ttbar_6f", "gg_4g"])
def test_generate_alone_matches_eval_and_oracle(torch, oracle, name):
    """heget_generate writes exactly the momenta heget_eval generates."""
    _, nout, rs, _, seed, _ = CASES[name]
    p = make(name)
    n = 3 * 1024 + 37
    mom = p.generate(n, seed=seed, counter_offset=11, sqrt_s=rs)
    _, ref_dev = p.eval(n=n, seed=seed, counter_offset=11, sqrt_s=rs, want_momenta=True)
    torch.cuda.synchronize()
    assert torch.equal(mom, ref_dev)
    ref = oracle.generate(seed, n, nout, rs, counter_offset=11)
    assert np.max(np.abs(to_aos(mom) - ref)) < (1e-10 if nout == 2 else 1e-13) * rs
    assert p.generate(0, seed=seed).numel() == 0


@pytest.mark.parametrize("name", ["ee_mumu", "gg_ttbar_6f", "ud_udhh_4b"])
def test_helicity_table_path_matches_nest(torch, oracle, name):
    """The full helicity product runs as the loop nest; the same rows in
    another order run the per-row table loop.  Both match the oracle and each
    other."""
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    _, nout, rs, _, seed, _ = CASES[name]
    proc = processes.by_name(name)
    mom = oracle.generate(seed ^ 0x99, 1500, nout, rs)
    t = to_soa(torch, mom)
    nest = H.Process(proc).eval(momenta=t).cpu().numpy()
    table = H.Process(proc, helicities=list(proc.helicities)[::-1]).eval(momenta=t).cpu().numpy()
    ref = B.reference(oracle, name, mom)
    B.check(oracle, name, mom, table, ref=ref)
    B.check(oracle, name, mom, nest, ref=ref)
    err = rel_err(nest, table)
    print(f"{name}: nest vs table max rel diff {err.max():.2e}")
    assert np.median(err) < 1e-14


def _boost(mom, beta):
    """Lorentz boost of every momentum by velocity beta (3-vector, |beta| < 1)"""
    b = np.asarray(beta, dtype=float)
    b2 = b @ b
    g = 1.0 / math.sqrt(1.0 - b2)
    E, p = mom[..., 0], mom[..., 1:]
    bp = p @ b
    out = mom.copy()
    out[..., 0] = g * (E + bp)
    out[..., 1:] = p + (((g - 1.0) * bp / b2 + g * E)[..., None]) * b
    return out


@pytest.mark.parametrize("name,general", [("ud_udhh_4b", True), ("gg_4g", False), ("ee_mumu", True)])
def test_lorentz_invariance_on_gpu(torch, oracle, name, general):
    """|M|^2 is a Lorentz scalar: the GPU result on boosted and rotated events
    equals the GPU result on the originals.  gg -> gggg is boosted along the
    beam and rotated about it only, which keeps its generation cut
    (pT, Delta R) unchanged."""
    _, nout, rs, _, seed, _ = CASES[name]
    mom = oracle.generate(seed ^ 0xB005, 1024, nout, rs)
    rng = np.random.default_rng(17)
    if general:
        beta = rng.normal(size=3)
        beta *= 0.9 / np.linalg.norm(beta)
        moved = random_rotation(_boost(mom, beta), 4)
    else:
        moved = _boost(mom, [0.0, 0.0, 0.7])
        phi = 0.83
        R = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
        moved[..., 1:3] = moved[..., 1:3] @ R.T
    p = make(name)
    a = p.eval(momenta=to_soa(torch, mom)).cpu().numpy()
    b = p.eval(momenta=to_soa(torch, moved)).cpu().numpy()
    assert np.array_equal(a == 0, b == 0)
    nz = a != 0
    assert nz.sum() > 500
    err = rel_err(b[nz], a[nz])
    print(f"{name}: frame change max rel diff {err.max():.2e}, median {np.median(err):.2e}")
    # the boost amplifies rounding (energies grow up to x4.4 at beta = 0.9); the gauge
    # cancellations of ud -> udhh -> 4b leave a frame-dependent FP64 rounding of about
    # 1e-12 per event (the oracle spreads as much under the same frame change)
    med, worst = (1e-11, 1e-9) if name == "ud_udhh_4b" else (1e-13, 1e-11)
    assert np.median(err) < med
    assert err.max() < worst


def test_bose_symmetry_on_gpu(torch, oracle):
    """gg -> gggg: exchanging final-state gluons leaves |M|^2 unchanged."""
    _, nout, rs, _, seed, _ = CASES["gg_4g"]
    mom = oracle.generate(seed ^ 0xB05E, 1024, nout, rs)
    perm = mom[:, [0, 1, 4, 2, 5, 3], :]
    p = make("gg_4g")
    a = p.eval(momenta=to_soa(torch, mom)).cpu().numpy()
    b = p.eval(momenta=to_soa(torch, np.ascontiguousarray(perm))).cpu().numpy()
    assert np.array_equal(a == 0, b == 0)
    nz = a != 0
    assert rel_err(b[nz], a[nz]).max() < 1e-12
