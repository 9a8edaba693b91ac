"""GPU parity of u ubar -> t tbar + 1, 2, 3 gluons against the oracle's sum
over Feynman diagrams with explicit SU(3) colour.

The kernels are generated from diagram call lists: 5, 38 and 393 diagrams, 4,
12 and 48 colour flows; from two gluons on, the helicity rows one at a time
and the program divided into device functions (Sec. 5.3); uu_ttggg_cf the
same with the colour form compressed to its distinct factors (Sec. 5.4).
Checked: |M|^2 on the oracle's events (every event passing the cut within
1e-12 of the extended-precision oracle, events failing it exactly 0), the
mixed-precision error, the flat-tree momenta and weights generated from the
seed, the cross section, and the two colour forms against each other."""
import math

import numpy as np
import pytest

import fp64_bounds as B

pytestmark = pytest.mark.gpu

ROOTS = 1000.0
MT = 175.0
NG = {"uu_ttg": 1, "uu_ttgg": 2, "uu_ttggg": 3, "uu_ttggg_cf": 3}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def procs(torch):
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    return {(n, p): H.Process(processes.by_name(n), precision=p) for n in NG for p in ("fp64", "mixed")}


def to_aos(t):
    return np.ascontiguousarray(np.transpose(t.cpu().numpy(), (2, 0, 1)))


def to_soa(torch, mom):
    return torch.from_numpy(np.ascontiguousarray(np.transpose(mom, (1, 2, 0)))).cuda()


@pytest.mark.parametrize("name", list(NG))
def test_me2_matches_oracle(torch, oracle, procs, name):
    """momenta in: the oracle's events (a few 256-lane blocks and a ragged tail)"""
    for mom in B.tree_events(oracle, name):
        print(f"{name}: {len(mom)} events", flush=True)
        me2 = procs[(name, "fp64")].eval(momenta=to_soa(torch, mom)).cpu().numpy()
        B.check(oracle, name, mom, me2)


@pytest.mark.parametrize("name", list(NG))
def test_mixed_precision_error(torch, oracle, procs, name):
    """mixed precision (FP32 wavefunctions and colour form, FP64 momenta,
    denominators and |M|^2 sum): the error against the oracle is reported"""
    for mom in B.tree_events(oracle, name):
        me2 = procs[(name, "mixed")].eval(momenta=to_soa(torch, mom)).cpu().numpy()
        ref = B.reference(oracle, name, mom, extended=False)
        nz = ref != 0
        assert np.all(me2[~nz] == 0.0)
        err = np.abs(me2[nz] - ref[nz]) / ref[nz]
        print(f"{name} mixed: max rel err {err.max():.2e}, median {np.median(err):.2e} ({nz.sum()} events)")
        assert np.median(err) < 1e-5 and err.max() < 1e-3


def test_compressed_equals_dense(torch, oracle, procs):
    """the same flows through the dense and the compressed colour form"""
    mom = B.tree_events(oracle, "uu_ttggg")[0]
    t = to_soa(torch, mom)
    a = procs[("uu_ttggg", "fp64")].eval(momenta=t).cpu().numpy()
    b = procs[("uu_ttggg_cf", "fp64")].eval(momenta=t).cpu().numpy()
    nz = a != 0
    assert np.array_equal(nz, b != 0)
    assert np.max(np.abs(b[nz] / a[nz] - 1)) < 1e-13


@pytest.mark.parametrize("name,n,offset", [("uu_ttg", 1000, 0), ("uu_ttggg", 300, 77)])
def test_momenta_and_weights_match_oracle(torch, oracle, procs, name, n, offset):
    from oracle import phase_space_tree as T
    ng = NG[name]
    mom, w = procs[(name, "fp64")].generate(n, seed=0x5454, counter_offset=offset, sqrt_s=ROOTS, want_weights=True)
    torch.cuda.synchronize()
    ref_mom, ref_w = T.generate(0x5454, n, ROOTS, B._tt_gluons_tree(ng), 4 + ng, counter_offset=offset,
                                leg_mass=[0, 0, MT, MT] + [0] * ng)
    got = to_aos(mom)
    assert np.abs(got - ref_mom).max() < 1e-12 * ROOTS
    ok = ref_w > 0
    assert np.array_equal(w.cpu().numpy() > 0, ok)
    assert np.abs(w.cpu().numpy()[ok] / ref_w[ok] - 1).max() < 1e-12


@pytest.mark.parametrize("name,n", [("uu_ttgg", 2048), ("uu_ttggg", 512)])
def test_integrate_matches_oracle(torch, oracle, procs, name, n):
    """sigma over n generated events: the flat tree's weight, the cut, the
    1/4 spin and 1/9 colour averages and the 1/n_g! symmetry factor"""
    from oracle import phase_space_tree as T
    ng = NG[name]
    proc = procs[(name, "fp64")]
    r = proc.integrate(n, seed=0x5455, sqrt_s=ROOTS)
    mom, w = T.generate(0x5455, n, ROOTS, B._tt_gluons_tree(ng), 4 + ng, leg_mass=[0, 0, MT, MT] + [0] * ng)
    f = B.reference(oracle, name, mom, extended=False)
    sig, err, _, _ = oracle.cross_section(f, w, ROOTS, proc.ir.n_a_n_b, proc.ir.symmetry)
    print(f"{name} sigma: GPU {r['sigma_pb']:.6e} pb, rel to oracle {r['sigma_gev2'] / sig - 1:.2e}")
    assert r["n_accepted"] == int(np.count_nonzero(f))
    assert abs(r["sigma_gev2"] / sig - 1) <= 1e-12
    assert abs(r["err_gev2"] / err - 1) <= 1e-9
