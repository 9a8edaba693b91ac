"""heget_integrate_noalloc against heget_integrate through the C ABI: the same
kernels, counters and reduction order, so the same bits, on two calls in a
row with the second smaller; sizes above the scratch's limit are refused; the
call leaves the device's free memory unchanged."""
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("sigma_gev2", "err_gev2", "sigma_pb", "err_pb", "sum_w", "sum_w2", "n_generated", "n_accepted")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.mark.parametrize("name,n1,n2", [
    ("gg_ttbar_6f", 1 << 20, 4099),     # one block per 256 events
    ("gg_4g", 70000, 301),              # persistent grid with a workspace slot per block
    ("ee_mumu", 65536, 2),
])
def test_noalloc_matches_integrate(torch, name, n1, n2):
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    p = H.Process(processes.by_name(name))
    for n, seed in ((n1, 0x1234), (n2, 0x5678)):
        print(f"no-alloc {name} n={n}", flush=True)
        ref = p.integrate(n, seed=seed)
        got = p.integrate_noalloc(n, seed=seed)
        torch.cuda.synchronize()
        for k in FIELDS:
            assert got[k] == ref[k], (name, n, k, got[k], ref[k])
    p.close()


def test_noalloc_allocates_nothing_and_refuses_oversize(torch):
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes, _lib
    p = H.Process(processes.gg_ttbar_6f())
    p.integrate_noalloc(1 << 16, seed=1)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    r1 = p.integrate_noalloc(1 << 18, seed=2)
    r2 = p.integrate_noalloc(1 << 12, seed=3)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    assert r1["n_generated"] == 1 << 18 and r2["n_generated"] == 1 << 12
    with pytest.raises(H.HegetError) as e:
        p.integrate_noalloc(_lib.HEGET_NOALLOC_MAX_EVENTS + 1, seed=4)
    assert e.value.status == _lib.HEGET_E_INVALID and "limit" in str(e.value)
    with pytest.raises(H.HegetError):
        p.integrate_noalloc(1, seed=5)
    p.close()
