"""heget_integrate_async against heget_integrate: the same sums bit for bit,
for steps queued back to back on one stream with no wait between them, the
partials buffer grown in the middle of the queue and a smaller step after it."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,prec", [("gg_ttbar_6f", "fp64"), ("gg_ttbar_6f", "mixed"), ("ud_udhh_4b", "fp64")])
def test_queued_steps_equal_synchronous_ones(name, prec):
    import torch
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    print(f"integrate_async {name} {prec}", flush=True)
    p = H.Process(processes.by_name(name), precision=prec)
    steps = [(5000, 11), (5000, 12), (70001, 13), (300, 14), (70001, 15)]
    sums = torch.full((len(steps), 3), float("nan"), dtype=torch.float64, device="cuda")
    for k, (n, seed) in enumerate(steps):
        p.integrate_async(n, sums[k], seed=seed)
    torch.cuda.synchronize()
    got = sums.cpu().tolist()
    for k, (n, seed) in enumerate(steps):
        ref = p.integrate(n, seed=seed)
        assert got[k] == [ref["sum_w"], ref["sum_w2"], float(ref["n_accepted"])], (k, n, seed)
        assert p.result_from_sums(got[k], n) == ref
