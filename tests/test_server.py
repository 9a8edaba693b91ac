"""The serving engine (heget_server_*) through the C ABI: continuous batching of
cross-section requests over resident processes.

Every request's result must be bit-identical to heget_integrate (and, when
asked for, its per-event |M|^2 to heget_eval) of that request alone on the
same process handle, whatever else is in flight; the arena bounds the device
memory of the requests in flight; same-process requests are fused into shared
launches and launches overlap on their streams.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# C2 in mixed precision runs its DDM-basis kernel here (the 120-flow FP32 MFMA
# kernel is kept off the GPU for now, see test_gpu_parity.MIXED_MFMA_OFF)
NAMES = ["ee_mumu", "gg_ttbar_6f", "gg_4g_cf", "ud_udhh_4b"]
SQRT_S = {"ee_mumu": 200.0, "gg_ttbar_6f": 1000.0, "gg_4g_cf": 1000.0, "ud_udhh_4b": 2000.0}


@pytest.fixture(scope="module")
def handles():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    hs = [H.Process(processes.by_name(n), precision="mixed") for n in NAMES]
    hs.append(H.Process(processes.by_name("gg_ttbar_6f"), precision="fp64"))
    return hs


def _requests(seed, count, nmax):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        proc = int(rng.integers(0, 5))
        name = NAMES[proc] if proc < 4 else "gg_ttbar_6f"
        n = int(np.exp(rng.uniform(np.log(300), np.log(nmax))))
        rs = SQRT_S[name] * 2.0 ** rng.uniform(-0.5, 0.5)
        out.append((proc, n, int(rng.integers(1, 2**63)), rs, bool(k % 3 == 0)))
    return out


def _alone(handles, proc, n, seed, rs):
    import torch
    p = handles[proc]
    r = p.integrate(n, seed=seed, sqrt_s=rs)
    me2 = p.eval(n=n, seed=seed, sqrt_s=rs)
    torch.cuda.synchronize()
    return r, me2.cpu().numpy()


def test_results_identical_alone_and_in_the_mix(handles):
    import paper_1305_0708_amd as H
    reqs = _requests(11, 48, 70000)
    srv = H.Server(handles, arena_bytes=64 << 20, slots_per_process=2, max_batch_blocks=512,
                   max_chunk_blocks=96)
    rng = np.random.default_rng(5)
    tickets = []
    for (proc, n, seed, rs, want) in reqs:
        tickets.append(srv.submit(proc, n, seed, rs, want_me2=want))
        time.sleep(float(rng.uniform(0, 0.002)))      # requests arrive while others run
    got = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print(st)
    assert st["requests_done"] == len(reqs)
    assert st["segments"] >= len(reqs)
    assert st["max_busy_slots"] >= 2
    for (proc, n, seed, rs, want), g in zip(reqs, got):
        ref, ref_me2 = _alone(handles, proc, n, seed, rs)
        assert g[0] == ref, (proc, n, g[0], ref)
        assert g[1] > 0
        if want:
            assert np.array_equal(g[2], ref_me2), (proc, n)


def test_fusion_of_small_requests(handles):
    """Many small requests of one process queued together share launches."""
    import paper_1305_0708_amd as H
    srv = H.Server(handles[:2], arena_bytes=16 << 20, slots_per_process=1, max_batch_blocks=4096,
                   max_chunk_blocks=1024)
    # occupy the slot with a large request so the small ones queue up behind it
    big = srv.submit(1, 1 << 20, 3, 1000.0)
    small = [srv.submit(1, 1000 + 37 * k, 100 + k, 1000.0) for k in range(40)]
    for t in [big] + small:
        srv.poll(t)
    st = srv.stats()
    srv.close()
    print(st)
    assert st["segments"] >= 41
    assert st["launches"] < 41          # several requests per fused launch


def test_admission_bounded_by_arena(handles):
    import paper_1305_0708_amd as H
    arena = 1 << 20
    srv = H.Server(handles[:2], arena_bytes=arena, slots_per_process=2, max_batch_blocks=256,
                   max_chunk_blocks=64)
    # each request keeps 8 bytes per event of |M|^2: only a few fit at once
    reqs = [(0, 40000 + 1000 * k, 7 + k, 200.0) for k in range(12)]
    tickets = [srv.submit(p, n, s, rs, want_me2=True) for (p, n, s, rs) in reqs]
    got = [srv.poll(t) for t in tickets]
    st = srv.stats()
    with pytest.raises(H.HegetError) as e:
        srv.submit(0, 200000, 1, 200.0, want_me2=True)      # 1.6 MB > arena
    assert e.value.status == -1
    srv.close()
    assert 0 < st["arena_high_water"] <= arena
    for (p, n, s, rs), g in zip(reqs, got):
        ref, ref_me2 = _alone(handles, p, n, s, rs)
        assert g[0] == ref
        assert np.array_equal(g[2], ref_me2)


def test_bad_requests(handles):
    import paper_1305_0708_amd as H
    srv = H.Server(handles[:1], arena_bytes=1 << 20)
    for args in [(1, 1000, 1, 200.0), (0, 1, 1, 200.0), (0, 1000, 1, 0.0)]:
        with pytest.raises(H.HegetError) as e:
            srv.submit(*args)
        assert e.value.status == -1
    with pytest.raises(H.HegetError):
        srv.poll(12345)
    srv.submit(0, 5000, 9, 200.0)
    srv.close()            # drains the queued request


def test_resonance_tree_process_alone_and_in_the_mix(handles):
    """a process whose events come from its resonance tree (per-event weights in
    the batch kernel) gives the same bits served as integrated alone"""
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    tree = H.Process(processes.by_name("gg_ttbar_6f_bw"), precision="fp64")
    hs = list(handles) + [tree]
    srv = H.Server(hs, arena_bytes=64 << 20, slots_per_process=2, max_batch_blocks=512, max_chunk_blocks=96)
    reqs = [(len(hs) - 1, n, 1000 + n, 1000.0 * f) for n, f in ((5000, 1.0), (777, 0.9), (40000, 1.2))]
    reqs += [(1, 3000, 7, 1000.0), (0, 2000, 9, 200.0)]
    tickets = [srv.submit(proc, n, seed, rs) for proc, n, seed, rs in reqs]
    got = [srv.poll(t) for t in tickets]
    srv.close()
    for (proc, n, seed, rs), g in zip(reqs, got):
        ref = hs[proc].integrate(n, seed=seed, sqrt_s=rs)
        assert g[0] == ref, (proc, n, g[0], ref)
