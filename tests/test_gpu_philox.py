"""The counter-based random numbers on the GPU against the oracle's Philox:
bit for bit (integer work: the uniforms are exact functions of the Philox
words), across counter words, seed words and draw blocks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.mark.parametrize("seed,offset,n,n_u", [
    (0x48454746, 0, 3 * 256 + 17, 24),            # C1's seed, 12 draw blocks, ragged tail
    (0x48454747, (1 << 32) - 5, 300, 16),         # the counter's low word wraps into the high word
    (0xFEDCBA9876543210, 12345, 1000, 7),         # both key words, an odd number of draws
    (0, 0, 1, 1),
])
def test_uniforms_bitwise(torch, oracle, seed, offset, n, n_u):
    import paper_1305_0708_amd as H
    got = H.uniforms(n, n_u, seed=seed, counter_offset=offset).cpu().numpy().T
    ref = oracle.uniforms_bulk(seed, n, n_u, counter_offset=offset)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_uniforms_feed_rambo(torch, oracle):
    """the uniforms heget_eval's RAMBO draws: the oracle's RAMBO on the
    device's uniforms gives the device's momenta"""
    import paper_1305_0708_amd as H
    from paper_1305_0708_amd import processes
    n = 64
    u = H.uniforms(n, 16, seed=7, counter_offset=3).cpu().numpy().T
    p = H.Process(processes.by_name("gg_4g"))
    _, mom = p.eval(n=n, seed=7, counter_offset=3, sqrt_s=1000.0, want_momenta=True)
    mom = np.transpose(mom.cpu().numpy(), (2, 0, 1))
    for i in range(n):
        q, _ = oracle.rambo(1000.0, u[i])
        assert np.max(np.abs(q - mom[i, 2:])) < 1e-12 * 1000.0


def test_uniforms_edge_cases(torch):
    import paper_1305_0708_amd as H
    assert H.uniforms(0, 4).numel() == 0
    with pytest.raises(H.HegetError):
        H.uniforms(-1, 4)
    with pytest.raises(H.HegetError):
        H.uniforms(10, 0)
