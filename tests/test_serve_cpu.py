"""Host-side checks of the synthetic serving workload (no GPU)."""
import math

import numpy as np

from paper_1305_0708_amd import serve


def test_poisson_mix_shape_and_determinism():
    nominal = [200.0, 1000.0, 1000.0, 2000.0]
    a = serve.poisson_mix(0x48454749, 4000, 200.0, [40, 30, 20, 10], nominal)
    b = serve.poisson_mix(0x48454749, 4000, 200.0, [40, 30, 20, 10], nominal)
    assert a == b
    t = np.array([r.t_arrival for r in a])
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 4000 - 1 / 200.0) < 0.1 / 200.0          # mean gap 5 ms
    frac = np.bincount([r.process for r in a], minlength=4) / 4000
    assert np.allclose(frac, [0.4, 0.3, 0.2, 0.1], atol=0.03)
    n = np.array([r.n for r in a])
    assert n.min() >= 1024 and n.max() < 1 << 20
    # log-uniform: ln n is flat on [ln 2^10, ln 2^20)
    u = (np.log(n + 0.5) - math.log(1024)) / math.log(1024)
    assert abs(u.mean() - 0.5) < 0.02
    for r in a:
        ratio = r.sqrt_s / nominal[r.process]
        assert 2 ** -0.5 <= ratio <= 2 ** 0.5
    assert len({r.seed for r in a}) == 4000


def test_request_seed_is_stable():
    assert serve.request_seed(1, 0) == serve.request_seed(1, 0)
    assert serve.request_seed(1, 0) != serve.request_seed(1, 1)
    assert serve.request_seed(1, 0) != serve.request_seed(2, 0)
