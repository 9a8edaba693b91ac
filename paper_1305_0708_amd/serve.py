"""Synthetic request streams and their replay against the serving engine.

The serving workload: a Poisson stream of cross-section requests over several
resident processes, each request with its own event count (log-uniform),
Philox seed and sqrt(s_hat) (the process's nominal value times 2^U(-1/2, 1/2)).
`replay_engine` submits each request at its arrival time to a `Server` and
collects submit-to-completion latencies measured by the engine;
`replay_unbatched` serves the same stream one request at a time with plain
heget_integrate calls in arrival order, the reference point for batching.
"""
import hashlib
import math
import struct
import time
from dataclasses import dataclass

import numpy as np


@dataclass
class Request:
    t_arrival: float   # seconds after the start of the stream
    process: int       # index into the server's process list
    n: int
    seed: int
    sqrt_s: float


def request_seed(stream_seed, k):
    """Philox key of request k: the first 8 bytes of SHA-256(stream seed, k)."""
    return struct.unpack("<Q", hashlib.sha256(struct.pack("<QQ", stream_seed, k)).digest()[:8])[0]


def poisson_mix(seed, n_requests, rate, weights, nominal_sqrt_s, n_min=1 << 10, n_max=1 << 20):
    """n_requests arrivals at `rate` per second; process k drawn with
    probability weights[k]; n = floor(exp(U(ln n_min, ln n_max)))."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=float)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    procs = rng.choice(len(w), size=n_requests, p=w / w.sum())
    ns = np.floor(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_requests))).astype(np.int64)
    scale = 2.0 ** rng.uniform(-0.5, 0.5, size=n_requests)
    return [Request(float(t[k]), int(procs[k]), int(ns[k]), request_seed(seed, k),
                    float(nominal_sqrt_s[procs[k]] * scale[k])) for k in range(n_requests)]


def _sleep_until(t):
    while True:
        dt = t - time.perf_counter()
        if dt <= 0:
            return
        time.sleep(min(dt, 0.001) if dt < 0.002 else dt - 0.001)


def summary(lat, events, wall):
    lat = np.asarray(lat)
    return {"requests": int(len(lat)), "events": int(events), "wall_s": wall, "events_per_s": events / wall,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean())}


def replay_engine(server, requests):
    """Submit every request at its arrival time; latency = the engine's
    submit-to-completion time of the request."""
    t0 = time.perf_counter()
    tickets = []
    for r in requests:
        _sleep_until(t0 + r.t_arrival)
        tickets.append(server.submit(r.process, r.n, r.seed, r.sqrt_s))
    results, lat = [], []
    for t in tickets:
        res, l = server.poll(t)[:2]
        results.append(res)
        lat.append(l)
    wall = time.perf_counter() - t0
    return results, summary(lat, sum(r.n for r in requests), wall)


def replay_unbatched(handles, requests):
    """One request at a time in arrival order (heget_integrate on
    handles[process]); latency = completion time - arrival time."""
    t0 = time.perf_counter()
    results, lat = [], []
    for r in requests:
        _sleep_until(t0 + r.t_arrival)
        res = handles[r.process].integrate(r.n, seed=r.seed, sqrt_s=r.sqrt_s)
        lat.append(time.perf_counter() - t0 - r.t_arrival)
        results.append(res)
    wall = time.perf_counter() - t0
    return results, summary(lat, sum(r.n for r in requests), wall)
