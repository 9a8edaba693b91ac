"""Oracle (test infrastructure only): adaptive importance sampling of the
phase-space uniforms in the manner of VEGAS (G. P. Lepage, J. Comput. Phys. 27
(1978) 192) -- the role the BASES integrator plays in the paper's integrations
(gBASES, Sec. 1 and Sec. 6).

Each uniform dimension d has a grid of B bins with edges 0 = e_0 < ... < e_B = 1.
A uniform r goes to bin j = floor(r B) and to x = e_j + (r B - j)(e_(j+1) - e_j);
the event's weight takes the Jacobian prod_d B (e_(j+1) - e_j).  After each
iteration the grid is refined from d_j = sum over the iteration's events in bin
j of w^2 (w the full event weight):

  1. smoothing: (d_0 + d_1) / 2, (d_(j-1) + d_j + d_(j+1)) / 3, (d_(B-2) + d_(B-1)) / 2;
  2. compression: with x_j = d_j / sum d, r_j = ((x_j - 1) / ln x_j)^alpha (0 for x_j = 0);
  3. the new edges cut the old bins so that each new bin holds sum r / B, the
     share of an old bin growing linearly across it.

Iteration k draws its uniforms from counters k N .. (k + 1) N - 1.  The
iterations combine with inverse-variance weights.  Written with numpy; no code
shared with the library.
"""
import math

import numpy as np

from . import uniforms_bulk

ALPHA = 1.5


def uniform_grid(D, B):
    return np.tile(np.arange(B + 1) / B, (D, 1))


def map_uniforms(r, edges):
    """r [n][D] -> (x [n][D], Jacobian [n], bins [n][D])"""
    B = edges.shape[1] - 1
    j = np.minimum((r * B).astype(np.int64), B - 1)
    D = r.shape[1]
    lo = np.take_along_axis(np.broadcast_to(edges[None, :, :], (r.shape[0], D, B + 1)), j[:, :, None], 2)[:, :, 0]
    hi = np.take_along_axis(np.broadcast_to(edges[None, :, :], (r.shape[0], D, B + 1)), j[:, :, None] + 1, 2)[:, :, 0]
    x = lo + (r * B - j) * (hi - lo)
    jac = np.prod(B * (hi - lo), axis=1)
    return x, jac, j


def histogram(bins, w, B):
    """d[D][B] = sum of w^2 over the events in each bin of each dimension (exact sums)"""
    D = bins.shape[1]
    d = np.zeros((D, B))
    w2 = w * w
    for k in range(D):
        for b in range(B):
            d[k, b] = math.fsum(w2[bins[:, k] == b].tolist())
    return d


def refine(edges, d, alpha=ALPHA):
    """one VEGAS refinement of every dimension's edges from its bin sums d"""
    D, B1 = edges.shape
    B = B1 - 1
    out = edges.copy()
    for k in range(D):
        e, dk = edges[k], d[k]
        sm = np.empty(B)
        sm[0] = (dk[0] + dk[1]) / 2.0
        sm[-1] = (dk[-2] + dk[-1]) / 2.0
        for j in range(1, B - 1):
            sm[j] = (dk[j - 1] + dk[j] + dk[j + 1]) / 3.0
        S = sum(sm)
        if not S > 0:
            continue
        r = np.zeros(B)
        for j in range(B):
            x = sm[j] / S
            if x <= 0.0:
                r[j] = 0.0
            elif x >= 1.0:
                r[j] = 1.0
            else:
                r[j] = ((x - 1.0) / math.log(x)) ** alpha
        R = sum(r) / B
        new = [0.0]
        acc, j = 0.0, 0
        for m in range(1, B):
            target = m * R
            while j < B - 1 and acc + r[j] < target:
                acc += r[j]
                j += 1
            new.append(e[j] + (target - acc) / r[j] * (e[j + 1] - e[j]) if r[j] > 0 else e[j])
        new.append(1.0)
        out[k] = new
    return out


def combine(sigmas, errs):
    """inverse-variance average of the iterations: (sigma, err, chi^2 per degree of freedom)"""
    s = np.asarray(sigmas, dtype=np.float64)
    v = np.asarray(errs, dtype=np.float64) ** 2
    wv = 1.0 / v
    mean = float(np.sum(wv * s) / np.sum(wv))
    err = float(1.0 / math.sqrt(np.sum(wv)))
    chi2 = float(np.sum((s - mean) ** 2 / v) / max(len(s) - 1, 1))
    return mean, err, chi2


def integrate(f, seed, n, iterations, D, B, alpha=ALPHA):
    """f(x [n][D]) -> integrand values [n] (the event weight before the grid's
    Jacobian).  Returns the per-iteration (sigma, err), the combination and
    the final grid."""
    edges = uniform_grid(D, B)
    per = []
    for it in range(iterations):
        r = uniforms_bulk(seed, n, D, counter_offset=it * n)
        x, jac, bins = map_uniforms(r, edges)
        w = f(x) * jac
        sw, sw2 = math.fsum(w.tolist()), math.fsum((w * w).tolist())
        sig = sw / n
        err = math.sqrt(max(sw2 / n - sig * sig, 0.0) / (n - 1))
        per.append((sig, err))
        edges = refine(edges, histogram(bins, w, B), alpha)
    return per, combine([p[0] for p in per], [p[1] for p in per]), edges
