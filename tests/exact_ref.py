"""Exact-rational brute-force k-means used to pin the oracle.

This module is written independently of the oracle: it never prunes, never
sorts center distances and computes in ``fractions.Fraction``.  It is plain
batch k-means (Alg. 1) on a weighted point set, with the tie key
(dist, k != previous, k) and the Sec. 3.2 stopping rule, which is what the
weighted sort-means loop (Alg. 2) must reproduce exactly.
"""

from __future__ import annotations

from fractions import Fraction


def sqd(x, c):
    return sum((Fraction(a) - Fraction(b)) ** 2 for a, b in zip(x, c))


def nearest(x, centers, prev):
    """argmin over k of (||x-c_k||^2, k != prev, k); returns (k, dist)."""
    best = None
    for k, c in enumerate(centers):
        key = (sqd(x, c), k != prev, k)
        if best is None or key < best:
            best = key
    return best[2], best[0]


def lloyd(points, weights, init, max_iters, eps, m0=None):
    """Exact weighted Lloyd iterations.

    points: list of integer 3-tuples; weights: positive integers;
    init: list of 3-tuples (int/Fraction).  Returns a list of per-iteration
    records dict(m, sse, centers) and the converged flag."""
    n = len(points)
    W = sum(weights)
    centers = [tuple(Fraction(v) for v in c) for c in init]
    m = list(m0) if m0 is not None else [0] * n
    eps_q = Fraction(eps)
    hist = []
    prev_sse = None
    converged = False
    for t in range(1, max_iters + 1):
        dists = []
        for i in range(n):
            k, d = nearest(points[i], centers, m[i])
            m[i] = k
            dists.append(d)
        sse = sum(Fraction(w) * d for w, d in zip(weights, dists)) / W
        new = []
        for k, c in enumerate(centers):
            wk = sum(weights[i] for i in range(n) if m[i] == k)
            if wk == 0:
                new.append(c)
            else:
                new.append(tuple(
                    sum(Fraction(weights[i]) * points[i][ch] for i in range(n) if m[i] == k) / wk
                    for ch in range(3)))
        centers = new
        hist.append(dict(m=list(m), sse=sse, centers=[tuple(c) for c in centers]))
        if sse == 0 or (t >= 2 and (prev_sse - sse) / sse <= eps_q):
            converged = True
            break
        prev_sse = sse
    return hist, converged
