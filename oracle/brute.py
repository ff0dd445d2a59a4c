"""Brute-force second oracle for tiny constellations (test infrastructure).

Works from Bayes' rule on the Gaussian likelihoods themselves, in 60-digit
mpmath arithmetic, instead of the log-sum-exp route of ``oracle.c``:

    p(y | x_j) = (2 pi sigma^2)^(-D/2) exp(-|y - x_j|^2 / (2 sigma^2))
    P(j | y)   = p(y | x_j) / sum_i p(y | x_i)            (uniform prior)
    P(b_k = b | y) = sum_{j : bit k of label j is b} P(j | y)
    LLR_k = ln P(b_k = 0 | y) - ln P(b_k = 1 | y)
    u = -log2 P(t | y),   v = -sum_k log2 P(b_k = b_k(t) | y)

so MI = log2 M - mean(u) and GMI = m - mean(v). Pure Python loops: only for
M <= 16 and a few thousand samples.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np

mpmath.mp.dps = 60


def demap(X, labels, Y, snr_db, tx=None):
    X = np.asarray(X, dtype=np.float64)
    labels = np.asarray(labels, dtype=np.int64)
    Y = np.asarray(Y, dtype=np.float64)
    M, D = X.shape
    m = int(round(math.log2(M)))
    es = mpmath.fsum(mpmath.mpf(float(X[j, d])) ** 2 for j in range(M) for d in range(D)) / M
    sigma2 = es / (D * mpmath.power(10, mpmath.mpf(snr_db) / 10))
    norm = mpmath.power(2 * mpmath.pi * sigma2, -mpmath.mpf(D) / 2)
    N = Y.shape[0]
    llr = np.empty((N, m))
    u = np.empty(N)
    v = np.empty(N)
    for n in range(N):
        p = []
        for j in range(M):
            d2 = mpmath.fsum((mpmath.mpf(float(Y[n, d])) - mpmath.mpf(float(X[j, d]))) ** 2
                             for d in range(D))
            p.append(norm * mpmath.exp(-d2 / (2 * sigma2)))
        total = mpmath.fsum(p)
        post = [pj / total for pj in p]
        pb = [[mpmath.fsum(post[j] for j in range(M) if ((labels[j] >> k) & 1) == b)
               for b in (0, 1)] for k in range(m)]
        for k in range(m):
            llr[n, k] = float(mpmath.log(pb[k][0]) - mpmath.log(pb[k][1]))
        if tx is not None:
            t = int(tx[n])
            u[n] = float(-mpmath.log(post[t], 2))
            v[n] = float(-mpmath.fsum(mpmath.log(pb[k][(labels[t] >> k) & 1], 2)
                                      for k in range(m)))
    out = {"llr": llr}
    if tx is not None:
        out["u"], out["v"] = u, v
        out["mi"] = math.log2(M) - float(np.mean(u))
        out["gmi"] = m - float(np.mean(v))
    return out
