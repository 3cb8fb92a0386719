"""The relaxation modulus and its batch-means error from oracle stress
samples, by their definitions (helpers for the GPU correlator tests).

G[l][k] = sum over chains and the components xy, yz, zx of the multiple-tau
correlation C of x = sigma_ab with y = sigma_ab + sigma^v_ab (Sec. 2.3,
Green-Kubo form with the virtual stress), divided by 3 M cnt.  The chains are
split into `batches` contiguous groups of equal size (group b: chains
[M b / B, M (b + 1) / B)); G_err is the standard error of the B group means,
sqrt(sum_b (G_b - mean)^2 / (B - 1) / B).
"""
from __future__ import annotations

import numpy as np

import oracle


def oracle_G(samples, levels, batches=1, virtual=False):
    """samples [T][M][12] -> (G [levels][16], G_err [levels][16], cnt)."""
    T, M, _ = samples.shape
    per_chain = np.zeros((M, levels, 16))
    cnt = None
    for k in range(M):
        for c in range(3):
            x = np.ascontiguousarray(samples[:, k, (9 if virtual else 3) + c])
            y = np.ascontiguousarray(samples[:, k, 3 + c] + samples[:, k, 9 + c])
            C, n = oracle.multitau(x, y, levels=levels, lags=16)
            per_chain[k] += C
            cnt = n
    den = np.maximum(cnt, 1).astype(np.float64)
    G = np.where(cnt > 0, per_chain.sum(axis=0) / (3.0 * M * den), 0.0)
    G_err = np.zeros_like(G)
    if batches >= 2:
        means = []
        for b in range(batches):
            c0, c1 = M * b // batches, M * (b + 1) // batches
            means.append(per_chain[c0:c1].sum(axis=0) / (3.0 * (c1 - c0) * den))
        means = np.array(means)
        G_err = np.sqrt(((means - means.mean(axis=0)) ** 2).sum(axis=0) / (batches - 1) / batches)
        G_err = np.where(cnt > 0, G_err, 0.0)
    return G, G_err, cnt
