"""Brute-force betweenness from the definition -- TEST INFRASTRUCTURE ONLY.

Eq. (1) of Section 2.1: bc[v] = sum over ordered pairs s != v != t of
sigma_st(v) / sigma_st.  No Brandes recursion is used:

* d(s,t) and sigma_st come from powers of the adjacency matrix: the number of
  walks of length k from s to t equals the number of shortest paths when k is
  the first power with a nonzero (s,t) entry, because every walk of length
  d(s,t) between s and t is a shortest path.
* sigma_st(v) = sigma_sv * sigma_vt when d(s,v) + d(v,t) = d(s,t), else 0
  (every shortest s-t path through v splits at v into two shortest paths).

Works on a batch of graphs at once (adjacency tensor [B, n, n]); exact integer
path counts in int64, the final quotients in float64.  Only for tiny n.
"""
from __future__ import annotations

import numpy as np


def adjacency(n: int, row_ptr, col) -> np.ndarray:
    a = np.zeros((n, n), dtype=np.int64)
    rp = np.asarray(row_ptr)
    for v in range(n):
        a[v, np.asarray(col[rp[v]:rp[v + 1]])] = 1
    return a


def distances_and_counts(adj: np.ndarray):
    """adj: [B, n, n] 0/1.  Returns (dist [B,n,n] with -1 unreachable, sigma [B,n,n])."""
    B, n, _ = adj.shape
    eye = np.broadcast_to(np.eye(n, dtype=np.int64), (B, n, n))
    dist = np.where(eye == 1, 0, -1).astype(np.int64)
    sigma = eye.copy()
    walk = eye.copy()
    for k in range(1, n):
        walk = np.matmul(walk, adj)
        new = (dist < 0) & (walk > 0)
        dist = np.where(new, k, dist)
        sigma = np.where(new, walk, sigma)
    return dist, sigma


def bc_bruteforce_batch(adj: np.ndarray) -> np.ndarray:
    """Ordered-pair betweenness for a batch of graphs, [B, n, n] -> [B, n]."""
    B, n, _ = adj.shape
    dist, sigma = distances_and_counts(adj)
    bc = np.zeros((B, n), dtype=np.float64)
    for v in range(n):
        d_sv = dist[:, :, v][:, :, None]        # [B, s, 1]
        d_vt = dist[:, v, :][:, None, :]        # [B, 1, t]
        s_sv = sigma[:, :, v][:, :, None]
        s_vt = sigma[:, v, :][:, None, :]
        through = (d_sv >= 0) & (d_vt >= 0) & (dist >= 0) & (d_sv + d_vt == dist)
        ok = np.ones((n, n), dtype=bool)
        ok[v, :] = False
        ok[:, v] = False
        np.fill_diagonal(ok, False)
        through &= ok[None]
        num = np.where(through, s_sv * s_vt, 0).astype(np.float64)
        den = np.where(through, sigma, 1).astype(np.float64)
        bc[:, v] = (num / den).sum(axis=(1, 2))
    return bc


def bc_bruteforce(n: int, row_ptr, col) -> np.ndarray:
    return bc_bruteforce_batch(adjacency(n, row_ptr, col)[None])[0]


def distance_sum_ordered(n: int, row_ptr, col) -> int:
    """Sum over ordered connected pairs s != t of (d(s,t) - 1)."""
    dist, _ = distances_and_counts(adjacency(n, row_ptr, col)[None])
    d = dist[0]
    mask = d > 0
    return int((d[mask] - 1).sum())
