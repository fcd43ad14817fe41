"""Plain numpy definition of the reorder selector's 16 graph features
(test infrastructure; FP64).  The selector is not part of the paper: it decides
whether reordering will pay for itself (the net-speedup question of Sec. 1.1,
Problem 2), from cheap samples of the edge list.

Samples
  spread:  K = 4096 positions p_k = floor(k * m / K), k < K  (m >= 1)
  windows: W = 64 windows of L = min(1024, m) consecutive edges starting at
           s_w = floor(w * (m - L) / (W - 1)), w < W

Features (f[0..15])
  0  log2(1 + n)                1  log2(1 + m)             2  log2(1 + m / max(n, 1))
  3  log2(1 + n * C_src / P)    4  same for dst    C = #equal pairs among the
                                                   spread samples, P = K(K-1)/2
  5  log2(1 + n * maxcount_src / K)               6  same for dst
  7  distinct_src / K           8  distinct_dst / K
  9  mean over windows of sum_e |src_e - dst_e| / (L * n)
  10 mean over windows of (#distinct src_e >> 5) / L      11 same for dst
  12 mean over windows of #(src_e == src_{e-1}) / (L - 1)   13 same for dst
  14 mean over windows of #(|src_e - src_{e-1}| < 32) / (L - 1)  15 same for dst
  (fractions with L = 1 are 0; every sample feature is 0 when m = 0)
"""
import math

import numpy as np

K_SPREAD = 4096
N_WIN = 64
WIN_LEN = 1024
N_FEAT = 16


def spread_positions(m):
    if m == 0:
        return np.zeros(0, np.int64)
    k = np.arange(K_SPREAD, dtype=np.int64)
    return (k * m) // K_SPREAD


def window_starts(m):
    L = min(WIN_LEN, m)
    if m == 0:
        return L, np.zeros(0, np.int64)
    w = np.arange(N_WIN, dtype=np.int64)
    return L, (w * (m - L)) // (N_WIN - 1)


def _collisions(a):
    _, counts = np.unique(a, return_counts=True)
    return int(np.sum(counts * (counts - 1) // 2)), int(counts.max()), int(counts.size)


def features(src, dst, n):
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    m = src.size
    f = np.zeros(N_FEAT, np.float64)
    f[0] = math.log2(1 + n)
    f[1] = math.log2(1 + m)
    f[2] = math.log2(1 + m / max(n, 1))
    if m == 0:
        return f
    p = spread_positions(m)
    P = K_SPREAD * (K_SPREAD - 1) / 2
    for j, a in ((0, src[p]), (1, dst[p])):
        c, mx, d = _collisions(a)
        f[3 + j] = math.log2(1 + n * c / P)
        f[5 + j] = math.log2(1 + n * mx / K_SPREAD)
        f[7 + j] = d / K_SPREAD
    L, starts = window_starts(m)
    acc = np.zeros(7, np.float64)
    for s in starts:
        ws, wd = src[s:s + L], dst[s:s + L]
        acc[0] += np.abs(ws - wd).sum() / (L * max(n, 1))
        acc[1] += np.unique(ws >> 5).size / L
        acc[2] += np.unique(wd >> 5).size / L
        if L > 1:
            acc[3] += np.count_nonzero(ws[1:] == ws[:-1]) / (L - 1)
            acc[4] += np.count_nonzero(wd[1:] == wd[:-1]) / (L - 1)
            acc[5] += np.count_nonzero(np.abs(ws[1:] - ws[:-1]) < 32) / (L - 1)
            acc[6] += np.count_nonzero(np.abs(wd[1:] - wd[:-1]) < 32) / (L - 1)
    f[9:16] = acc / N_WIN
    return f
