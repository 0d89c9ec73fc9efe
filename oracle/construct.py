"""Frozen-set construction by channel degradation: the oracle side.

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and the CPU leg of the
benchmark.  The GPU library never imports or calls anything here, and
nothing here imports the GPU library.

Section 3 of the paper freezes the least reliable synthetic channels; its
frozen sets come from the density-evolution construction it cites [MT09].
This module computes the error probability of every synthetic channel by
tracking each channel as a finite binary-input memoryless symmetric (BMS)
channel and degrading it to at most ``mu`` outputs after every polarization
step (Tal and Vardy, "How to construct polar codes"), with the merging done
by binning outputs on the binary entropy of their posterior (Pedarsani,
Hassani, Tal and Telatar, "On the construction of polar codes").  Merging
outputs gives a degraded channel, so every reported error probability is an
upper bound on the true one.

Representation: a list of output pairs (a, b), a >= b >= 0, a = W(y|0),
b = W(y|1) for one output y of a conjugate pair {y, y'} (W(y'|0) = b,
W(y'|1) = a); sum(a + b) = 1.  Error probability of the ML decision
P_e = sum(b); Bhattacharyya parameter Z = sum(2 sqrt(a b)); capacity
I = sum((a + b) (1 - h2(b / (a + b)))).

One polarization step of W (index bit 0: the first-decoded "minus" channel
at child 2j, bit 1: the "plus" channel at child 2j + 1, as in the
Bhattacharyya recursion), over all ordered pairs (i, j) of outputs:
  minus: (a_i a_j + b_i b_j,  a_i b_j + b_i a_j)
  plus:  (a_i a_j, b_i b_j)  and  (max(a_i b_j, b_i a_j), min(a_i b_j, b_i a_j))
Merge: output k goes to bin min(mu - 1, floor(mu h2(b_k / (a_k + b_k)))),
and each bin's outputs are summed in output order; empty bins are dropped and
the others kept in ascending bin order.  The channel of every index, the root
included, is merged.  All arithmetic is in double precision, products and
sums rounded one at a time (no fused multiply-add).
"""
from __future__ import annotations

import numpy as np


def h2(q):
    """Binary entropy in bits (0 at q = 0)."""
    q = np.asarray(q, np.float64)
    out = np.zeros_like(q)
    m = (q > 0) & (q < 1)
    qq = q[m]
    out[m] = -qq * np.log2(qq) - (1 - qq) * np.log2(1 - qq)
    return out


def bsc(p: float) -> np.ndarray:
    """BSC(p), p < 1/2: one output pair."""
    return np.array([[1.0 - p, p]], np.float64)


def bec(eps: float) -> np.ndarray:
    """BEC(eps): the perfect pair (1 - eps, 0) and the erasure, a
    self-conjugate output written as the pair (eps/2, eps/2)."""
    return np.array([[1.0 - eps, 0.0], [eps / 2.0, eps / 2.0]], np.float64)


def minus(w: np.ndarray) -> np.ndarray:
    a, b = w[:, 0], w[:, 1]
    aa = (a[:, None] * a[None, :] + b[:, None] * b[None, :]).reshape(-1)
    bb = (a[:, None] * b[None, :] + b[:, None] * a[None, :]).reshape(-1)
    return np.stack([aa, bb], axis=1)


def plus(w: np.ndarray) -> np.ndarray:
    a, b = w[:, 0], w[:, 1]
    p1a = (a[:, None] * a[None, :]).reshape(-1)
    p1b = (b[:, None] * b[None, :]).reshape(-1)
    x = (a[:, None] * b[None, :]).reshape(-1)
    y = (b[:, None] * a[None, :]).reshape(-1)
    # outputs interleaved per ordered pair: (i, j) type 1, then (i, j) type 2
    out = np.empty((p1a.size * 2, 2), np.float64)
    out[0::2, 0] = p1a
    out[0::2, 1] = p1b
    out[1::2, 0] = np.maximum(x, y)
    out[1::2, 1] = np.minimum(x, y)
    return out


def merge(w: np.ndarray, mu: int) -> np.ndarray:
    """Degrade to at most mu outputs by entropy binning (sums in output order)."""
    tot = w[:, 0] + w[:, 1]
    keep = tot > 0
    w = w[keep]
    tot = tot[keep]
    k = np.minimum(mu - 1, np.floor(mu * h2(w[:, 1] / tot)).astype(np.int64))
    bins, slot = np.unique(k, return_inverse=True)   # occupied bins, ascending
    acc = np.zeros((bins.size, 2), np.float64)
    np.add.at(acc, slot, w)       # unbuffered: each bin summed in output order
    return acc


def error_probability(w: np.ndarray) -> float:
    """P_e = sum of b over the outputs, added one by one in output order."""
    s = 0.0
    for v in w[:, 1]:
        s += float(v)
    return s


def capacity(w: np.ndarray) -> float:
    tot = w[:, 0] + w[:, 1]
    m = tot > 0
    return float((tot[m] * (1.0 - h2(w[m, 1] / tot[m]))).sum())


def synthetic_error_probabilities(log2n: int, w0: np.ndarray, mu: int) -> np.ndarray:
    """P_e of the N synthetic channels (index i: bit n-1 chooses the first
    step, as in the Bhattacharyya recursion), each an upper bound."""
    level = [merge(w0, mu)]
    for _ in range(log2n):
        nxt = []
        for w in level:
            nxt.append(merge(minus(w), mu))
            nxt.append(merge(plus(w), mu))
        level = nxt
    return np.array([error_probability(w) for w in level], np.float64)


def channel_error_probability(log2n: int, index: int, w0: np.ndarray, mu: int) -> float:
    """P_e of synthetic channel `index` alone: the steps along its path only
    (most significant index bit first), so single channels of very long codes
    can be checked one by one."""
    w = merge(w0, mu)
    for k in range(log2n - 1, -1, -1):
        w = merge(plus(w) if (index >> k) & 1 else minus(w), mu)
    return error_probability(w)


def frozen_from_pe(pe: np.ndarray, n_frozen: int = -1, fer_bound: float = 0.1):
    """Freeze the channels with the largest error probability (ties: lower
    index first).  n_frozen >= 0: that many; -1: the largest information set
    whose union bound sum(P_e) stays <= fer_bound (Section 3)."""
    n = pe.size
    order = sorted(range(n), key=lambda i: (-pe[i], i))  # worst first
    if n_frozen < 0:
        s = 0.0
        k = 0
        for i in reversed(order):   # best channels first
            if s + pe[i] > fer_bound:
                break
            s += pe[i]
            k += 1
        n_frozen = n - k
    mask = np.zeros(n, np.uint8)
    mask[order[:n_frozen]] = 1
    return mask, n_frozen


def brute_force_error_probabilities(log2n: int, p: float) -> np.ndarray:
    """Exact P_e of the synthetic channels W_N^(i) of BSC(p), N <= 8, by
    enumerating every channel output y and every past u_0..u_{i-1}:
    P_e(i) = 1/2 sum_{y, u<i} min(W(y, u<i | 0), W(y, u<i | 1)), with
    W(y, u<i | u_i) = 2^-(N-1) sum_{u>i} prod_j BSC(y_j | (uG)_j)."""
    from oracle.naive import kron_g

    n = 1 << log2n
    g = kron_g(log2n)
    us = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)
    xs = us @ g % 2                                     # codeword of every u
    ys = us                                             # every output word
    dist = (xs[:, None, :] != ys[None, :, :]).sum(axis=2)   # [u, y]
    lik = (p ** dist) * ((1 - p) ** (n - dist))         # W^N(y | x(u))
    out = np.zeros(n)
    for i in range(n):
        # group u by (u_<i, u_i), summing over u_>i
        key = us[:, :i] @ (1 << np.arange(i)) if i else np.zeros(1 << n, np.int64)
        tot = np.zeros((1 << i, 2, 1 << n))
        np.add.at(tot, (key, us[:, i]), lik)
        w = tot / 2 ** (n - 1)
        out[i] = 0.5 * np.minimum(w[:, 0, :], w[:, 1, :]).sum()
    return out
