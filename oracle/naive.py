"""Naive and brute-force SC decoders, for pinning the C oracle on tiny codes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``kron_g`` builds G_N = F^{(x)n} as an explicit 0/1 matrix (Section 3,
  Arikan's construction [Ari08]); ``encode_matrix`` multiplies by it mod 2.
* ``naive_sc`` evaluates the SC rule one leaf at a time (Section 4's recursive
  decoder, unrolled per bit): leaf i's LLR is recomputed from the channel
  LLRs every time, and the partial sums it needs are obtained by re-encoding
  the already decided bits with the explicit matrix, never from a stored
  partial-sum vector.  Same f and g as the oracle, so it must agree bit for
  bit.  N <= 64.
* ``brute_sc`` is SC by its likelihood definition: the LLR of leaf i given the
  earlier decisions marginalises over every completion of the later bits,
      L_i = ln sum_{u>i} prod_j W(y_j | x_j(u<i, 0, u>i))
          - ln sum_{u>i} prod_j W(y_j | x_j(u<i, 1, u>i)),
  with W(y|x) proportional to exp((1 - 2x) L_j / 2) for channel LLR L_j.
  Exact box-plus SC computes the same numbers, so it pins the FP64 box-plus
  oracle.  N <= 16.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def kron_g(log2n: int) -> np.ndarray:
    f = np.array([[1, 0], [1, 1]], dtype=np.int64)
    g = np.ones((1, 1), dtype=np.int64)
    for _ in range(log2n):
        g = np.kron(g, f)
    return g


def encode_matrix(u) -> np.ndarray:
    u = np.asarray(u, dtype=np.int64)
    n = u.shape[-1]
    if n == 0:
        return np.zeros(0, np.uint8)
    return (u @ kron_g(n.bit_length() - 1) % 2).astype(np.uint8)


def f_minsum(a, b):
    a = F32(a)
    b = F32(b)
    m = min(abs(a), abs(b))
    return F32(-m) if bool(np.signbit(a)) != bool(np.signbit(b)) else F32(m)


def g_f32(a, b, u):
    a = F32(a)
    b = F32(b)
    return F32(b - a) if u else F32(b + a)


def _leaf_llr(alpha, i, decided):
    """LLR of leaf i of the node whose input LLRs are ``alpha``; ``decided``
    holds this node's decisions for its leaves 0..i-1."""
    m = len(alpha)
    if m == 1:
        return alpha[0]
    h = m // 2
    if i < h:
        return _leaf_llr([f_minsum(alpha[j], alpha[j + h]) for j in range(h)], i, decided)
    beta = encode_matrix(decided[:h])
    return _leaf_llr([g_f32(alpha[j], alpha[j + h], int(beta[j])) for j in range(h)], i - h,
                     decided[h:])


def naive_sc(llr, frozen, fval, teacher=None):
    """Per-bit FP32 min-sum SC.  Returns (u_hat, leaf LLRs float32)."""
    llr = [F32(v) for v in np.asarray(llr, dtype=np.float32)]
    n = len(llr)
    if n > 64:
        raise ValueError("naive_sc is for N <= 64")
    u, used, leaves = [], [], []
    for i in range(n):
        li = _leaf_llr(llr, i, used)
        leaves.append(li)
        ui = int(fval[i]) if frozen[i] else int(li < 0)
        u.append(ui)
        used.append(int(teacher[i]) if teacher is not None else ui)
    return np.array(u, np.uint8), np.array(leaves, np.float32)


def _logsumexp(v: np.ndarray) -> float:
    m = float(np.max(v))
    return m + float(np.log(np.sum(np.exp(v - m))))


def brute_leaf_llr(llr, i, decided) -> float:
    llr = np.asarray(llr, dtype=np.float64)
    n = llr.shape[0]
    g = kron_g(n.bit_length() - 1)
    rest = n - i - 1
    tails = ((np.arange(1 << rest)[:, None] >> np.arange(rest)[None, :]) & 1).astype(np.int64)
    out = []
    for b in (0, 1):
        u = np.zeros((1 << rest, n), np.int64)
        u[:, :i] = np.asarray(decided[:i], dtype=np.int64)[None, :]
        u[:, i] = b
        u[:, i + 1:] = tails
        x = u @ g % 2
        metric = ((1 - 2 * x) * llr[None, :]).sum(axis=1) / 2.0
        out.append(_logsumexp(metric))
    return out[0] - out[1]


def brute_sc(llr, frozen, fval, teacher=None):
    """SC by the likelihood definition in FP64.  Returns (u_hat, leaf LLRs)."""
    n = len(llr)
    if n > 16:
        raise ValueError("brute_sc is for N <= 16")
    u, used, leaves = [], [], []
    for i in range(n):
        li = brute_leaf_llr(llr, i, used)
        leaves.append(li)
        ui = int(fval[i]) if frozen[i] else int(li < 0)
        u.append(ui)
        used.append(int(teacher[i]) if teacher is not None else ui)
    return np.array(u, np.uint8), np.array(leaves, np.float64)


# ---------------------------------------------------------------------------
# Fixed point (Section 4: fixed-point LLRs, phi-table check update), per bit.
# Integers in units of 2^-frac, saturated to +-32767 (kinds 0 and 1) or to
# +-127 (kind 2, min-sum on 8-bit integers).
# ---------------------------------------------------------------------------
FIXED_MAX = 32767
FIXED8_MAX = 127


def _sat(x: int, lim: int) -> int:
    return max(-lim, min(lim, x))


def f_fixed(a: int, b: int, kind: int, table) -> int:
    mag = min(abs(a), abs(b))
    if kind == 1:
        n = len(table)
        phi = lambda x: int(table[x]) if x < n else 0  # noqa: E731
        mag = min(mag, phi(min(phi(abs(a)) + phi(abs(b)), n - 1)))
    return -mag if (a < 0) != (b < 0) else mag


def _leaf_fixed(alpha, i, decided, kind, table):
    lim = FIXED8_MAX if kind == 2 else FIXED_MAX
    m = len(alpha)
    if m == 1:
        return alpha[0]
    h = m // 2
    if i < h:
        return _leaf_fixed([f_fixed(alpha[j], alpha[j + h], kind, table) for j in range(h)], i, decided, kind, table)
    beta = encode_matrix(decided[:h])
    return _leaf_fixed([_sat(alpha[j + h] - alpha[j] if beta[j] else alpha[j + h] + alpha[j], lim) for j in range(h)],
                       i - h, decided[h:], kind, table)


def naive_sc_fixed(llr_q, frozen, fval, kind, table, teacher=None):
    """Per-bit fixed-point SC (partial sums by explicit re-encoding).
    Returns (u_hat, leaf LLRs as integers)."""
    llr = [int(v) for v in np.asarray(llr_q)]
    n = len(llr)
    if n > 64:
        raise ValueError("naive_sc_fixed is for N <= 64")
    u, used, leaves = [], [], []
    for i in range(n):
        li = _leaf_fixed(llr, i, used, kind, table)
        leaves.append(li)
        ui = int(fval[i]) if frozen[i] else int(li < 0)
        u.append(ui)
        used.append(int(teacher[i]) if teacher is not None else ui)
    return np.array(u, np.uint8), np.array(leaves, np.int64)


def naive_scl(llr, frozen, fval, list_size):
    """Per-bit SC list decoding with FP32 min-sum leaf LLRs computed by
    _leaf_llr on each path's own decisions (N <= 32): at an information leaf
    every path offers both bits, metric PM + |lambda| for the bit against
    the hard decision [lambda < 0]; candidates ordered by (metric, path,
    bit), the first list_size kept in that order; frozen leaves add |lambda|
    when the frozen value disagrees.  Returns (u_hat of the least metric,
    ties to the lower path, its metric)."""
    llr = [F32(v) for v in np.asarray(llr, dtype=np.float32)]
    n = len(llr)
    if n > 32:
        raise ValueError("naive_scl is for N <= 32")
    paths = [([], F32(0.0))]
    for i in range(n):
        lam = [_leaf_llr(llr, i, u) for u, _ in paths]
        if frozen[i]:
            b = int(fval[i])
            paths = [(u + [b], F32(pm + abs(l)) if b != int(l < 0) else pm) for (u, pm), l in zip(paths, lam)]
            continue
        cand = []
        for p, ((u, pm), l) in enumerate(zip(paths, lam)):
            for b in (0, 1):
                cand.append((F32(pm + abs(l)) if b != int(l < 0) else pm, p, b))
        cand.sort(key=lambda c: (float(c[0]), c[1], c[2]))
        paths = [(paths[p][0] + [b], pm) for pm, p, b in cand[:list_size]]
    best = min(range(len(paths)), key=lambda k: (float(paths[k][1]), k))
    return np.array(paths[best][0], np.uint8), paths[best][1]
