"""Seeded synthetic inputs for polar SC decoding.

Shared by the tests and the benchmark.  This module draws random numbers and
maps channel outputs to LLRs; it holds none of the decoding or encoding
arithmetic.  The caller supplies x = u G_N (from whichever encoder it trusts).

Channels (Section 1 and Section 3 of the paper):
  * DV-QKD: binary symmetric channel with error probability p (the QBER),
    LLR_j = (1 - 2 y_j) ln((1 - p) / p).
  * CV-QKD after binarisation: BPSK (0 -> +1, 1 -> -1) over additive white
    Gaussian noise of standard deviation sigma, LLR_j = 2 y_j / sigma^2.
LLRs are formed in float64 and rounded once to float32.

Random numbers come from numpy's counter-based Philox generator keyed by the
seed, so every frame is reproducible on any host.
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed)))


def draw_bits(g: np.random.Generator, n: int) -> np.ndarray:
    return g.integers(0, 2, size=n, dtype=np.uint8)


def bsc_noise(g: np.random.Generator, n: int, p: float) -> np.ndarray:
    return (g.random(n) < p).astype(np.uint8)


def gauss_noise(g: np.random.Generator, n: int) -> np.ndarray:
    return g.standard_normal(n)


def bsc_llr(y: np.ndarray, p: float) -> np.ndarray:
    l0 = math.log((1.0 - p) / p)
    return ((1.0 - 2.0 * y.astype(np.float64)) * l0).astype(np.float32)


def biawgn_llr(x: np.ndarray, noise: np.ndarray, sigma: float) -> np.ndarray:
    y = (1.0 - 2.0 * x.astype(np.float64)) + sigma * noise
    return (2.0 * y / (sigma * sigma)).astype(np.float32)


def fixed_point(llr, frac: int = 4, limit: int = 32767) -> np.ndarray:
    """Input recipe for the fixed-point decoders: channel LLRs as integers in
    units of 2^-frac (round half to even, saturated to +-limit), stored as
    float32."""
    q = np.clip(np.round(np.asarray(llr, np.float64) * (1 << frac)), -limit, limit)
    return q.astype(np.float32)


def bsc_z0(p: float) -> float:
    """Bhattacharyya parameter of BSC(p)."""
    return 2.0 * math.sqrt(p * (1.0 - p))


def biawgn_z0(sigma: float) -> float:
    """Bhattacharyya parameter of BPSK over AWGN with noise std sigma."""
    return math.exp(-1.0 / (2.0 * sigma * sigma))


def biawgn_channel(sigma: float, cells: int = 2000, span: float = 8.0) -> np.ndarray:
    """BPSK over AWGN(sigma) as a finite symmetric channel (the input of the
    degrading construction): the output magnitude |y| is cut into `cells`
    equal cells over [0, 1 + span sigma), the last one open to infinity, and
    cell k gives the pair (P(y in cell | +1), P(-y in cell | +1)) from the
    Gaussian distribution function.  Returns (cells, 2) float64 pairs with
    a >= b >= 0 summing to 1."""
    edges = np.linspace(0.0, 1.0 + span * sigma, cells + 1)
    edges[-1] = np.inf

    r = sigma * math.sqrt(2.0)

    def upper(t):  # P(Y > t | x = +1), Y ~ N(1, sigma^2)
        return np.array([0.5 * math.erfc((v - 1.0) / r) if np.isfinite(v) else 0.0 for v in t])

    def lower(t):  # P(Y <= t | x = +1)
        return np.array([0.5 * math.erfc((1.0 - v) / r) if np.isfinite(v) else 0.0 for v in t])

    a = upper(edges[:-1]) - upper(edges[1:])
    b = lower(-edges[:-1]) - lower(-edges[1:])
    a = np.maximum(a, 0.0)
    b = np.minimum(np.maximum(b, 0.0), a)
    w = np.stack([a, b], 1)
    return w / w.sum()


def bsc_capacity(p: float) -> float:
    h = -p * math.log2(p) - (1.0 - p) * math.log2(1.0 - p)
    return 1.0 - h


def frame(seed: int, log2n: int, channel: str, param: float, frozen: np.ndarray, encode):
    """One frame: information word u, revealed frozen values and channel LLRs.

    ``encode(u) -> x`` is supplied by the caller; ``frozen`` is a 0/1 byte
    mask.  Returns (u, fval, llr) with fval = u on frozen positions, 0 else."""
    n = 1 << log2n
    g = rng(seed)
    u = draw_bits(g, n)
    x = np.asarray(encode(u), dtype=np.uint8)
    if channel == "bsc":
        llr = bsc_llr(x ^ bsc_noise(g, n, param), param)
    elif channel == "biawgn":
        llr = biawgn_llr(x, gauss_noise(g, n), param)
    elif channel == "noiseless":
        llr = bsc_llr(x, param)
    else:
        raise ValueError(f"unknown channel {channel!r}")
    fval = (u & np.asarray(frozen, dtype=np.uint8)).astype(np.uint8)
    return u, fval, llr


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """0/1 bytes (..., N) -> uint32 words (..., max(1, N/32)); bit i in word
    i >> 5 at position i & 31."""
    bits = np.asarray(bits, dtype=np.uint8)
    n = bits.shape[-1]
    nw = max(1, (n + 31) // 32)
    pad = nw * 32 - n
    if pad:
        bits = np.concatenate([bits, np.zeros(bits.shape[:-1] + (pad,), np.uint8)], axis=-1)
    by = np.packbits(bits.reshape(bits.shape[:-1] + (nw * 4, 8)), axis=-1, bitorder="little")
    return np.ascontiguousarray(by.reshape(bits.shape[:-1] + (nw * 4,))).view(np.uint32)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint32))
    by = w.view(np.uint8)
    bits = np.unpackbits(by, axis=-1, bitorder="little")
    return bits[..., :n].astype(np.uint8)
