"""Frame-error-rate (FER) and efficiency harness: the oracle side.

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and the CPU leg of the
benchmark.  The GPU library never imports or calls anything here, and
nothing here imports the GPU library.

What the paper measures (Jouguet & Kunz-Jacques): the frame error rate of SC
decoding at a given code rate and channel (Table 1, its FER and beta
columns), the FER entering the secret key rate (Section 2.1, eq. (5)), and
the target FER of 0.1 to which frozen sets are sized (Section 3).  The
efficiency is beta = R / C, C the channel capacity (Section 2.1).

Synthetic frames come from a counter-based generator, Philox4x32-10 (Salmon,
Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11), written here from its published definition; the GPU harness
implements the same generator independently, so both sides build the same
frames without either reading the other's.

Frame f of a run with seed s, key = (s mod 2^32, f):
  u word w (bits 32w .. 32w+31)      = Philox((w >> 2, 0, 0, 0), key)[w & 3]
  channel error at bit i (BSC(p))    = Philox((i >> 2, 1, 0, 0), key)[i & 3] < T,
                                       T = floor(p 2^32)
  x = u G_N, y = x xor e, L_i = (1 - 2 y_i) L0, L0 = float32(ln((1 - p) / p))
  (for the fixed-point decoders L0 in units of 2^-4, rounded half to even)
  frozen values = u on the frozen set
(for N < 32 the low N bits of word 0).  A frame is in error when u-hat != u.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

# Philox4x32 round multipliers and key increments (the published constants)
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32(counters, key, rounds: int = 10) -> np.ndarray:
    """Philox4x32-R on an array of 128-bit counters.

    counters: uint32 array of shape (..., 4); key: two uint32 (or arrays
    broadcastable to counters[..., 0]).  Each round multiplies counter words
    0 and 2 by the two multipliers (64-bit products split into high and low
    halves), swaps and xors the halves with words 1 and 3 and the key, then
    bumps the key by the two Weyl increments.  Returns uint32 (..., 4)."""
    c = np.asarray(counters, dtype=np.uint64) & MASK32
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK32
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    for _ in range(rounds):
        p0 = c0 * np.uint64(PHILOX_M0)
        p1 = c2 * np.uint64(PHILOX_M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(PHILOX_W0)) & np.uint64(MASK32)
        k1 = (k1 + np.uint64(PHILOX_W1)) & np.uint64(MASK32)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def _stream(stream_id: int, n_words: int, key) -> np.ndarray:
    """Words 0 .. n_words-1 of one generator stream: word j is output j & 3 of
    the block with counter (j >> 2, stream_id, 0, 0)."""
    blocks = (n_words + 3) // 4
    ctr = np.zeros((blocks, 4), np.uint64)
    ctr[:, 0] = np.arange(blocks, dtype=np.uint64)
    ctr[:, 1] = stream_id
    return philox4x32(ctr, key).reshape(-1)[:n_words]


def bsc_threshold(p: float) -> int:
    """T = floor(p 2^32): a channel error where the uniform word is < T."""
    return int(math.floor(p * 4294967296.0))


def bsc_l0(p: float) -> np.float32:
    """|LLR| of a BSC(p) output, computed in double and rounded once."""
    return np.float32(math.log((1.0 - p) / p))


def bsc_frame(seed: int, frame: int, log2n: int, p: float, mask: np.ndarray, fixed_point: int = 0):
    """(u bits, frozen values, LLRs float32, channel error bits) of frame f;
    fixed_point 1 (or True): LLRs in units of 2^-4 (the 16-bit fixed-point
    decoders' input); 2: in units of 2^-2 capped at 127 (the 8-bit kind's)."""
    n = 1 << log2n
    key = (seed & MASK32, frame & MASK32)
    words = _stream(0, max(1, n // 32), key)
    u = ((words[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).astype(np.uint8).reshape(-1)[:n]
    e = (_stream(1, n, key) < np.uint32(bsc_threshold(p))).astype(np.uint8)
    x = oracle.encode(log2n, u)
    y = x ^ e
    l0d = math.log((1.0 - p) / p)
    l0 = (bsc_l0(p) if not fixed_point else
          np.float32(oracle.quantize([l0d], 2, oracle.FIXED8_MAX)[0]) if int(fixed_point) == 2 else
          np.float32(oracle.quantize([l0d])[0]))
    llr = np.where(y == 1, -l0, l0).astype(np.float32)
    fval = (u & mask).astype(np.uint8)
    return u, fval, llr, e


def bsc_capacity(p: float) -> float:
    """C = 1 - h2(p) bits per channel use."""
    if p <= 0.0 or p >= 1.0:
        return 1.0
    return 1.0 + p * math.log2(p) + (1.0 - p) * math.log2(1.0 - p)


def fer_bsc(seed: int, frame0: int, n_frames: int, log2n: int, p: float, mask: np.ndarray,
            boxplus: bool = False, n_threads: int | None = None, fixed_kind: int | None = None):
    """Monte-Carlo FER of SC decoding on BSC(p): returns (frames in error,
    bit errors, per-frame error flags).  Frames are decoded by the oracle's
    SC decoder (FP32 min-sum, FP64 box-plus, or with fixed_kind the
    fixed-point decoder on fixed-point frames), one per host thread."""
    import concurrent.futures as cf
    import os

    def one(f):
        fixed = 0 if fixed_kind is None else (2 if fixed_kind == oracle.FIXED_MINSUM8 else 1)
        u, fval, llr, _ = bsc_frame(seed, frame0 + f, log2n, p, mask, fixed_point=fixed)
        if fixed_kind is not None:
            uh = oracle.sc_decode_fixed(llr.astype(np.int32), mask, fval, fixed_kind)[0]
        else:
            uh = oracle.sc_decode(llr, mask, fval, boxplus=boxplus)[0]
        return int((uh != u).sum())

    n_threads = n_threads or max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(n_threads) as ex:
        bit_err = np.array(list(ex.map(one, range(n_frames))), np.int64)
    flags = (bit_err > 0).astype(np.uint8)
    return int(flags.sum()), int(bit_err.sum()), flags
