"""Pins of the FER harness's oracle side (oracle/fer.py), no GPU:
the generator against the published Philox4x32 known-answer vectors, the
channel statistics against their definition, the frame construction against
its closed form, and the Monte-Carlo FER against an exact enumeration of
every (u, error pattern) pair on small codes."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import fer

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    kat = json.load(open(os.path.join(HERE, "golden", "philox4x32_kat.json")))
    for v in kat["vectors"]:
        ctr = np.array([int(x, 16) for x in v["counter"]], np.uint64)[None, :]
        key = tuple(int(x, 16) for x in v["key"])
        out = fer.philox4x32(ctr, key, rounds=v["rounds"])[0]
        assert [f"{int(x):08x}" for x in out] == v["output"]


def test_philox_vectorised_equals_scalar_and_depends_on_every_input():
    g = np.random.default_rng(3)
    ctr = g.integers(0, 2**32, (64, 4), dtype=np.uint64)
    key = (int(g.integers(0, 2**32)), int(g.integers(0, 2**32)))
    many = fer.philox4x32(ctr, key)
    for i in range(0, 64, 9):
        assert np.array_equal(many[i], fer.philox4x32(ctr[i:i + 1], key)[0])
    base = fer.philox4x32(ctr[:1], key)[0]
    for j in range(4):  # every counter word and key word changes the output
        c2 = ctr[:1].copy()
        c2[0, j] ^= 1
        assert not np.array_equal(fer.philox4x32(c2, key)[0], base)
    assert not np.array_equal(fer.philox4x32(ctr[:1], (key[0] ^ 1, key[1]))[0], base)
    assert not np.array_equal(fer.philox4x32(ctr[:1], (key[0], key[1] ^ 1))[0], base)


def test_channel_and_info_bits_statistics():
    """Error indicators are Bernoulli(p) and u bits Bernoulli(1/2) (within
    five standard deviations over 2^20 draws), frames differ."""
    log2n, p = 20, 0.03
    mask = np.zeros(1 << log2n, np.uint8)
    u, fval, llr, e = fer.bsc_frame(7, 0, log2n, p, mask)
    n = u.size
    assert abs(e.mean() - p) < 5 * math.sqrt(p * (1 - p) / n)
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(0.25 / n)
    u2, _, _, e2 = fer.bsc_frame(7, 1, log2n, p, mask)
    assert (u != u2).mean() > 0.45 and (e != e2).any()
    u3, _, _, _ = fer.bsc_frame(8, 0, log2n, p, mask)
    assert (u != u3).mean() > 0.45


def test_frame_closed_form():
    """LLRs are +-L0 with L0 = ln((1-p)/p) rounded once to float32; the sign
    is the hard decision of y = uG xor e; frozen values are u on the mask."""
    log2n, p = 12, 0.02
    mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(p), 819)
    u, fval, llr, e = fer.bsc_frame(1, 5, log2n, p, mask)
    l0 = np.float32(math.log(49.0))
    assert fer.bsc_l0(p) == l0
    assert set(np.unique(np.abs(llr))) == {l0}
    assert np.array_equal((llr < 0).astype(np.uint8), oracle.encode(log2n, u) ^ e)
    assert np.array_equal(fval, u & mask)
    assert fer.bsc_threshold(0.5) == 2**31


def _exact_fer(log2n, p, mask):
    """Exact SC frame error rate by enumeration: average over every u (the
    generator draws u uniformly) and every error pattern weighted by its
    BSC probability (the decoder breaks LLR ties towards 0, so the error
    rate depends on u and is averaged, not taken at u = 0)."""
    n = 1 << log2n
    l0 = fer.bsc_l0(p)
    total = 0.0
    for ub in itertools.product((0, 1), repeat=n):
        u = np.array(ub, np.uint8)
        x = oracle.encode(log2n, u)
        fval = u & mask
        for eb in itertools.product((0, 1), repeat=n):
            e = np.array(eb, np.uint8)
            w = int(e.sum())
            pe = p ** w * (1 - p) ** (n - w)
            llr = np.where((x ^ e) == 1, -l0, l0).astype(np.float32)
            uh = oracle.sc_decode(llr, mask, fval)[0]
            total += pe * float((uh != u).any())
    return total / 2 ** n


@pytest.mark.parametrize("log2n,mask_bits,p", [
    (2, [1, 0, 0, 0], 0.1),
    (2, [1, 1, 1, 0], 0.2),
    (3, [1, 1, 1, 0, 1, 0, 0, 0], 0.08),
])
def test_monte_carlo_fer_matches_exact_enumeration(log2n, mask_bits, p):
    mask = np.array(mask_bits, np.uint8)
    exact = _exact_fer(log2n, p, mask)
    frames = 6000
    errs, bits, flags = fer.fer_bsc(11, 0, frames, log2n, p, mask)
    assert flags.sum() == errs and bits >= errs
    sd = math.sqrt(exact * (1 - exact) / frames)
    assert abs(errs / frames - exact) < 5 * sd + 1e-12, (errs / frames, exact)


def test_fer_extremes():
    """Rate 0 never errs; the noiseless channel never errs; frame counts add."""
    log2n = 10
    n = 1 << log2n
    errs, _, _ = fer.fer_bsc(2, 0, 30, log2n, 0.1, np.ones(n, np.uint8))
    assert errs == 0
    mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(0.05), n // 2)
    errs, _, _ = fer.fer_bsc(2, 0, 30, log2n, 1e-12, mask)
    assert errs == 0
    a, _, fa = fer.fer_bsc(3, 0, 40, log2n, 0.05, mask)
    b, _, fb = fer.fer_bsc(3, 40, 40, log2n, 0.05, mask)
    c, _, fc = fer.fer_bsc(3, 0, 80, log2n, 0.05, mask)
    assert a + b == c and np.array_equal(np.concatenate([fa, fb]), fc)


def test_capacity():
    assert abs(fer.bsc_capacity(0.02) - 0.858559) < 1e-6
    assert abs(fer.bsc_capacity(0.03) - 0.805608) < 1e-6
    assert fer.bsc_capacity(0.5) == pytest.approx(0.0, abs=1e-15)
