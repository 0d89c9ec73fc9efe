"""Input generator: determinism, bit packing and channel formulas."""
import math

import numpy as np

import synth


def test_pack_unpack_round_trip():
    g = np.random.default_rng(0)
    for n in (1, 2, 31, 32, 33, 64, 1000, 4096):
        b = g.integers(0, 2, n).astype(np.uint8)
        w = synth.pack_bits(b)
        assert w.dtype == np.uint32 and w.size == max(1, (n + 31) // 32)
        assert np.array_equal(synth.unpack_bits(w, n), b)
    # bit i lives in word i >> 5 at position i & 31
    b = np.zeros(64, np.uint8)
    b[37] = 1
    assert synth.pack_bits(b).tolist() == [0, 1 << 5]


def test_frames_are_deterministic():
    mask = np.zeros(256, np.uint8)
    mask[:100] = 1
    ident = lambda u: u  # noqa: E731
    a = synth.frame(42, 8, "bsc", 0.1, mask, ident)
    b = synth.frame(42, 8, "bsc", 0.1, mask, ident)
    c = synth.frame(43, 8, "bsc", 0.1, mask, ident)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert not np.array_equal(a[2], c[2])
    assert np.array_equal(a[1], a[0] & mask)


def test_channel_llr_formulas():
    y = np.array([0, 1], np.uint8)
    l = synth.bsc_llr(y, 0.03)
    assert l[0] == np.float32(math.log(0.97 / 0.03)) and l[1] == -l[0]
    x = np.array([0, 1], np.uint8)
    l2 = synth.biawgn_llr(x, np.array([0.0, 0.0]), 0.5)
    assert l2.tolist() == [8.0, -8.0]
    assert abs(synth.bsc_z0(0.02) - 0.28) < 1e-12
    assert abs(synth.bsc_capacity(0.02) - 0.858559) < 1e-6
