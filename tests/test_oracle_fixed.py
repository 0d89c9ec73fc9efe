"""Pins of the oracle's fixed-point SC (Section 4: fixed-point LLRs and the
phi = -ln tanh(x/2) table as the check update), no GPU.

* the table against phi evaluated at 60 digits (mpmath), its monotonicity
  and its involution (phi is its own inverse);
* the recursive fixed-point decoder against the per-bit naive decoder
  (partial sums by explicit re-encoding) in the same integer arithmetic,
  with saturation exercised;
* saturating min-sum against the FP32 min-sum oracle where nothing
  saturates (integer-valued FP32 min-sum is exact, so they must agree bit
  for bit);
* the phi-table update against the FP64 exact box-plus update, converging
  as the grid is refined;
* the 8-bit saturating min-sum kind: the same per-bit pin, saturation at
  +-127 by hand-built frames, and equality with the 16-bit kind where no
  value can reach 127."""
import math

import numpy as np
import pytest

import oracle
from oracle import naive


def test_phi_table_against_definition():
    import mpmath

    mpmath.mp.dps = 60
    t = oracle.phi_table()
    assert t.size == oracle.FIXED_TABLE_LEN and t[0] == oracle.FIXED_MAX
    step = mpmath.mpf(1) / (1 << oracle.FIXED_FRAC)
    for i in range(1, t.size):
        v = -mpmath.log(mpmath.tanh(i * step / 2)) / step
        assert t[i] == min(oracle.FIXED_MAX, int(mpmath.floor(v + mpmath.mpf("0.5")))), i
    assert np.all(np.diff(t) <= 0)                  # phi decreases
    assert t[-1] == 0 and t[1] > 0
    # involution: phi(phi(x)) = x, up to the rounding of both lookups
    for i in range(1, 60):
        j = int(t[i])
        if j < t.size:
            assert abs(int(t[j]) - i) <= max(1, i // 8), i


@pytest.mark.parametrize("kind", [oracle.FIXED_MINSUM, oracle.FIXED_PHI, oracle.FIXED_MINSUM8])
@pytest.mark.parametrize("log2n", [1, 2, 3, 4, 5, 6])
def test_fixed_decoder_equals_naive_per_bit(kind, log2n):
    g = np.random.default_rng(40 + 10 * kind + log2n)
    n = 1 << log2n
    table = oracle.phi_table()
    lim = oracle.FIXED8_MAX if kind == oracle.FIXED_MINSUM8 else oracle.FIXED_MAX
    for trial in range(6):
        if trial % 3 == 0:   # near saturation: large magnitudes
            llr = g.integers(-lim, lim + 1, n)
        elif trial % 3 == 1:  # BSC-like
            llr = np.where(g.random(n) < 0.1, -62, 62)
        else:                 # small values, zeros
            llr = g.integers(-80, 81, n)
        frozen = (g.random(n) < 0.4).astype(np.uint8)
        fval = (g.integers(0, 2, n) & frozen).astype(np.uint8)
        u, leaf = oracle.sc_decode_fixed(llr, frozen, fval, kind, want_leaf=True)
        nu, nleaf = naive.naive_sc_fixed(llr, frozen, fval, kind, table)
        assert np.array_equal(u, nu) and np.array_equal(leaf, nleaf), (trial, u, nu)
        t = g.integers(0, 2, n).astype(np.uint8)  # teacher forcing too
        u2, leaf2 = oracle.sc_decode_fixed(llr, frozen, fval, kind, teacher=t, want_leaf=True)
        nu2, nleaf2 = naive.naive_sc_fixed(llr, frozen, fval, kind, table, teacher=t)
        assert np.array_equal(leaf2, nleaf2) and np.array_equal(u2, nu2)


def test_saturation_closed_form():
    """N = 2: inputs (30000, 30000), rate 1: the first leaf is f = 30000,
    decided 0, and the second g = 30000 + 30000 saturates to 32767.  Inputs
    (30000, -30000) with the first bit frozen to 1: f = -30000, and
    g = -30000 - 30000 saturates to -32767."""
    u, leaf = oracle.sc_decode_fixed([30000, 30000], [0, 0], [0, 0], oracle.FIXED_MINSUM, want_leaf=True)
    assert list(leaf) == [30000, 32767] and list(u) == [0, 0]
    u, leaf = oracle.sc_decode_fixed([30000, -30000], [1, 0], [1, 0], oracle.FIXED_MINSUM, want_leaf=True)
    assert list(leaf) == [-30000, -32767] and list(u) == [1, 1]
    with pytest.raises(ValueError):
        oracle.sc_decode_fixed([40000, 0], [0, 0], [0, 0])


@pytest.mark.parametrize("log2n", [6, 10, 14])
def test_saturating_minsum_equals_fp32_minsum_without_saturation(log2n):
    g = np.random.default_rng(70 + log2n)
    n = 1 << log2n
    for k in range(3):
        llr = np.where(g.random(n) < 0.08, -1, 1) * g.integers(1, 2, n)  # sums stay below 2^15
        frozen = (g.random(n) < [0.2, 0.5, 0.8][k]).astype(np.uint8)
        fval = (g.integers(0, 2, n) & frozen).astype(np.uint8)
        u, leaf = oracle.sc_decode_fixed(llr, frozen, fval, oracle.FIXED_MINSUM, want_leaf=True)
        uf, leaff, _ = oracle.sc_decode(llr.astype(np.float32), frozen, fval, want_leaf=True)
        assert np.abs(leaff).max() < oracle.FIXED_MAX
        assert np.array_equal(u, uf) and np.array_equal(leaf.astype(np.float32), leaff)


def test_phi_table_update_converges_to_exact_boxplus():
    """The table update sign min(T[T[|a|] + T[|b|]], |a|, |b|) is the exact
    update 2 atanh(tanh(a/2) tanh(b/2)) up to the table's quantization: on
    [0, 4]^2 its largest error shrinks as the grid is refined (measured
    0.044, 0.013, 0.0019 at 2^-8, 2^-10, 2^-12), so a wrong formula or a
    wrong table would show as an error that does not vanish."""
    worst = []
    for frac, length in ((8, 4096), (10, 16384), (12, 65536)):
        table = oracle.phi_table(frac, length)
        d = 2.0 ** -frac
        w = 0.0
        for A in np.linspace(0.0, 4.0, 41):
            for B in np.linspace(0.0, 4.0, 41):
                qa, qb = int(round(A / d)), int(round(B / d))
                fq = oracle.f_fixed(oracle.FIXED_PHI, qa, -qb, table) * d
                fe = -oracle.f_boxplus(qa * d, qb * d) if qa and qb else 0.0
                w = max(w, abs(fq - fe))
        worst.append(w)
    assert worst[0] > worst[1] > worst[2] and worst[2] < 0.005, worst


def test_quantize():
    q = oracle.quantize([0.03, -0.03, 1.0, -2047.99, 5000.0, -5000.0])
    assert list(q) == [0, 0, 16, -32768 + 1, 32767, -32767]
    assert list(oracle.quantize([0.0625 * 3.5, 0.0625 * 2.5])) == [4, 2]  # ties to even


def test_int8_saturation_closed_form():
    """8-bit kind, N = 2: inputs (100, 100), rate 1: f = 100 decided 0, and
    g = 200 saturates to 127; (100, -100) with the first bit frozen to 1:
    f = -100, g = -200 saturates to -127.  Inputs beyond +-127 are refused."""
    k = oracle.FIXED_MINSUM8
    u, leaf = oracle.sc_decode_fixed([100, 100], [0, 0], [0, 0], k, want_leaf=True)
    assert list(leaf) == [100, 127] and list(u) == [0, 0]
    u, leaf = oracle.sc_decode_fixed([100, -100], [1, 0], [1, 0], k, want_leaf=True)
    assert list(leaf) == [-100, -127] and list(u) == [1, 1]
    with pytest.raises(ValueError):
        oracle.sc_decode_fixed([128, 0], [0, 0], [0, 0], k)
    assert oracle.f_fixed(k, 90, -100) == -90


@pytest.mark.parametrize("log2n", [3, 5, 6])
def test_int8_minsum_equals_int16_minsum_without_saturation(log2n):
    """With inputs of +-1 and N <= 64 no LLR can pass N, so nothing reaches
    127 and the 8-bit kind must equal the 16-bit saturating min-sum; a rate-1
    frame of 100s shows the 8-bit kind saturating where the other does not."""
    g = np.random.default_rng(90 + log2n)
    n = 1 << log2n
    for k in range(6):
        llr = np.where(g.random(n) < 0.3, -1, 1) * (k % 2)
        frozen = (g.random(n) < [0.2, 0.5, 0.8][k % 3]).astype(np.uint8)
        fval = (g.integers(0, 2, n) & frozen).astype(np.uint8)
        t = g.integers(0, 2, n).astype(np.uint8)
        u16, l16 = oracle.sc_decode_fixed(llr, frozen, fval, oracle.FIXED_MINSUM, teacher=t, want_leaf=True)
        u8, l8 = oracle.sc_decode_fixed(llr, frozen, fval, oracle.FIXED_MINSUM8, teacher=t, want_leaf=True)
        assert np.abs(l16).max() <= n < oracle.FIXED8_MAX
        assert np.array_equal(u8, u16) and np.array_equal(l8, l16)
    ones = np.full(n, 100)
    z = np.zeros(n, np.uint8)
    _, l16 = oracle.sc_decode_fixed(ones, z, z, oracle.FIXED_MINSUM, want_leaf=True)
    _, l8 = oracle.sc_decode_fixed(ones, z, z, oracle.FIXED_MINSUM8, want_leaf=True)
    assert l16[-1] == min(100 * n, oracle.FIXED_MAX) and l8[-1] == oracle.FIXED8_MAX
