"""Pins for the oracle SC decoder (Section 4's recursive decoder, [Ari08]).

* FP32 min-sum: bit-exact agreement with the naive per-bit evaluation of the
  SC rule (explicit re-encoding of decided bits, N <= 64), including leaf
  LLRs, teacher forcing and inputs full of exact zeros.
* FP64 box-plus: agreement with SC by its likelihood definition (brute force
  over all completions, N <= 16), and the scalar f against 400-digit mpmath.
* Closed forms at full scale: noiseless frames, rate 1, rate 0, N = 1 and 2.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
import synth
from oracle import naive


def _f32_bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def _llr_kinds(g, n):
    yield "bsc", np.where(g.random(n) < 0.2, -1.0, 1.0).astype(np.float32) * np.float32(math.log(49.0))
    yield "gauss", (2.0 * ((1 - 2 * g.integers(0, 2, n)) + 0.9 * g.standard_normal(n)) / 0.81).astype(np.float32)
    yield "ints_with_zeros", g.integers(-2, 3, n).astype(np.float32)
    yield "signed_zeros", np.where(g.random(n) < 0.5, np.float32(-0.0), np.float32(0.0)) + \
        np.where(g.random(n) < 0.3, g.integers(-3, 4, n), 0).astype(np.float32)


def _masks(g, n):
    yield np.zeros(n, np.uint8)
    yield np.ones(n, np.uint8)
    for dens in (0.2, 0.5, 0.8):
        yield (g.random(n) < dens).astype(np.uint8)
    if n >= 2:
        m, _, _ = oracle.frozen_set(n.bit_length() - 1, 0.4, n // 2)
        yield m


@pytest.mark.parametrize("log2n", range(0, 7))
def test_minsum_matches_naive_per_bit(log2n):
    n = 1 << log2n
    g = np.random.default_rng(1000 + log2n)
    cases = 0
    for kind, llr in _llr_kinds(g, n):
        for mask in _masks(g, n):
            fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
            u, leaf, _ = oracle.sc_decode(llr, mask, fval, want_leaf=True)
            un, ln = naive.naive_sc(llr, mask, fval)
            assert np.array_equal(u, un), (kind, mask)
            assert np.array_equal(_f32_bits(leaf), _f32_bits(ln)), (kind, mask)
            # teacher forcing with an arbitrary teacher
            t = g.integers(0, 2, n).astype(np.uint8)
            t[mask == 1] = fval[mask == 1]
            u2, leaf2, _ = oracle.sc_decode(llr, mask, fval, teacher=t, want_leaf=True)
            un2, ln2 = naive.naive_sc(llr, mask, fval, teacher=t)
            assert np.array_equal(u2, un2)
            assert np.array_equal(_f32_bits(leaf2), _f32_bits(ln2))
            cases += 1
    assert cases >= 20


def test_minsum_beta_is_reencoded_decisions():
    g = np.random.default_rng(5)
    for log2n in (4, 9, 13):
        n = 1 << log2n
        mask = (g.random(n) < 0.4).astype(np.uint8)
        fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
        llr = g.standard_normal(n).astype(np.float32)
        u, _, beta = oracle.sc_decode(llr, mask, fval, want_beta=True)
        assert np.array_equal(beta, oracle.encode(log2n, u))
        assert np.array_equal(u[mask == 1], fval[mask == 1])


@pytest.mark.parametrize("log2n", range(0, 5))
def test_boxplus_matches_brute_force_likelihood(log2n):
    n = 1 << log2n
    g = np.random.default_rng(2000 + log2n)
    for rep in range(6):
        sigma = 0.7 + 0.2 * rep
        x = g.integers(0, 2, n)
        llr = (2.0 * ((1 - 2 * x) + sigma * g.standard_normal(n)) / sigma ** 2).astype(np.float32)
        for mask in _masks(g, n):
            fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
            u, leaf, _ = oracle.sc_decode(llr, mask, fval, boxplus=True, want_leaf=True)
            ub, lb = naive.brute_sc(llr, mask, fval)
            np.testing.assert_allclose(leaf, lb, rtol=1e-11, atol=1e-11)
            tiny = np.abs(lb) < 1e-9
            assert np.array_equal(u[~tiny], ub[~tiny])


def test_boxplus_teacher_forcing_matches_brute_force():
    g = np.random.default_rng(77)
    n = 16
    for _ in range(5):
        llr = (3.0 * g.standard_normal(n)).astype(np.float32)
        mask = (g.random(n) < 0.5).astype(np.uint8)
        fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
        t = g.integers(0, 2, n).astype(np.uint8)
        t[mask == 1] = fval[mask == 1]
        _, leaf, _ = oracle.sc_decode(llr, mask, fval, boxplus=True, teacher=t, want_leaf=True)
        _, lb = naive.brute_sc(llr, mask, fval, teacher=t)
        np.testing.assert_allclose(leaf, lb, rtol=1e-11, atol=1e-11)


def test_boxplus_f_against_mpmath():
    mpmath.mp.dps = 400
    g = np.random.default_rng(11)
    a = np.exp(g.uniform(np.log(1e-30), np.log(316.0), 400)) * np.where(g.random(400) < 0.5, -1, 1)
    b = np.exp(g.uniform(np.log(1e-30), np.log(316.0), 400)) * np.where(g.random(400) < 0.5, -1, 1)
    worst = 0.0
    for x, y in zip(a, b):
        ref = 2 * mpmath.atanh(mpmath.tanh(mpmath.mpf(x) / 2) * mpmath.tanh(mpmath.mpf(y) / 2))
        got = oracle.f_boxplus(float(x), float(y))
        worst = max(worst, abs(got - float(ref)) / abs(float(ref)))
    assert worst < 4e-15


def test_minsum_upper_bounds_boxplus():
    g = np.random.default_rng(12)
    for _ in range(2000):
        a, b = (g.standard_normal(2) * 5).astype(np.float32)
        fm = oracle.f_minsum(a, b)
        fb = oracle.f_boxplus(float(a), float(b))
        assert abs(fm) >= abs(fb)
        if fb != 0.0:
            assert (fm < 0) == (fb < 0)


def test_minsum_f_and_g_definitions():
    L = np.float32(3.5)
    assert oracle.f_minsum(L, -2.0) == -2.0
    assert oracle.f_minsum(-L, -2.0) == 2.0
    assert oracle.f_minsum(0.0, -2.0) == 0.0
    assert oracle.g_f32(1.5, 2.0, 0) == 3.5
    assert oracle.g_f32(1.5, 2.0, 1) == 0.5


def test_n1_and_n2_closed_forms():
    g = np.random.default_rng(3)
    for _ in range(200):
        l0, l1 = g.integers(-3, 4, 2).astype(np.float32)
        # N = 1: u0 = [L0 < 0]
        u, _, _ = oracle.sc_decode(np.array([l0], np.float32), np.zeros(1, np.uint8), np.zeros(1, np.uint8))
        assert u[0] == int(l0 < 0)
        # N = 2: u0 = [f(L0, L1) < 0]; u1 = [L1 + (1 - 2 u0) L0 < 0]
        fm = np.float32(min(abs(l0), abs(l1))) * (-1 if np.signbit(l0) != np.signbit(l1) else 1)
        u0 = int(fm < 0)
        u1 = int(np.float32(l1 + (1 - 2 * u0) * l0) < 0)
        u, _, _ = oracle.sc_decode(np.array([l0, l1], np.float32), np.zeros(2, np.uint8), np.zeros(2, np.uint8))
        assert (u[0], u[1]) == (u0, u1)


def test_rate1_counterexample_hard_decision_is_not_sc():
    # alpha = (0, -1), no frozen bits: SC gives u = (0, 1), x-hat = (1, 1),
    # while the hard decision of alpha would be (0, 1).
    u, _, beta = oracle.sc_decode(np.array([0.0, -1.0], np.float32), np.zeros(2, np.uint8),
                                  np.zeros(2, np.uint8), want_beta=True)
    assert list(u) == [0, 1]
    assert list(beta) == [1, 1]


@pytest.mark.parametrize("boxplus", [False, True])
def test_noiseless_round_trip_at_scale(boxplus):
    if boxplus:
        log2n, sigma = 16, 0.97
        k = int(0.45 * (1 << log2n))
        mask, _, _ = oracle.frozen_set(log2n, synth.biawgn_z0(sigma), (1 << log2n) - k)
        u, fval, llr = synth.frame(5, log2n, "noiseless", 0.03, mask, lambda v: oracle.encode(log2n, v))
        llr = (llr / np.float32(math.log(97 / 3)) * np.float32(2.0 / sigma ** 2)).astype(np.float32)
    else:
        log2n = 20
        mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(0.03), 1 << 18)
        u, fval, llr = synth.frame(6, log2n, "noiseless", 0.03, mask, lambda v: oracle.encode(log2n, v))
    uh, leaf, _ = oracle.sc_decode(llr, mask, fval, boxplus=boxplus, want_leaf=True)
    assert np.array_equal(uh, u)
    assert np.all(leaf[mask == 0] != 0)


@pytest.mark.parametrize("boxplus", [False, True])
def test_rate1_is_hard_decision_reencoded(boxplus):
    log2n = 16
    n = 1 << log2n
    g = np.random.default_rng(9)
    sign = np.where(g.random(n) < 0.5, -1.0, 1.0)
    if boxplus:
        # box-plus of small values shrinks like x^2/2 per minus step and can
        # underflow to 0; |L| >= 15 keeps every LLR >= 15 - 16 ln 2 > 0
        llr = (sign * (15.0 + 15.0 * g.random(n))).astype(np.float32)
    else:
        llr = (sign * (0.5 + g.random(n))).astype(np.float32)
    uh, _, _ = oracle.sc_decode(llr, np.zeros(n, np.uint8), np.zeros(n, np.uint8), boxplus=boxplus)
    assert np.array_equal(uh, oracle.encode(log2n, (llr < 0).astype(np.uint8)))


def test_rate0_returns_frozen_values():
    n = 1 << 12
    g = np.random.default_rng(10)
    fval = g.integers(0, 2, n).astype(np.uint8)
    llr = g.standard_normal(n).astype(np.float32)
    for bp in (False, True):
        uh, _, _ = oracle.sc_decode(llr, np.ones(n, np.uint8), fval, boxplus=bp)
        assert np.array_equal(uh, fval)


def test_batch_matches_single():
    g = np.random.default_rng(13)
    log2n = 10
    n = 1 << log2n
    mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(0.02), 200)
    llr = np.where(g.random((5, n)) < 0.05, -1.0, 1.0).astype(np.float32)
    fval = (g.integers(0, 2, (5, n)) & mask).astype(np.uint8)
    ub = oracle.sc_decode_batch(llr, mask, fval, n_threads=3)
    for k in range(5):
        u, _, _ = oracle.sc_decode(llr[k], mask, fval[k])
        assert np.array_equal(ub[k], u)
