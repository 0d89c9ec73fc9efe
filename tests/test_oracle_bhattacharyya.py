"""Pins for the oracle's Bhattacharyya recursion and frozen-set rule (Section 3).

Independent references used here:
  * exact rationals (fractions.Fraction) for small N;
  * a 50-digit mpmath recursion that carries Z and W = 1 - Z separately
    (minus: Z' = Z (1 + W), W' = W^2; plus: Z' = Z^2, W' = W (1 + Z)), whose
    unbounded exponent removes the saturation of Z at 1 that plain double has;
  * the sum rule Z- + Z+ = 2 Z, so sum_i Z_i = N Z0;
  * the partial order of synthetic channels.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import synth


def _exact_z(log2n, z0: Fraction):
    zs = [z0]
    for _ in range(log2n):
        nxt = []
        for z in zs:
            nxt.append(2 * z - z * z)
            nxt.append(z * z)
        zs = nxt
    return zs


def test_bec_n4_hand_values():
    lz, _ = oracle.bhattacharyya(2, 0.5)
    # Z0 = 1/2: minus/minus 15/16, minus/plus 9/16, plus/minus 7/16, plus/plus 1/16
    assert np.array_equal(np.exp(lz), np.array([0.9375, 0.5625, 0.4375, 0.0625]))


@pytest.mark.parametrize("log2n", [1, 2, 3, 4, 5, 6])
def test_matches_exact_rationals(log2n):
    z0 = Fraction(3, 10)
    exact = _exact_z(log2n, z0)
    lz, lw = oracle.bhattacharyya(log2n, 0.3)
    for i, z in enumerate(exact):
        assert math.isclose(lz[i], math.log(z), rel_tol=1e-13, abs_tol=1e-13)
        assert math.isclose(lw[i], math.log(1 - z), rel_tol=1e-13, abs_tol=1e-13)


def _mp_pairs(log2n, z0):
    mpmath.mp.dps = 50
    zs = [(mpmath.mpf(z0), 1 - mpmath.mpf(z0))]
    for _ in range(log2n):
        nxt = []
        for z, w in zs:
            nxt.append((z * (1 + w), w * w))  # minus
            nxt.append((z * z, w * (1 + z)))  # plus
        zs = nxt
    lz = np.array([float(mpmath.log(z)) for z, _ in zs])
    lw = np.array([float(mpmath.log(w)) for _, w in zs])
    return lz, lw


@pytest.mark.parametrize("log2n,z0", [(10, synth.bsc_z0(0.02)), (12, synth.bsc_z0(0.02)),
                                      (11, synth.biawgn_z0(0.97)), (12, 0.05)])
def test_matches_mpmath_reference(log2n, z0):
    mlz, mlw = _mp_pairs(log2n, z0)
    lz, lw = oracle.bhattacharyya(log2n, z0)
    np.testing.assert_allclose(lz, mlz, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(lw, mlw, rtol=1e-11, atol=1e-12)
    # the frozen set for every cut agrees with the one ranked by mpmath values
    mr = mlw - mlz
    order = np.lexsort((np.arange(len(mr)), mr))
    for nf in (1, len(mr) // 5, 819 if log2n == 12 else len(mr) // 3, len(mr) - 1):
        mask, got, _ = oracle.frozen_set(log2n, z0, nf)
        ref = np.zeros(len(mr), np.uint8)
        ref[order[:nf]] = 1
        assert got == nf
        assert np.array_equal(mask, ref)


@pytest.mark.parametrize("log2n,z0", [(8, 0.5), (14, synth.bsc_z0(0.03)), (16, synth.biawgn_z0(1.2))])
def test_sum_rule(log2n, z0):
    lz, _ = oracle.bhattacharyya(log2n, z0)
    assert math.isclose(np.exp(lz).sum(), (1 << log2n) * z0, rel_tol=1e-12)


@pytest.mark.parametrize("log2n,z0", [(12, synth.bsc_z0(0.02)), (16, synth.biawgn_z0(0.97))])
def test_partial_order(log2n, z0):
    """Z decreases when a 0 bit of the index becomes 1, and when an adjacent
    pattern 01 becomes 10 (plus applied before minus):
    (2z - z^2)^2 - (2 z^2 - z^4) = 2 z^2 (1 - z)^2 >= 0."""
    _, _, r = oracle.frozen_set(log2n, z0, 0)
    n = 1 << log2n
    idx = np.arange(n)
    tol = 1e-9 * np.maximum(1.0, np.abs(r))
    for b in range(log2n):
        lo = idx[(idx >> b) & 1 == 0]
        hi = lo | (1 << b)
        assert np.all(r[hi] >= r[lo] - tol[lo])
    for k in range(log2n - 1):
        sel = idx[((idx >> k) & 3) == 1]           # bits (k+1, k) = 0 1
        swapped = sel ^ (3 << k)                    # -> 1 0
        assert np.all(r[swapped] >= r[sel] - tol[sel])


@pytest.mark.parametrize("log2n,z0,nf", [
    (12, synth.bsc_z0(0.02), 819),
    (20, synth.bsc_z0(0.03), 262144),
])
def test_boundary_is_tie_free(log2n, z0, nf):
    mask, got, r = oracle.frozen_set(log2n, z0, nf)
    assert got == nf and int(mask.sum()) == nf
    gap = r[mask == 0].min() - r[mask == 1].max()
    assert gap > 1e-6


def test_boundary_is_tie_free_n24():
    log2n = 24
    k = int(0.45 * (1 << log2n))
    nf = (1 << log2n) - k
    mask, got, r = oracle.frozen_set(log2n, synth.biawgn_z0(0.97), nf)
    assert got == nf
    gap = r[mask == 0].min() - r[mask == 1].max()
    assert gap > 1e-8


@pytest.mark.parametrize("log2n,z0", [(10, synth.bsc_z0(0.02)), (16, synth.bsc_z0(0.05)),
                                      (16, synth.biawgn_z0(0.8))])
def test_union_bound_rule(log2n, z0):
    mask, nf, _ = oracle.frozen_set(log2n, z0, -1, 0.1)
    lz, _ = oracle.bhattacharyya(log2n, z0)
    z = np.exp(lz)
    info = z[mask == 0]
    frozen = z[mask == 1]
    assert info.sum() <= 0.1
    # the next channel in reliability order would break the bound
    assert info.sum() + frozen.min() > 0.1
    assert info.size == 0 or info.max() <= frozen.min()


def test_invalid_args():
    with pytest.raises(ValueError):
        oracle.frozen_set(4, 0.3, 17)
    with pytest.raises(ValueError):
        oracle.bhattacharyya(4, 1.0)
