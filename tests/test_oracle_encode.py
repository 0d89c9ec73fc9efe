"""Pins for the oracle encoder x = u G_N (Section 3, Arikan's construction)."""
import numpy as np
import pytest

import oracle
from oracle import naive


@pytest.mark.parametrize("log2n", range(0, 7))
def test_encode_equals_kronecker_matrix(log2n):
    n = 1 << log2n
    g = np.random.default_rng(log2n)
    for _ in range(20):
        u = g.integers(0, 2, n, dtype=np.uint8)
        assert np.array_equal(oracle.encode(log2n, u), naive.encode_matrix(u))


def test_kronecker_matrix_is_lower_triangular_with_unit_diagonal():
    # F^{(x)n} is lower triangular with ones on the diagonal; row i has
    # 2^{popcount(i)} ones.
    for log2n in range(0, 7):
        gm = naive.kron_g(log2n)
        assert np.array_equal(np.triu(gm, 1), np.zeros_like(gm))
        assert np.all(np.diag(gm) == 1)
        for i in range(1 << log2n):
            assert gm[i].sum() == 1 << bin(i).count("1")


@pytest.mark.parametrize("log2n", [1, 5, 10, 16, 20])
def test_encode_is_an_involution(log2n):
    n = 1 << log2n
    u = np.random.default_rng(100 + log2n).integers(0, 2, n, dtype=np.uint8)
    x = oracle.encode(log2n, u)
    assert np.array_equal(oracle.encode(log2n, x), u)


def test_encode_unit_vectors_give_matrix_rows():
    log2n = 6
    gm = naive.kron_g(log2n)
    for i in range(64):
        e = np.zeros(64, np.uint8)
        e[i] = 1
        assert np.array_equal(oracle.encode(log2n, e), gm[i].astype(np.uint8))


def test_encode_linear():
    g = np.random.default_rng(7)
    for log2n in (3, 9, 12):
        n = 1 << log2n
        a = g.integers(0, 2, n, dtype=np.uint8)
        b = g.integers(0, 2, n, dtype=np.uint8)
        assert np.array_equal(oracle.encode(log2n, a ^ b), oracle.encode(log2n, a) ^ oracle.encode(log2n, b))
