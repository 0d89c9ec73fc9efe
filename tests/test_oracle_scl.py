"""Pins of the SC list decoding oracle (oracle.scl_decode), each independent
of its code:
  * L = 1 is SC: equal to oracle.sc_decode on random and Bhattacharyya codes;
  * a per-bit list decoder on naive.py's re-encoding SC (N <= 32) gives the
    same decisions and metric, ties included;
  * with min-sum updates the metric of a complete path equals the
    correlation discrepancy sum_j |L_j| [x_j != (L_j < 0)] of its codeword
    x = u G_N (the max-log maximum-likelihood metric): checked in exact
    arithmetic (LLRs on a coarse dyadic grid) on the returned path at N up to
    2^12;
  * with L >= 2^K every path survives, so the output minimises the
    discrepancy over all 2^K codewords (brute force on small codes);
  * noiseless frames decode correctly at every L.
Planted slips in a copy of the oracle's C source are caught."""
import ctypes
import itertools
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle import naive


def _rand_frame(g, n, dyadic=True):
    frozen = (g.random(n) < g.uniform(0.2, 0.8)).astype(np.uint8)
    fval = (g.integers(0, 2, n) & frozen).astype(np.uint8)
    if dyadic:
        llr = (g.integers(-8, 9, n) * 0.25).astype(np.float32)  # zeros and ties included
    else:
        llr = g.standard_normal(n).astype(np.float32)
    return llr, frozen, fval


def _discrepancy(llr, u):
    x = oracle.encode(int(np.log2(llr.size)), u)
    hard = (llr < 0).astype(np.uint8)
    return float(np.sum(np.abs(llr.astype(np.float64)) * (x != hard)))


@pytest.mark.parametrize("log2n", [0, 1, 3, 6, 9, 12])
def test_list_one_is_sc(log2n):
    g = np.random.default_rng(700 + log2n)
    for k in range(6):
        fr = _rand_frame(g, 1 << log2n, dyadic=k % 2 == 0)
        u_sc = oracle.sc_decode(*fr)[0]
        u_l, _ = oracle.scl_decode(*fr, 1)
        assert np.array_equal(u_sc, u_l)
    if log2n >= 6:
        mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(0.05), (1 << log2n) // 2)
        u, fval, llr = synth.frame(17, log2n, "bsc", 0.05, mask, lambda v: oracle.encode(log2n, v))
        assert np.array_equal(oracle.scl_decode(llr, mask, fval, 1)[0], oracle.sc_decode(llr, mask, fval)[0])


@pytest.mark.parametrize("list_size", [1, 2, 3, 4, 8])
def test_equals_naive_per_bit_list_decoder(list_size):
    g = np.random.default_rng(800 + list_size)
    for _ in range(60):
        n = int(g.choice([1, 2, 4, 8, 16, 32]))
        fr = _rand_frame(g, n, dyadic=bool(g.integers(0, 2)))
        u1, pm1 = oracle.scl_decode(*fr, list_size)
        u2, pm2 = naive.naive_scl(*fr, list_size)
        assert np.array_equal(u1, u2) and pm1 == pm2


@pytest.mark.parametrize("log2n,list_size", [(4, 2), (8, 4), (10, 8), (12, 4)])
def test_metric_is_correlation_discrepancy(log2n, list_size):
    g = np.random.default_rng(900 + log2n)
    for _ in range(4):
        fr = _rand_frame(g, 1 << log2n)
        u, pm = oracle.scl_decode(*fr, list_size)
        assert np.array_equal(u[fr[1] == 1], fr[2][fr[1] == 1])
        assert float(pm) == _discrepancy(fr[0], u)


@pytest.mark.parametrize("log2n", [2, 3, 4])
def test_full_list_is_max_log_ml(log2n):
    g = np.random.default_rng(1000 + log2n)
    n = 1 << log2n
    for _ in range(40):
        k = int(g.integers(0, min(n, 5) + 1))
        frozen = np.ones(n, np.uint8)
        frozen[g.choice(n, k, replace=False)] = 0
        fval = (g.integers(0, 2, n) & frozen).astype(np.uint8)
        llr = (g.integers(-8, 9, n) * 0.25).astype(np.float32)
        u, pm = oracle.scl_decode(llr, frozen, fval, 1 << k)
        info = np.flatnonzero(frozen == 0)
        best = np.inf
        for bits in itertools.product((0, 1), repeat=k):
            uu = fval.copy()
            uu[info] = bits
            best = min(best, _discrepancy(llr, uu))
        assert float(pm) == best == _discrepancy(llr, u)


@pytest.mark.parametrize("list_size", [1, 2, 8])
def test_noiseless(list_size):
    log2n = 10
    mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(0.05), 300)
    g = np.random.default_rng(5)
    u = g.integers(0, 2, 1 << log2n).astype(np.uint8)
    x = oracle.encode(log2n, u)
    llr = np.where(x == 1, -2.0, 2.0).astype(np.float32)
    got, pm = oracle.scl_decode(llr, mask, u & mask, list_size)
    assert np.array_equal(got, u) and pm == 0.0


SRC = os.path.join(os.path.dirname(oracle.__file__), "sc_oracle.c")
PLANTS = {
    "penalty_on_agreement": ("if (b != (lam[k] < 0.0f)) c.pm = cur[k].pm + fabsf(lam[k]);",
                             "if (b == (lam[k] < 0.0f)) c.pm = cur[k].pm + fabsf(lam[k]);"),
    "frozen_no_penalty": ("if (b != (lam[k] < 0.0f)) cur[k].pm = cur[k].pm + fabsf(lam[k]);", ";"),
    "ties_by_bit_descending": ("return x->bit < y->bit;", "return x->bit > y->bit;"),
    "g_without_partial_sums": ("out[j] = g_f32(par[j], par[j + h], beta[j]);", "out[j] = g_f32(par[j], par[j + h], 0);"),
    "best_is_last_min": ("if (cur[k].pm < cur[best].pm) best = k;", "if (cur[k].pm <= cur[best].pm) best = k;"),
}


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = PLANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, str(c), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    lib.oracle_scl_decode.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]

    def mutant(llr, frozen, fval, list_size):
        n = llr.size
        u = np.empty(n, np.uint8)
        pm = ctypes.c_float(0)
        args = [np.ascontiguousarray(a) for a in (llr, frozen, fval)]
        lib.oracle_scl_decode(int(np.log2(n)), list_size, *[P(a.ctypes.data) for a in args], P(u.ctypes.data),
                              ctypes.addressof(pm))
        return u, np.float32(pm.value)

    g = np.random.default_rng(1234)
    caught = False
    for _ in range(300):
        n = int(g.choice([2, 4, 8, 16, 32]))
        fr = _rand_frame(g, n)
        L = int(g.choice([1, 2, 4, 8]))
        got = mutant(*fr, L)
        ref = naive.naive_scl(*fr, L)
        if not (np.array_equal(got[0], ref[0]) and got[1] == ref[1]):
            caught = True
            break
    assert caught, name
