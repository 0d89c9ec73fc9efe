"""Pins of the degrading construction oracle (oracle/construct.py) against
facts fixed independently of it: the exact Bhattacharyya recursion on the
BEC (which the degrading construction must reproduce at any N, since a BEC
stays a two-output BEC under both steps and under binning), brute-force
error probabilities of every synthetic channel of BSC codes with N <= 8,
capacity conservation of the polar transform, and the defining properties
of a merge (error probability kept, capacity never raised).  Planted slips
in a copy of the oracle's steps are caught by these pins."""
import numpy as np
import pytest

import oracle
from oracle import construct as C


@pytest.mark.parametrize("log2n", [1, 4, 10, 14])
@pytest.mark.parametrize("eps", [0.05, 0.3, 0.5, 0.8])
def test_bec_equals_bhattacharyya_recursion(log2n, eps):
    pe = C.synthetic_error_probabilities(log2n, C.bec(eps), 16)
    lz, _ = oracle.bhattacharyya(log2n, eps)
    half_z = np.exp(lz) / 2.0
    # linear-domain products against the log-domain recursion: rounding grows
    # by about one ulp per level; below 1e-280 both sides are near underflow
    big = half_z > 1e-280
    assert np.allclose(pe[big], half_z[big], rtol=1e-10, atol=0)
    assert np.all(pe[~big] < 1e-279)


@pytest.mark.parametrize("log2n", [1, 2, 3])
@pytest.mark.parametrize("p", [0.02, 0.11, 0.3])
def test_bsc_unmerged_equals_brute_force(log2n, p):
    exact = C.brute_force_error_probabilities(log2n, p)
    pe = C.synthetic_error_probabilities(log2n, C.bsc(p), 1 << 30)
    assert np.allclose(pe, exact, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("mu", [2, 4, 8, 16])
def test_merged_is_upper_bound_of_brute_force(mu):
    for p in (0.02, 0.11):
        exact = C.brute_force_error_probabilities(3, p)
        pe = C.synthetic_error_probabilities(3, C.bsc(p), mu)
        assert np.all(pe >= exact * (1 - 1e-12)), (p, mu)


def test_brute_force_matches_bsc_closed_forms():
    # N = 2: P_e(W-) = 2p(1-p) (xor of two BSC outputs), P_e(W+) = p^2 + p(1-p)
    # (both copies wrong, or a tie between them broken the wrong way half the time)
    for p in (0.02, 0.11, 0.3):
        bf = C.brute_force_error_probabilities(1, p)
        assert np.isclose(bf[0], 2 * p * (1 - p), rtol=1e-14)
        assert np.isclose(bf[1], p * p + p * (1 - p), rtol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_polar_step_conserves_capacity_and_mass(seed):
    g = np.random.default_rng(seed)
    m = 7
    a = g.random(m)
    b = a * g.random(m)
    w = np.stack([a, b], 1)
    w /= w.sum()
    wm, wp = C.minus(w), C.plus(w)
    assert np.isclose(wm.sum(), 1.0, rtol=1e-14) and np.isclose(wp.sum(), 1.0, rtol=1e-14)
    assert np.all(wm[:, 0] >= wm[:, 1]) and np.all(wp[:, 0] >= wp[:, 1])
    assert np.isclose(C.capacity(wm) + C.capacity(wp), 2 * C.capacity(w), rtol=1e-12)
    # the minus channel is worse and the plus channel better than W
    assert C.capacity(wm) <= C.capacity(w) <= C.capacity(wp)


@pytest.mark.parametrize("mu", [2, 3, 8, 64])
def test_merge_keeps_error_probability_and_degrades(mu):
    g = np.random.default_rng(mu)
    a = g.random(500)
    b = a * g.random(500)
    w = np.stack([a, b], 1)
    w /= w.sum()
    wq = C.merge(w, mu)
    assert wq.shape[0] <= mu
    assert np.isclose(C.error_probability(wq), C.error_probability(w), rtol=1e-13)
    assert C.capacity(wq) <= C.capacity(w) + 1e-15
    # binning on entropy loses at most 1/mu bit (each bin spans 1/mu of entropy)
    assert C.capacity(w) - C.capacity(wq) <= 1.0 / mu + 1e-12


@pytest.mark.parametrize("index", [0, 1, 77, 200, 255])
def test_single_channel_path_equals_full_tree(index):
    w0 = C.bsc(0.05)
    full = C.synthetic_error_probabilities(8, w0, 8)
    assert C.channel_error_probability(8, index, w0, 8) == full[index]


def test_frozen_from_pe_union_bound_and_ties():
    pe = np.array([0.3, 0.01, 0.01, 0.001, 0.2, 0.02, 0.02, 1e-5])
    mask, nf = C.frozen_from_pe(pe, -1, 0.035)
    # best first: 7 (1e-5), 3 (.001), 1 (.01), 2 (.01) -> 0.02101; 5 (.02) would exceed
    assert nf == 4 and list(np.flatnonzero(mask == 0)) == [1, 2, 3, 7]
    mask, nf = C.frozen_from_pe(pe, 5)
    # worst first: 0, 4, then the tie 5/6 freezes the lower index first, then 6, then 1
    assert list(np.flatnonzero(mask)) == [0, 1, 4, 5, 6]


def test_bsc_degrading_beats_bhattacharyya_rate():
    """At the FER-0.1 union bound, the degraded error probabilities (upper
    bounds on P_e, tighter than Z) admit at least as many information bits
    as the Bhattacharyya bound on BSC 2% at N = 2^12."""
    p = 0.02
    pe = C.synthetic_error_probabilities(12, C.bsc(p), 32)
    _, nf_deg = C.frozen_from_pe(pe, -1, 0.1)
    _, nf_z, _ = oracle.frozen_set(12, 2 * np.sqrt(p * (1 - p)), -1, 0.1)
    assert nf_deg <= nf_z


PLANTS = {
    "minus_drops_bb": lambda w: np.stack([(w[:, 0][:, None] * w[:, 0][None, :]).reshape(-1),
                                          (w[:, 0][:, None] * w[:, 1][None, :]
                                           + w[:, 1][:, None] * w[:, 0][None, :]).reshape(-1)], 1),
    "plus_drops_cross": lambda w: np.stack([(w[:, 0][:, None] * w[:, 0][None, :]).reshape(-1),
                                            (w[:, 1][:, None] * w[:, 1][None, :]).reshape(-1)], 1),
}


@pytest.mark.parametrize("name", sorted(PLANTS) + ["children_swapped", "merge_wrong_bin"])
def test_planted_mistake_is_caught(monkeypatch, name):
    if name in PLANTS:
        monkeypatch.setattr(C, name.split("_")[0], PLANTS[name])
    elif name == "children_swapped":
        mi, pl = C.minus, C.plus
        monkeypatch.setattr(C, "minus", pl)
        monkeypatch.setattr(C, "plus", mi)
    else:
        orig_h2 = C.h2
        monkeypatch.setattr(C, "h2", lambda q: orig_h2(np.minimum(2 * np.asarray(q), 0.5)))
    caught = False
    try:
        test_bsc_unmerged_equals_brute_force(3, 0.11)
        test_merged_is_upper_bound_of_brute_force(4)
        test_bec_equals_bhattacharyya_recursion(10, 0.3)
        test_polar_step_conserves_capacity_and_mass(0)
    except AssertionError:
        caught = True
    assert caught, name
