"""CPU proofs of the exact shortcuts the GPU decoder takes, before any GPU runs them.

1. Rate-0 node (every leaf frozen): its partial sums are the frozen values
   re-encoded, beta = v G_m, with no LLR work.
2. Rate-1 node (no leaf frozen), FP32 min-sum: the partial sums depend only on
   the sign / zero state of the node's input LLRs.  Hard decisions are NOT SC
   when exact zeros occur (alpha = (0, -1) gives x-hat = (1, 1)), so the rule
   is the three-state recursion, written here on 64-bit words exactly as the
   kernel evaluates it:
       left:  S_L = S_lo ^ S_hi,  Z_L = Z_lo | Z_hi
       right: Z_R = Z_lo & Z_hi,  S_R = Z_hi ? (S_lo ^ beta_L) : S_hi
       beta = [beta_L ^ beta_R, beta_R];  leaf: beta = S & ~Z
   with the early exit "no zeros -> beta = S".
3. The in-word polar transform x ^= (x >> h) & LOW_h for h = 1..32.
4. Repetition node (every leaf frozen but the last): the last leaf's LLR is
   the g chain down the right spine, the left sibling of size h at offset o
   contributing the partial sums W_h[o, o + h) of the frozen values, W_h being
   the frozen word with G_h applied inside every aligned h-block; the node's
   partial sums are then G over (frozen values, decision).
Each is checked against the plain oracle (no shortcuts)."""
import itertools

import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1
LOW = {1: 0x5555555555555555, 2: 0x3333333333333333, 4: 0x0F0F0F0F0F0F0F0F,
       8: 0x00FF00FF00FF00FF, 16: 0x0000FFFF0000FFFF, 32: 0x00000000FFFFFFFF}


def nodemask(o, m):
    return (((1 << m) - 1) << o) & M64


def word_transform(x, m):
    for h in (1, 2, 4, 8, 16, 32):
        if h >= m:
            break
        x ^= (x >> h) & LOW[h]
    return x


def rate1_beta(S, Z, o, m):
    nm = nodemask(o, m)
    if Z & nm == 0:
        return S & nm
    if m == 1:
        return S & ~Z & nm
    h = m // 2
    lo = nodemask(o, h)
    SL = (S ^ (S >> h)) & lo
    ZL = (Z | (Z >> h)) & lo
    bL = rate1_beta(SL, ZL, o, h)
    Zhi = Z >> h
    Shi = S >> h
    ZR = (Z & Zhi) & lo
    SR = ((Zhi & (S ^ bL)) | (~Zhi & Shi)) & lo
    bR = rate1_beta((SR << h) & M64, (ZR << h) & M64, o + h, h)
    return (bL ^ (bR >> h)) | bR


def _to_word(bits, o=0):
    w = 0
    for i, b in enumerate(bits):
        w |= int(b) << (o + i)
    return w


def _sign_zero(llr, o=0):
    S = _to_word([v < 0 for v in llr], o)
    Z = _to_word([v == 0 for v in llr], o)
    return S, Z


@pytest.mark.parametrize("m", [1, 2, 4, 8])
def test_rate1_three_state_exhaustive(m):
    g = np.random.default_rng(m)
    for pattern in itertools.product((-1, 0, 1), repeat=m):
        mag = (0.5 + g.random(m)).astype(np.float32)
        llr = (np.array(pattern, np.float32) * mag).astype(np.float32)
        _, _, beta = oracle.sc_decode(llr, np.zeros(m, np.uint8), np.zeros(m, np.uint8), want_beta=True)
        for o in (0, 64 - m):
            S, Z = _sign_zero(llr, o)
            assert rate1_beta(S, Z, o, m) == _to_word(beta, o), (pattern, o)


@pytest.mark.parametrize("m", [16, 32, 64])
def test_rate1_three_state_random(m):
    g = np.random.default_rng(100 + m)
    for trial in range(400):
        pz = [0.0, 0.05, 0.3, 0.7][trial % 4]
        llr = (g.integers(-3, 4, m) * (1 + g.random(m))).astype(np.float32)
        llr[g.random(m) < pz] = 0.0
        _, _, beta = oracle.sc_decode(llr, np.zeros(m, np.uint8), np.zeros(m, np.uint8), want_beta=True)
        o = 0 if m == 64 else int(g.integers(0, 64 // m)) * m
        S, Z = _sign_zero(llr, o)
        assert rate1_beta(S, Z, o, m) == _to_word(beta, o)


def test_rate1_no_zero_is_hard_decision():
    g = np.random.default_rng(5)
    for _ in range(200):
        llr = (g.standard_normal(64)).astype(np.float32)
        llr[llr == 0] = 1.0
        _, _, beta = oracle.sc_decode(llr, np.zeros(64, np.uint8), np.zeros(64, np.uint8), want_beta=True)
        assert np.array_equal(beta, (llr < 0).astype(np.uint8))


def test_rate0_beta_is_reencoded_frozen_values():
    g = np.random.default_rng(6)
    for m in (1, 2, 4, 8, 16, 32, 64):
        for _ in range(20):
            v = g.integers(0, 2, m).astype(np.uint8)
            llr = g.standard_normal(m).astype(np.float32)
            u, _, beta = oracle.sc_decode(llr, np.ones(m, np.uint8), v, want_beta=True)
            assert np.array_equal(u, v)
            assert word_transform(_to_word(v), m) == _to_word(beta)


def test_word_transform_is_the_encoder():
    g = np.random.default_rng(7)
    for m in (1, 2, 4, 8, 16, 32, 64):
        for _ in range(20):
            u = g.integers(0, 2, m).astype(np.uint8)
            x = oracle.encode(m.bit_length() - 1, u)
            assert word_transform(_to_word(u), m) == _to_word(x)


def rep_node_model(llr, fval):
    """The repetition-node shortcut on a node of size m at offset 0."""
    m = llr.size
    V = _to_word(fval[:-1])
    W = [V]
    h = 1
    while h < m:
        W.append(W[-1] ^ ((W[-1] >> h) & LOW[h]))
        h *= 2
    x = [np.float32(v) for v in llr]
    h = m // 2
    while h >= 1:
        lg = h.bit_length() - 1
        ol = m - 2 * h
        sib = (W[lg] >> ol) & ((1 << h) - 1)
        for j in range(h):
            a, b = x[ol + j], x[ol + h + j]
            x[ol + h + j] = np.float32(b - a) if (sib >> j) & 1 else np.float32(b + a)
        h //= 2
    last = x[m - 1]
    u = int(last < 0)
    return word_transform(V | (u << (m - 1)), m), last


@pytest.mark.parametrize("m", [2, 4, 8, 16, 32, 64])
def test_repetition_node_shortcut(m):
    g = np.random.default_rng(200 + m)
    mask = np.ones(m, np.uint8)
    mask[-1] = 0
    for trial in range(300):
        llr = (g.integers(-3, 4, m) * (0.5 + g.random(m))).astype(np.float32)
        if trial % 3 == 0:
            llr[g.random(m) < 0.3] = 0.0
        fval = (g.integers(0, 2, m) & mask).astype(np.uint8)
        _, leaf, beta = oracle.sc_decode(llr, mask, fval, want_leaf=True, want_beta=True)
        got_beta, last = rep_node_model(llr, fval)
        assert got_beta == _to_word(beta)
        assert np.float32(last).view(np.uint32) == leaf[-1].view(np.uint32)


# ---------------------------------------------------------------------------
# Straight-line small-node decoders: the kernel compiles one per frozen
# pattern of an aligned 8- or 16-leaf node that is closed under the order of
# the synthetic channels.  Check that its case list is exactly that closed
# family, and that every aligned node of Bhattacharyya-built codes has one.
# ---------------------------------------------------------------------------
import os
import re

import synth

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_1204_5882_amd", "csrc", "sc_kernels.h")


def _weaker(j, m):
    """Indices whose Bhattacharyya parameter is at least Z_j by one step:
    drop a 1 of j, or move a 1 one place towards the least significant bit."""
    out = []
    for b in range(m):
        if (j >> b) & 1:
            out.append(j & ~(1 << b))
            if b > 0 and not (j >> (b - 1)) & 1:
                out.append((j & ~(1 << b)) | (1 << (b - 1)))
    return out


def closed_patterns(m):
    size = 1 << m
    res = []
    for F in range(1 << size):
        if all((F >> i) & 1 for j in range(size) if (F >> j) & 1 for i in _weaker(j, m)):
            res.append(F)
    return res


def _kernel_cases():
    src = open(SRC).read()
    body = src[src.index("__device__ __forceinline__ uint32_t spec_local"):]
    body = body[: body.index("\n}\n")]
    m16, m8 = body.split("} else {", 1)
    grab = lambda t: sorted(int(x, 16) for x in re.findall(r"case (0x[0-9a-f]+):", t))
    return {3: grab(m8), 4: grab(m16)}


def test_closed_pattern_counts():
    # 3 patterns of 2 leaves (FF, FI, II), 5 of 4, 10 of 8, 27 of 16
    assert [len(closed_patterns(m)) for m in (1, 2, 3, 4)] == [3, 5, 10, 27]


@pytest.mark.parametrize("m", [3, 4])
def test_kernel_specializes_exactly_the_closed_patterns(m):
    assert _kernel_cases()[m] == closed_patterns(m)


@pytest.mark.parametrize("log2n,z0,n_frozen", [
    (12, synth.bsc_z0(0.02), 819),
    (16, synth.bsc_z0(0.05), -1),
    (20, synth.bsc_z0(0.03), 262144),
    (18, synth.biawgn_z0(0.97), -1),
])
def test_every_aligned_node_of_real_codes_is_closed(log2n, z0, n_frozen):
    mask, _, _ = oracle.frozen_set(log2n, z0, n_frozen)
    for m in (3, 4):
        closed = set(closed_patterns(m))
        rows = mask.reshape(-1, 1 << m).astype(np.uint64)
        pats = (rows << np.arange(1 << m, dtype=np.uint64)).sum(axis=1)
        assert set(int(p) for p in np.unique(pats)) <= closed


def _is_closed(F, m):
    size = 1 << m
    return all((F >> i) & 1 for j in range(size) if (F >> j) & 1 for i in _weaker(j, m))


def test_hot_32_and_64_leaf_cases_are_closed_patterns():
    """The straight-line 32- and 64-leaf cases of the generic node must be
    closed patterns too (a non-closed one could never occur in these codes)."""
    src = open(SRC).read()
    body = src[src.index("__device__ __forceinline__ void blk_node("):]
    body = body[: body.index("} else if constexpr (PRUNE && M == SPEC_M)")]
    p64 = [int(x, 16) for x in re.findall(r"case (0x[0-9a-f]+)ull:", body)]
    p32 = [int(x, 16) for x in re.findall(r"case (0x[0-9a-f]+)u:", body)]
    assert len(p64) >= 3 and len(p32) >= 3
    assert all(_is_closed(p, 6) for p in p64)
    assert all(_is_closed(p, 5) for p in p32)


def test_hot_patterns_cover_most_mixed_blocks():
    """The specialized 64-leaf cases cover most mixed blocks of the benchmark's
    code (N = 2^20, BSC 0.03, rate 0.75): a performance property, checked so
    that a change of the construction that shifts the patterns is noticed.
    Codes of other rates have other frequent patterns and take the generic
    node more often (still exact)."""
    log2n, z0, n_frozen = 20, synth.bsc_z0(0.03), 262144
    src = open(SRC).read()
    body = src[src.index("__device__ __forceinline__ void blk_node("):]
    body = body[: body.index("} else if constexpr (PRUNE && M == SPEC_M)")]
    p64 = {int(x, 16) for x in re.findall(r"case (0x[0-9a-f]+)ull:", body)}
    mask, _, _ = oracle.frozen_set(log2n, z0, n_frozen)
    rows = mask.reshape(-1, 64).astype(np.uint64)
    pats = (rows << np.arange(64, dtype=np.uint64)).sum(axis=1)
    full = np.uint64(0xFFFFFFFFFFFFFFFF)
    mixed = [int(p) for p in pats if p not in (0, full, full >> np.uint64(1))]
    assert sum(p in p64 for p in mixed) / len(mixed) > 0.5


# ---------------------------------------------------------------------------
# Rate-1 floor of the phi-table update (fixed point, units of 2^-4): with
# every input magnitude at or above 67 the table update is min(|a|, |b|)
# (T[i] = 0 for i >= 67, so the sum of lookups is 0 and T[0] caps nothing),
# which keeps the bound, and g in a rate-1 node adds two terms of one sign:
# the partial sums are the hard decisions.  Below it they need not be.
# ---------------------------------------------------------------------------
PHI_FLOOR = 67


def _kernel_phi_floor():
    src = open(SRC).read()
    body = src[src.index("constexpr float rate1_floor(int L)"):]
    body = body[: body.index("\n}\n")]
    return float(re.search(r":\s*([0-9.]+)f;", body).group(1))


def test_phi_floor_from_the_table():
    t = oracle.phi_table()
    assert t[PHI_FLOOR - 1] > 0 and np.all(t[PHI_FLOOR:] == 0)
    # the least bound B with f(a, b) >= B whenever |a|, |b| >= B
    closed = [b for b in range(1, t.size) if oracle.f_fixed(oracle.FIXED_PHI, b, b) >= b]
    assert closed[0] == PHI_FLOOR
    assert oracle.f_fixed(oracle.FIXED_PHI, PHI_FLOOR - 1, PHI_FLOOR - 1) == 44
    g = np.random.default_rng(11)
    for a, b in itertools.chain(itertools.product(range(PHI_FLOOR, PHI_FLOOR + 200), (PHI_FLOOR, 300)),
                                g.integers(PHI_FLOOR, oracle.FIXED_MAX + 1, (2000, 2))):
        for sa, sb in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
            assert oracle.f_fixed(oracle.FIXED_PHI, sa * int(a), sb * int(b)) == sa * sb * min(int(a), int(b))
    # the kernel descends every rate-1 node with an input magnitude <= its floor
    assert _kernel_phi_floor() == PHI_FLOOR - 1


@pytest.mark.parametrize("m", [2, 8, 64, 1024])
def test_phi_rate1_above_floor_is_hard_decision(m):
    g = np.random.default_rng(300 + m)
    zero = np.zeros(m, np.uint8)
    for trial in range(60):
        mag = g.choice([PHI_FLOOR, PHI_FLOOR + 1, 100, 1000, oracle.FIXED_MAX], m) if trial % 2 else \
            g.integers(PHI_FLOOR, oracle.FIXED_MAX + 1, m)
        llr = (mag * (1 - 2 * g.integers(0, 2, m))).astype(np.int32)
        u, _ = oracle.sc_decode_fixed(llr, zero, zero, oracle.FIXED_PHI)
        x = oracle.encode(m.bit_length() - 1, u)
        assert np.array_equal(x, (llr < 0).astype(np.uint8))


def test_phi_rate1_below_floor_is_not_hard_decision():
    # f(1, -1) = -0 decides 0, then g = -1 + 1 = 0 decides 0: x-hat = (0, 0), hard (0, 1)
    u, _ = oracle.sc_decode_fixed(np.array([1, -1], np.int32), np.zeros(2, np.uint8), np.zeros(2, np.uint8),
                                  oracle.FIXED_PHI)
    assert oracle.encode(1, u).tolist() == [0, 0]
    g = np.random.default_rng(12)
    differs = 0
    for _ in range(200):
        llr = (g.integers(1, PHI_FLOOR, 64) * (1 - 2 * g.integers(0, 2, 64))).astype(np.int32)
        u, _ = oracle.sc_decode_fixed(llr, np.zeros(64, np.uint8), np.zeros(64, np.uint8), oracle.FIXED_PHI)
        differs += not np.array_equal(oracle.encode(6, u), (llr < 0).astype(np.uint8))
    assert differs > 0


# ---------------------------------------------------------------------------
# Rate-1 floor of exact box-plus: with every input magnitude of a node of
# 2^L leaves at least F_L, every exact LLR inside the node is at least 1e-5
# (the smallest lies on the left spine, x -> f(x, x) applied L times), so SC
# takes the hard decisions.  The kernel's table holds F_L rounded up.
# ---------------------------------------------------------------------------
def _kernel_boxplus_floor():
    src = open(SRC).read()
    body = src[src.index("constexpr float BOXPLUS_FLOOR[13]"):]
    body = body[body.index("{") + 1: body.index("}")]
    return [float(x.strip().rstrip("f")) for x in body.split(",")]


def _spine_threshold(L, target="1e-5"):
    import mpmath as mp

    mp.mp.dps = 50
    f = lambda x: 2 * mp.atanh(mp.tanh(x / 2) ** 2)  # noqa: E731
    lo, hi = mp.mpf(0), mp.mpf(20)
    for _ in range(120):
        mid = (lo + hi) / 2
        x = mid
        for _ in range(L):
            x = f(x)
        if x >= mp.mpf(target):
            hi = mid
        else:
            lo = mid
    return float(hi)


def test_boxplus_floor_table_is_tight_and_safe():
    table = _kernel_boxplus_floor()
    assert len(table) == 13 and table[0] == 0.0
    for L in range(1, 13):
        t = _spine_threshold(L)
        assert t <= table[L] < t + 0.02, (L, t, table[L])
    assert all(b > a for a, b in zip(table, table[1:]))


@pytest.mark.parametrize("L", [1, 3, 6, 9, 12])
def test_boxplus_rate1_above_floor_is_hard_decision(L):
    table = _kernel_boxplus_floor()
    g = np.random.default_rng(400 + L)
    m = 1 << L
    zero = np.zeros(m, np.uint8)
    for trial in range(20 if L < 12 else 4):
        mag = table[L] + (g.exponential(0.5, m) if trial % 2 else np.where(g.random(m) < 0.7, 0.0, g.random(m)))
        llr = (mag * (1 - 2 * g.integers(0, 2, m))).astype(np.float32)
        llr = np.where(np.abs(llr) < table[L], np.copysign(np.float32(table[L]), llr), llr).astype(np.float32)
        u, leaf, beta = oracle.sc_decode(llr, zero, zero, boxplus=True, want_leaf=True, want_beta=True)
        assert np.array_equal(beta, (llr < 0).astype(np.uint8))
        assert np.abs(leaf).min() >= 1e-5 * 0.99


def test_boxplus_below_floor_can_reach_tiny_llrs():
    # inputs at half the floor drive the left spine far below 1e-5
    table = _kernel_boxplus_floor()
    m = 1 << 6
    llr = np.full(m, table[6] / 2, np.float32)
    _, leaf, _ = oracle.sc_decode(llr, np.zeros(m, np.uint8), np.zeros(m, np.uint8), boxplus=True, want_leaf=True)
    assert np.abs(leaf).min() < 1e-5
