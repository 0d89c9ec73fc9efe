"""GPU parity of the fixed-point decoders (Section 4's arithmetic: fixed-point
LLRs, check update from a phi = -ln tanh(x/2) table) against the oracle's
integer implementation: u-hat and every leaf LLR bit-exact, for saturating
min-sum (POLAR_F_MINSUM_Q16), the phi table (POLAR_F_PHI_Q16) and saturating
min-sum on 8-bit integers (POLAR_F_MINSUM_Q8), at every size, pruned and
unpruned, with leaf dumps, at N = 2^20 and 2^24, and the device's phi table
equal to the oracle's."""
import sys

import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import bsc_frames, biawgn_frames, decode

pytestmark = pytest.mark.gpu

KINDS = {2: oracle.FIXED_MINSUM, 3: oracle.FIXED_PHI, 4: oracle.FIXED_MINSUM8}  # library f_kind -> oracle kind


def _lim(fk):
    return oracle.FIXED8_MAX if fk == 4 else oracle.FIXED_MAX


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1204_5882_amd import polar as lp

    lp.load()


def _q(frames, fk=2):
    """Quantize the channel LLRs to units of 2^-4 (the 8-bit kind: 2^-2,
    saturated to 127), kept as float32 integers."""
    frac = 2 if fk == 4 else oracle.FIXED_FRAC
    return [(oracle.quantize(llr, frac, _lim(fk)).astype(np.float32), mask, fval) for llr, mask, fval in frames]


def _random_fixed_frames(log2n, g, count, fk=2):
    n = 1 << log2n
    lim = _lim(fk)
    frac = 2 if fk == 4 else oracle.FIXED_FRAC
    out = []
    for k in range(count):
        kind = k % 4
        if kind == 0:
            l0 = 14 if fk == 4 else 56
            llr = np.where(g.random(n) < 0.1, -l0, l0)                 # BSC 3% quantized
        elif kind == 1:
            llr = g.integers(-lim, lim + 1, n)                         # saturating sums
        elif kind == 2:
            llr = g.integers(-3, 4, n)                                 # zeros, tiny values
        else:
            llr = oracle.quantize(2.0 * ((1 - 2 * g.integers(0, 2, n)) + 0.9 * g.standard_normal(n)) / 0.81,
                                  frac, lim)
        dens = [0.0, 1.0, 0.3, 0.5, 0.7][k % 5]
        mask = (g.random(n) < dens).astype(np.uint8)
        if k % 7 == 6:
            mask, _, _ = oracle.frozen_set(log2n, 0.35, n // 2)
        fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
        out.append((np.asarray(llr, np.float32), mask, fval))
    return out


def _check(frames, fk, us, leaves=None, computed_only=False, what=""):
    for k, ((llr, mask, fval), u) in enumerate(zip(frames, us)):
        ref_u, ref_l = oracle.sc_decode_fixed(llr.astype(np.int32), mask, fval, KINDS[fk], want_leaf=True)
        assert np.array_equal(u, ref_u), f"{what} frame {k}: u-hat differs"
        if leaves is not None:
            lf = leaves[k]
            use = ~np.isnan(lf) if computed_only else np.ones(lf.size, bool)  # pruned nodes write no leaves
            assert np.array_equal(lf[use], ref_l[use].astype(np.float32)), f"{what} frame {k}: leaf LLRs differ"


def test_device_phi_table_equals_oracle_table():
    import torch

    from paper_1204_5882_amd import polar as lp

    t = lp.phi_table()
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle.phi_table().astype(np.float32))


@pytest.mark.parametrize("fk", [2, 3, 4])
@pytest.mark.parametrize("log2n", list(range(1, 17)))
def test_fixed_point_all_sizes_bit_exact(fk, log2n):
    g = np.random.default_rng(3000 + 100 * fk + log2n)
    frames = _random_fixed_frames(log2n, g, 10 if log2n <= 13 else 5, fk)
    for prune in (True, False):
        _say(f"case: fixed f_kind={fk} log2n={log2n} prune={prune}")
        us, _ = decode(frames, f_kind=fk, prune=prune)
        _check(frames, fk, us, what=f"prune={prune}")
    _say(f"case: fixed f_kind={fk} log2n={log2n} leaf dump")
    us, leaves = decode(frames, f_kind=fk, prune=False, dump=True)
    _check(frames, fk, us, leaves, what="dump")
    _say(f"case: fixed f_kind={fk} log2n={log2n} pruned leaf dump")
    us, leaves = decode(frames, f_kind=fk, prune=True, dump=True)
    _check(frames, fk, us, leaves, computed_only=True, what="pruned dump")
    if log2n <= 14:
        _say(f"case: fixed f_kind={fk} log2n={log2n} plain decoder")
        us, _ = decode(frames, f_kind=fk, plain=True)
        _check(frames, fk, us, what="plain")


@pytest.mark.parametrize("fk", [2, 3, 4])
def test_fixed_point_qkd_sizes(fk):
    """N = 2^20 BSC p = 0.03 rate 0.75 (16 frames) and N = 2^16 BIAWGN
    sigma = 0.97 rate 0.45 (8 frames), channel LLRs quantized to 2^-4
    (8-bit kind: 2^-2, saturated to 127)."""
    frames = _q(bsc_frames(20, 0.03, 262144, range(2000, 2016)), fk)
    _say(f"case: fixed f_kind={fk} N = 2^20 x16")
    us, _ = decode(frames, f_kind=fk)
    _check(frames, fk, us, what="2^20")
    frames = _q(biawgn_frames(16, 0.97, (1 << 16) - int(0.45 * (1 << 16)), range(6500, 6508)), fk)
    _say(f"case: fixed f_kind={fk} N = 2^16 BIAWGN x8 with leaf dump")
    us, leaves = decode(frames, f_kind=fk, prune=False, dump=True)
    _check(frames, fk, us, leaves, what="2^16 biawgn")


@pytest.mark.parametrize("fk", [2, 3, 4])
def test_fixed_point_max_size(fk):
    frames = _q(bsc_frames(24, 0.03, (1 << 24) // 4, [7001]), fk)
    _say(f"case: fixed f_kind={fk} N = 2^24")
    us, _ = decode(frames, f_kind=fk)
    _check(frames, fk, us, what="2^24")


def test_fixed_point_mixed_with_float_kinds_in_one_batch():
    """One batch holding all five check updates."""
    import torch

    from gpu_helpers import bits_host, frame_items

    from paper_1204_5882_amd import polar as lp

    g = np.random.default_rng(3500)
    kinds = [k % 5 for k in range(10)]
    frames = [_random_fixed_frames(13, g, k + 1, fk if fk >= 2 else 2)[k] for k, fk in enumerate(kinds)]
    items = []
    for fr, fk in zip(frames, kinds):
        items += frame_items([fr], fk)
    ctx = lp.Ctx(0)
    _say("case: five check updates in one batch")
    ctx.decode(items)
    torch.cuda.synchronize()
    for k, (fr, fk, it) in enumerate(zip(frames, kinds, items)):
        u = bits_host(it["u_hat"], fr[0].size)
        solo, _ = decode([fr], f_kind=fk)
        assert np.array_equal(u, solo[0]), k
        if fk >= 2:
            _check([fr], fk, [u], what=f"mixed frame {k}")
        elif fk == 0:
            assert np.array_equal(u, oracle.sc_decode(*fr)[0])
    ctx.close()


@pytest.mark.parametrize("log2n", [1, 2, 5, 6, 7, 10, 12, 14])
def test_phi_rate1_floor_boundary(log2n):
    """Rate-1 nodes whose input magnitudes sit on both sides of the phi
    update's rate-1 floor (67 in units of 2^-4), so that the kernel's floor
    tests go both ways at every node size, pruned and unpruned."""
    g = np.random.default_rng(3700 + log2n)
    n = 1 << log2n
    mags = np.array([1, 2, 44, 55, 56, 65, 66, 67, 68, 69, 134, 1000])
    frames = []
    for k in range(8):
        if k % 4 == 0:
            mag = g.choice(mags, n)
        elif k % 4 == 1:
            mag = g.choice([66, 67], n)
        elif k % 4 == 2:
            mag = np.where(g.random(n) < 0.02, g.choice([1, 66], n), g.integers(67, 200, n))
        else:
            mag = g.choice([56, 67, 68], n)
        llr = (mag * (1 - 2 * g.integers(0, 2, n))).astype(np.float32)
        mask = np.zeros(n, np.uint8) if k < 4 else (g.random(n) < [0.1, 0.3, 0.5, 0.05][k - 4]).astype(np.uint8)
        fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
        frames.append((llr, mask, fval))
    for prune in (True, False):
        _say(f"case: phi floor log2n={log2n} prune={prune}")
        us, _ = decode(frames, f_kind=3, prune=prune)
        _check(frames, 3, us, what=f"prune={prune}")
    _say(f"case: phi floor log2n={log2n} pruned leaf dump")
    us, leaves = decode(frames, f_kind=3, prune=True, dump=True)
    _check(frames, 3, us, leaves, computed_only=True, what="pruned dump")
