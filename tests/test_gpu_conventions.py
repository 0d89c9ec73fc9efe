"""GPU tests of the boundary's documented conventions (include/polar.h):
bits of frozen_vals outside the mask are ignored, u-hat of N < 32 leaves the
unused bits of its word zero, subnormal channel LLRs stay bit-exact under
min-sum (denormals are preserved on both sides), and one batch may mix
check updates and leaf-dump requests."""
import sys

import numpy as np
import pytest

import oracle

from gpu_helpers import (bits_host, bsc_frames, check_boxplus_decisions, check_boxplus_leaves, decode,
                         frame_items, random_frames, words_dev)

pytestmark = pytest.mark.gpu


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


def _decode_raw_vals(frames, raw_vals, f_kind):
    """Decode with frozen_vals words taken from raw_vals (bits outside the
    mask set at random) instead of the masked values."""
    import torch
    from paper_1204_5882_amd import polar as lp

    items = frame_items(frames, f_kind)
    for it, rv in zip(items, raw_vals):
        it["frozen_vals"] = words_dev(rv)
    ctx = lp.Ctx(0)
    ctx.decode(items)
    torch.cuda.synchronize()
    us = [bits_host(it["u_hat"], it["llr"].numel()) for it in items]
    ctx.close()
    return us


@pytest.mark.parametrize("log2n", [2, 5, 6, 9, 13, 16])
def test_frozen_vals_outside_mask_ignored(log2n):
    g = np.random.default_rng(1300 + log2n)
    frames = random_frames(log2n, g, 7)
    raw = [(fr[2] | (g.integers(0, 2, fr[2].size).astype(np.uint8) & (1 - fr[1]))).astype(np.uint8)
           for fr in frames]
    assert any((r != fr[2]).any() for r, fr in zip(raw, frames))
    refs = [oracle.sc_decode(*fr)[0] for fr in frames]
    _say(f"case: out-of-mask frozen-value bits, min-sum log2n={log2n}")
    us = _decode_raw_vals(frames, raw, 0)
    for k in range(len(frames)):
        assert np.array_equal(us[k], refs[k]), k
    _say(f"case: out-of-mask frozen-value bits, box-plus log2n={log2n}")
    us = _decode_raw_vals(frames, raw, 1)
    check_boxplus_decisions(frames, us, "raw frozen values")


@pytest.mark.parametrize("log2n", [1, 2, 3, 4])
def test_small_frames_leave_unused_word_bits_zero(log2n):
    import torch

    from paper_1204_5882_amd import polar as lp

    g = np.random.default_rng(1400 + log2n)
    frames = random_frames(log2n, g, 8)
    items = frame_items(frames)   # u_hat words start as all ones
    ctx = lp.Ctx(0)
    ctx.decode(items)
    torch.cuda.synchronize()
    n = 1 << log2n
    for it, fr in zip(items, frames):
        w = int(it["u_hat"].cpu().numpy().view(np.uint32)[0])
        assert w >> n == 0, hex(w)
        assert np.array_equal(bits_host(it["u_hat"], n), oracle.sc_decode(*fr)[0])
    ctx.close()


@pytest.mark.parametrize("log2n", [4, 8, 12, 15])
def test_subnormal_llrs_minsum_bit_exact(log2n):
    """Channel LLRs of subnormal magnitude (and zeros, and a few normals):
    every min-sum f is a min and every g one FP32 addition, so u-hat and the
    leaf LLRs stay bit-exact when denormals are preserved."""
    g = np.random.default_rng(1500 + log2n)
    n = 1 << log2n
    tiny = np.float32(1.4e-45)  # smallest positive subnormal
    frames = []
    for k in range(4):
        mult = g.integers(-2000, 2001, n).astype(np.float32)
        llr = (mult * tiny).astype(np.float32)
        if k % 2:
            normal = g.random(n) < 0.05
            llr[normal] = g.standard_normal(int(normal.sum())).astype(np.float32) * np.float32(1e-37)
        assert (np.abs(llr[llr != 0]) < np.float32(1.18e-38)).mean() > 0.7  # mostly subnormal
        mask = (g.random(n) < [0.0, 0.3, 0.5, 0.7][k]).astype(np.uint8)
        fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
        frames.append((llr, mask, fval))
    refs = [oracle.sc_decode(*fr, want_leaf=True) for fr in frames]
    for prune in (True, False):
        _say(f"case: subnormal LLRs log2n={log2n} prune={prune}")
        us, _ = decode(frames, prune=prune)
        for k in range(len(frames)):
            assert np.array_equal(us[k], refs[k][0]), (prune, k)
    _say(f"case: subnormal LLRs log2n={log2n} leaf dump")
    us, leaves = decode(frames, prune=False, dump=True)
    for k in range(len(frames)):
        assert np.array_equal(us[k], refs[k][0])
        assert np.all(leaves[k] == refs[k][1]), k


def test_batch_mixing_check_updates_and_dumps():
    """One polar_sc_decode_batch call holding min-sum and box-plus frames,
    with and without leaf dumps, of several sizes: four launches share the
    workspace's counter and slot area, and each frame must come out as it
    does alone."""
    import torch

    from paper_1204_5882_amd import polar as lp

    g = np.random.default_rng(1600)
    frames, kinds, dumps = [], [], []
    for k in range(16):
        log2n = [6, 11, 13, 15][k % 4]
        fr = (random_frames(log2n, g, 7)[k % 7] if k % 3 else
              bsc_frames(log2n, 0.03, (1 << log2n) // 4, [8000 + k])[0])
        frames.append(fr)
        kinds.append((k // 2) % 2)
        dumps.append(k % 4 in (1, 2))
    items = []
    for fr, fk, dp in zip(frames, kinds, dumps):
        items += frame_items([fr], fk, dp)
    ctx = lp.Ctx(0)
    _say("case: mixed check updates and dumps in one batch")
    ctx.decode(items)
    torch.cuda.synchronize()
    for k, (fr, fk, dp, it) in enumerate(zip(frames, kinds, dumps, items)):
        n = fr[0].size
        u = bits_host(it["u_hat"], n)
        lf = it["leaf_llr"].cpu().numpy() if dp else None
        if fk == 0:
            ref_u, ref_l, _ = oracle.sc_decode(*fr, want_leaf=True)
            assert np.array_equal(u, ref_u), k
            if dp:
                done = ~np.isnan(lf)
                assert np.all(lf[done] == ref_l[done]), k
        else:
            if dp:
                check_boxplus_leaves([fr], [u], [lf], f"mixed batch frame {k}", computed_only=True)
            else:
                check_boxplus_decisions([fr], [u], f"mixed batch frame {k}")
        solo, _ = decode([fr], f_kind=fk, dump=dp)
        assert np.array_equal(solo[0], u), f"frame {k} differs from its solo decode"
    ctx.close()
