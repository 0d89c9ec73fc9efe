"""Cooperative sweeps: a batch with fewer large frames than resident
workgroups launches the spare workgroups as helpers that share each frame's
large HBM level sweeps.  The sweeps are elementwise, so every value must be
identical with and without helpers: u-hat bit-exact against the oracle
(min-sum, fixed point) and against the helper-free decode (box-plus, with
leaf dumps), on frames large enough that their root sweeps are shared."""
import sys

import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import biawgn_frames, bsc_frames, check_boxplus_decisions, decode

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


def _opts(helpers, cutover=0):
    from paper_1204_5882_amd import polar as lp

    o = {lp.POLAR_OPT_HELPERS: helpers}
    if cutover:
        o[lp.POLAR_OPT_CUTOVER] = cutover
    return o


@pytest.mark.parametrize("log2n,n,cutover", [(20, 3, 11), (22, 2, 10), (19, 5, 9)])
def test_minsum_with_helpers_bit_exact(log2n, n, cutover):
    frames = bsc_frames(log2n, 0.03, (1 << log2n) // 4, [9100 + k for k in range(n)])
    refs = [oracle.sc_decode(*fr)[0] for fr in frames]
    for helpers in (1, 0):
        _say(f"case: min-sum log2n={log2n} frames={n} cutover={cutover} helpers={helpers}")
        us, _ = decode(frames, opts=_opts(helpers, cutover))
        for k in range(n):
            assert np.array_equal(us[k], refs[k]), (helpers, k)


def test_boxplus_with_helpers_equals_without():
    log2n = 22
    frames = biawgn_frames(log2n, 0.97, int((1 << log2n) * 0.55), [9200, 9201])
    _say("case: box-plus log2n=22 x2 with helpers, leaf dump")
    u1, l1 = decode(frames, f_kind=1, dump=True, opts=_opts(1))
    _say("case: box-plus log2n=22 x2 without helpers, leaf dump")
    u0, l0 = decode(frames, f_kind=1, dump=True, opts=_opts(0))
    for k in range(2):
        assert np.array_equal(u1[k], u0[k])
        assert np.array_equal(l1[k], l0[k], equal_nan=True)
    _say("case: box-plus log2n=22 x2 with helpers, pruned")
    u2, _ = decode(frames, f_kind=1, opts=_opts(1))
    check_boxplus_decisions(frames, u2, "box-plus with helpers")


def test_phi_with_helpers_bit_exact():
    log2n = 21
    frames = bsc_frames(log2n, 0.03, (1 << log2n) // 4, [9300, 9301, 9302])
    qframes = [(synth.fixed_point(fr[0]), fr[1], fr[2]) for fr in frames]
    refs = [oracle.sc_decode_fixed(oracle.quantize(fr[0]), fr[1], fr[2], oracle.FIXED_PHI)[0] for fr in frames]
    _say("case: phi table log2n=21 x3 with helpers")
    us, _ = decode(qframes, f_kind=3, opts=_opts(1))
    for k in range(3):
        assert np.array_equal(us[k], refs[k]), k


def test_one_frame_whole_gpu_and_mixed_sizes():
    """One frame per call (every other workgroup a helper), then a batch
    mixing sizes above and below the cutover, min-sum at cutover 11."""
    frames = bsc_frames(21, 0.03, (1 << 21) // 4, [9400])
    frames += bsc_frames(12, 0.03, 1024, [9401, 9402])
    frames += bsc_frames(18, 0.03, (1 << 18) // 4, [9403])
    refs = [oracle.sc_decode(*fr)[0] for fr in frames]
    _say("case: one 2^21 frame with helpers")
    us, _ = decode(frames[:1], opts=_opts(1, 11))
    assert np.array_equal(us[0], refs[0])
    _say("case: mixed sizes with helpers")
    us, _ = decode(frames, opts=_opts(1, 11))
    for k in range(len(frames)):
        assert np.array_equal(us[k], refs[k]), k


def test_q8_with_helpers_bit_exact():
    """8-bit kind, unpruned (the variant that takes helpers): the helpers
    read the int8 level types from the mailbox."""
    log2n = 21
    frames = bsc_frames(log2n, 0.03, (1 << log2n) // 4, [9500, 9501, 9502])
    qframes = [(synth.fixed_point(fr[0], frac=2, limit=127), fr[1], fr[2]) for fr in frames]
    refs = [oracle.sc_decode_fixed(oracle.quantize(fr[0], 2, oracle.FIXED8_MAX), fr[1], fr[2],
                                   oracle.FIXED_MINSUM8)[0] for fr in frames]
    for helpers in (1, 0):
        _say(f"case: 8-bit min-sum log2n=21 x3 unpruned helpers={helpers}")
        us, _ = decode(qframes, f_kind=4, prune=False, opts=_opts(helpers))
        for k in range(3):
            assert np.array_equal(us[k], refs[k]), (helpers, k)
