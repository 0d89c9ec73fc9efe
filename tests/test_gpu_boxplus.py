"""GPU parity of every box-plus production path against the FP64 oracle.

Box-plus (the exact check update of Section 4, 2 atanh(tanh(a/2) tanh(b/2)))
runs in FP32 on the GPU and in FP64 in the oracle, so decisions are compared
in teacher-forcing mode: the oracle re-runs with the GPU's u-hat as partial
sums, an information bit may differ only where the oracle's leaf LLR has
|L| < 1e-6 (codes built from the channel's Bhattacharyya parameters, the
configured workloads), or lies within the LLR tolerance of zero,
|L_ref| <= 1e-5 S_i (random non-closed masks, whose cancelling sums put
FP32 rounding above 1e-6), and frozen positions must hold the frozen values.
Leaf LLRs, where a dump is taken, must satisfy |dL| <= 1e-5 max(|L_ref|, S_i).

Covered here: the pruned decoder on non-closed random masks (the generic
16/32/64-leaf node paths) at every size and every built cutover, the
cutover 10 / 11 variants the autotuner may choose, the plain decoder, and the
N = 2^24 sixteen-frame workload in the exact launch configuration the
benchmark times.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import (biawgn_frames, check_boxplus_decisions, check_boxplus_leaves, decode,
                         random_frames)

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


@pytest.mark.parametrize("log2n", list(range(1, 17)))
def test_boxplus_pruned_random_masks_every_cutover(log2n):
    """Pruned box-plus on random (non-closed) frozen masks: the generic node
    at 16, 32 and 64 leaves, rate-0 / rate-1 / repetition shortcuts with the
    box-plus floor, LLRs with exact zeros; cutover 10, 11 and 12."""
    from paper_1204_5882_amd import polar as lp

    g = np.random.default_rng(900 + log2n)
    frames = random_frames(log2n, g, 10 if log2n <= 13 else 5)
    for cut in (10, 11, 12):
        _say(f"case: box-plus pruned random masks log2n={log2n} cutover={cut}")
        us, _ = decode(frames, f_kind=1, prune=True, opts={lp.POLAR_OPT_CUTOVER: cut})
        check_boxplus_decisions(frames, us, f"cutover {cut}")
    _say(f"case: box-plus pruned random masks log2n={log2n} leaf dump")
    us, leaves = decode(frames, f_kind=1, prune=True, dump=True)
    check_boxplus_leaves(frames, us, leaves, "pruned dump", computed_only=True)


@pytest.mark.parametrize("cut", [10, 11])
def test_boxplus_smaller_cutover_matches_oracle(cut):
    """The cutover 10 / 11 variants (choices of the autotuner) on
    Bhattacharyya-built codes whose frames reach several HBM levels."""
    from paper_1204_5882_amd import polar as lp

    frames = (biawgn_frames(15, 0.97, 18000, range(7200, 7204))
              + biawgn_frames(16, 1.1, 40000, range(7210, 7213)))
    for waves in (4, 8):
        _say(f"case: box-plus cutover {cut} waves {waves}")
        us, _ = decode(frames, f_kind=1, opts={lp.POLAR_OPT_CUTOVER: cut, lp.POLAR_OPT_WG_WAVES: waves})
        check_boxplus_decisions(frames, us, f"cutover {cut} waves {waves}", strict=True)


@pytest.mark.parametrize("log2n", [3, 6, 9, 12, 14])
def test_boxplus_plain_decoder(log2n):
    """The plain one-frame-per-launch decoder with box-plus."""
    g = np.random.default_rng(950 + log2n)
    frames = random_frames(log2n, g, 6) + biawgn_frames(
        log2n, 0.97, (1 << log2n) - int(0.45 * (1 << log2n)), [6100 + log2n])
    _say(f"case: box-plus plain decoder log2n={log2n}")
    us, _ = decode(frames, f_kind=1, plain=True)
    check_boxplus_decisions(frames, us, "plain")


@pytest.mark.timeout(900)
def test_cfg3_as_benchmarked():
    """N = 2^24, BIAWGN sigma = 0.97, rate 0.45, 16 frames, pruned box-plus
    in the library's default launch configuration (what the benchmark times):
    every frame's decisions teacher-forced against the FP64 oracle, and the
    leaf LLRs of one frame, pruned with the dump, within tolerance."""
    log2n = 24
    nf = (1 << 24) - int(0.45 * (1 << 24))
    frames = biawgn_frames(log2n, 0.97, nf, [3000 + k for k in range(16)])
    _say("case: cfg3 16 frames pruned box-plus")
    us, _ = decode(frames, f_kind=1, prune=True)
    tol, _ = check_boxplus_decisions(frames, us, "cfg3", strict=True)
    print(f"cfg3: {tol} tolerated decision differences over 16 frames")
    _say("case: cfg3 one frame pruned with leaf dump")
    us, leaves = decode(frames[:1], f_kind=1, prune=True, dump=True)
    check_boxplus_leaves(frames[:1], us, leaves, "cfg3 pruned dump", computed_only=True, strict=True)
