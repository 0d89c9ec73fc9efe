"""Seeded random sweep of the batch decoder against the oracle: each trial
draws a check-update kind (FP32 min-sum, box-plus, 16-bit min-sum, phi table,
8-bit min-sum), launch options (cutover, waves, frames per workgroup, graph
replay, sweep helpers, pruning), a batch of frame sizes, frozen masks (random
density, Bhattacharyya-built, all frozen or none) and channel LLRs (Gaussian,
a coarse grid with exact zeros, BSC).  Min-sum and the fixed-point kinds must
match bit for bit; box-plus by the teacher-forced FP64 rule of the other
box-plus tests."""
import sys

import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import check_boxplus_decisions, decode

pytestmark = pytest.mark.gpu

KINDS = {2: oracle.FIXED_MINSUM, 3: oracle.FIXED_PHI, 4: oracle.FIXED_MINSUM8}  # library f_kind -> oracle kind


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1204_5882_amd import polar as lp

    lp.load()


def _trial(seed):
    from paper_1204_5882_amd import polar as lp

    g = np.random.default_rng(seed)
    fk = int(g.integers(0, 5))
    logs = [int(g.integers(1, (14 if fk == 1 else 17) + 1)) for _ in range(int(g.integers(1, 10)))]
    opts = {lp.POLAR_OPT_CUTOVER: int(g.choice([0, 8, 9, 10, 11, 12])),
            lp.POLAR_OPT_WG_WAVES: int(g.choice([0, 4, 8])),
            lp.POLAR_OPT_FWG: int(g.choice([0, 1, 2, 4])),
            lp.POLAR_OPT_GRAPH: int(g.integers(0, 2)),
            lp.POLAR_OPT_HELPERS: int(g.integers(0, 2))}
    prune = bool(g.integers(0, 4) > 0)
    frames = []
    for log2n in logs:
        n = 1 << log2n
        mk = int(g.integers(0, 4))
        if mk == 0:
            mask = (g.random(n) < g.uniform(0, 1)).astype(np.uint8)
        elif mk == 1:
            mask, _, _ = oracle.frozen_set(log2n, float(g.uniform(0.05, 0.6)), int(g.integers(0, n + 1)))
        elif mk == 2:
            mask = np.full(n, int(g.integers(0, 2)), np.uint8)
        else:
            mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(0.03), n // 4)
        mask = np.asarray(mask, np.uint8)
        fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
        lk = int(g.integers(0, 3))
        if fk >= 2:
            lim = oracle.FIXED8_MAX if fk == 4 else oracle.FIXED_MAX
            l0 = 14 if fk == 4 else 56  # BSC 3% quantized
            llr = (g.integers(-lim, lim + 1, n) if lk == 0 else g.integers(-3, 4, n) if lk == 1
                   else np.where(g.random(n) < 0.05, -l0, l0))
        else:
            llr = (g.standard_normal(n) * float(g.uniform(0.5, 4)) if lk == 0 else g.integers(-8, 9, n) * 0.25
                   if lk == 1 else np.where(g.random(n) < 0.05, -3.476, 3.476))
        frames.append((np.asarray(llr, np.float32), mask, fval))
    return fk, logs, opts, prune, frames


@pytest.mark.parametrize("block", range(8))
def test_random_kinds_options_and_batches_match_oracle(block):
    for seed in range(block * 200, block * 200 + 200):
        fk, logs, opts, prune, frames = _trial(seed)
        what = f"seed {seed}: f_kind {fk}, prune {int(prune)}, log2n {logs}, options {opts}"
        print(what, flush=True)
        sys.stdout.flush()
        us, _ = decode(frames, f_kind=fk, prune=prune, opts=opts)
        if fk == 1:
            check_boxplus_decisions(frames, us, what=what)
            continue
        for k, ((llr, mask, fval), u) in enumerate(zip(frames, us)):
            if fk == 0:
                ref = oracle.sc_decode(llr, mask, fval)[0]
            else:
                ref = oracle.sc_decode_fixed(llr.astype(np.int32), mask, fval, KINDS[fk])[0]
            assert np.array_equal(u, ref), f"{what}: frame {k} differs in {int((u != ref).sum())} bits"
