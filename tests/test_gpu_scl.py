"""GPU parity of SC list decoding (polar_scl_decode_batch) with the oracle
(oracle.scl_decode): decisions and the chosen path's metric, exactly, for
list sizes 1..16 and N up to the on-chip limit N x L <= 32768, on random
masks (including ties: LLRs on a coarse grid, exact zeros) and on
Bhattacharyya-built codes; a batch mixing sizes; a seeded random sweep;
argument errors."""
import sys

import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import bits_host, frame_items

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


def _frames(g, log2n, count, kind):
    n = 1 << log2n
    out = []
    for k in range(count):
        if kind == "bsc":
            mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(0.05), n // 3)
            u, fval, llr = synth.frame(int(g.integers(1 << 30)), log2n, "bsc", 0.05, mask,
                                       lambda v: oracle.encode(log2n, v))
        else:
            mask = (g.random(n) < g.uniform(0.2, 0.8)).astype(np.uint8)
            fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
            if kind == "grid":
                llr = (g.integers(-8, 9, n) * 0.25).astype(np.float32)
            else:
                llr = g.standard_normal(n).astype(np.float32) * 2
        out.append((np.asarray(llr, np.float32), np.asarray(mask, np.uint8), np.asarray(fval, np.uint8)))
    return out


def _gpu_scl(frames, list_size):
    import torch

    from paper_1204_5882_amd import polar as lp

    items = frame_items(frames, 0)
    pm = torch.full((len(frames),), -1.0, dtype=torch.float32, device="cuda")
    ctx = lp.Ctx(0)
    ctx.scl_decode(items, list_size, path_metric=pm)
    torch.cuda.synchronize()
    us = [bits_host(it["u_hat"], it["llr"].numel()) for it in items]
    ctx.close()
    return us, pm.cpu().numpy()


CASES = [(1, 1), (1, 4), (2, 2), (3, 8), (5, 16), (6, 4), (8, 8), (10, 1), (10, 8), (10, 16), (11, 8), (12, 4),
         (13, 2), (14, 1), (11, 16), (12, 8), (13, 4), (14, 2), (15, 1)]


@pytest.mark.parametrize("log2n,list_size", CASES)
@pytest.mark.parametrize("kind", ["grid", "gauss", "bsc"])
def test_list_decoder_matches_oracle(log2n, list_size, kind):
    g = np.random.default_rng(log2n * 100 + list_size * 7 + len(kind))
    count = 6 if log2n <= 10 else 3
    frames = _frames(g, log2n, count, kind)
    _say(f"case: scl log2n={log2n} L={list_size} kind={kind} frames={count}")
    us, pms = _gpu_scl(frames, list_size)
    for k, fr in enumerate(frames):
        ref_u, ref_pm = oracle.scl_decode(*fr, list_size)
        assert np.array_equal(us[k], ref_u), (k, int((us[k] != ref_u).sum()))
        assert pms[k] == ref_pm, (k, pms[k], ref_pm)


def test_mixed_sizes_in_one_batch():
    g = np.random.default_rng(77)
    frames = []
    for log2n in (11, 3, 8, 1, 10, 5):
        frames += _frames(g, log2n, 1, "grid")
    _say("case: scl mixed sizes L=8")
    us, pms = _gpu_scl(frames, 8)
    for k, fr in enumerate(frames):
        ref_u, ref_pm = oracle.scl_decode(*fr, 8)
        assert np.array_equal(us[k], ref_u) and pms[k] == ref_pm, k


def test_many_frames_sampled():
    """1024 frames of N = 2^10 at L = 8 in one call, a sample checked."""
    g = np.random.default_rng(78)
    frames = _frames(g, 10, 1024, "gauss")
    _say("case: scl 1024 frames N=2^10 L=8")
    us, pms = _gpu_scl(frames, 8)
    for k in list(range(0, 1024, 97)) + [1023]:
        ref_u, ref_pm = oracle.scl_decode(*frames[k], 8)
        assert np.array_equal(us[k], ref_u) and pms[k] == ref_pm, k


def test_argument_errors():
    import torch

    from paper_1204_5882_amd import polar as lp

    g = np.random.default_rng(79)
    fr = _frames(g, 12, 1, "grid")
    ctx = lp.Ctx(0)
    for bad_l in (0, 17):
        with pytest.raises(lp.PolarError):
            ctx.scl_decode(frame_items(fr, 0), bad_l)
    with pytest.raises(lp.PolarError):  # N x L = 2^12 x 16 > 32768
        ctx.scl_decode(frame_items(fr, 0), 16)
    with pytest.raises(lp.PolarError):  # box-plus
        ctx.scl_decode(frame_items(fr, 1), 2)
    torch.cuda.synchronize()
    ctx.close()


def test_random_sweep_matches_oracle():
    """400 seeded trials: list size 1..16, a batch of 1..5 frames with
    N x L <= 32768, masks of random density, Bhattacharyya-built or uniform,
    LLRs Gaussian, on a coarse grid with zeros, or BSC."""
    import torch

    from paper_1204_5882_amd import polar as lp

    ctx = lp.Ctx(0)
    for seed in range(400):
        g = np.random.default_rng(10_000 + seed)
        lsz = int(g.integers(1, 17))
        maxlog = min(15, (32768 // lsz).bit_length() - 1)
        logs = [int(g.integers(1, maxlog + 1)) for _ in range(int(g.integers(1, 6)))]
        frames = []
        for log2n in logs:
            n = 1 << log2n
            mk = int(g.integers(0, 3))
            if mk == 0:
                mask = (g.random(n) < g.uniform(0, 1)).astype(np.uint8)
            elif mk == 1:
                mask = np.asarray(oracle.frozen_set(log2n, float(g.uniform(0.05, 0.6)), int(g.integers(0, n + 1)))[0],
                                  np.uint8)
            else:
                mask = np.full(n, int(g.integers(0, 2)), np.uint8)
            fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
            lk = int(g.integers(0, 3))
            llr = (g.standard_normal(n) * 2 if lk == 0 else g.integers(-8, 9, n) * 0.25 if lk == 1
                   else np.where(g.random(n) < 0.05, -3.476, 3.476))
            frames.append((np.asarray(llr, np.float32), mask, fval))
        _say(f"case: scl sweep seed {seed} L={lsz} log2n={logs}")
        items = frame_items(frames, 0)
        pm = torch.full((len(frames),), -1.0, dtype=torch.float32, device="cuda")
        ctx.scl_decode(items, lsz, path_metric=pm)
        torch.cuda.synchronize()
        pms = pm.cpu().numpy()
        for k, fr in enumerate(frames):
            u = bits_host(items[k]["u_hat"], fr[0].size)
            ref_u, ref_pm = oracle.scl_decode(*fr, lsz)
            assert np.array_equal(u, ref_u) and pms[k] == ref_pm, (seed, k)
    ctx.close()
