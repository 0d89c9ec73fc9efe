"""Helpers shared by the GPU tests: move seeded frames to the device, decode
them through the C ABI, bring results back as 0/1 bytes."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def torch_mod():
    import torch

    return torch


def words_dev(bits: np.ndarray):
    torch = torch_mod()
    return torch.from_numpy(synth.pack_bits(bits).view(np.int32).copy()).to("cuda")


def bits_host(t, n: int) -> np.ndarray:
    return synth.unpack_bits(t.cpu().numpy().view(np.uint32), n)


def frame_items(frames, f_kind=0, dump=False):
    """frames: list of (llr f32[N], mask bits, fval bits).  Builds the
    dictionaries the binding takes, with fresh output buffers."""
    torch = torch_mod()
    from paper_1204_5882_amd import polar as lp

    items = []
    for llr, mask, fval in frames:
        n = llr.size
        log2n = n.bit_length() - 1
        assert (1 << log2n) == n and mask.size == n and fval.size == n
        items.append(dict(
            log2n=log2n, f_kind=f_kind,
            llr=torch.from_numpy(np.ascontiguousarray(llr, np.float32)).to("cuda"),
            frozen_mask=words_dev(mask), frozen_vals=words_dev(fval),
            u_hat=torch.full((lp.n_words(log2n),), -1, dtype=torch.int32, device="cuda"),
            leaf_llr=(torch.full((n,), float("nan"), dtype=torch.float32, device="cuda") if dump else None)))
    return items


def decode(frames, f_kind=0, prune=True, dump=False, plain=False, ctx=None, opts=None):
    """Decode on the GPU; returns (list of u-hat bits, list of leaf LLRs or None)."""
    torch = torch_mod()
    from paper_1204_5882_amd import polar as lp

    own = ctx is None
    if own:
        ctx = lp.Ctx(0)
    ctx.set_option(lp.POLAR_OPT_PRUNE, 1 if prune else 0)
    for k, v in (opts or {}).items():
        ctx.set_option(k, v)
    items = frame_items(frames, f_kind, dump)
    ctx.decode(items, plain=plain)
    torch.cuda.synchronize()
    us = [bits_host(it["u_hat"], it["llr"].numel()) for it in items]
    leaves = [it["leaf_llr"].cpu().numpy() if dump else None for it in items]
    if own:
        ctx.close()
    return us, leaves


def bsc_frames(log2n, p, n_frozen, seeds):
    mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(p), n_frozen)
    out = []
    for s in seeds:
        u, fval, llr = synth.frame(s, log2n, "bsc", p, mask, lambda v: oracle.encode(log2n, v))
        out.append((llr, mask, fval))
    return out


def biawgn_frames(log2n, sigma, n_frozen, seeds):
    mask, _, _ = oracle.frozen_set(log2n, synth.biawgn_z0(sigma), n_frozen)
    out = []
    for s in seeds:
        u, fval, llr = synth.frame(s, log2n, "biawgn", sigma, mask, lambda v: oracle.encode(log2n, v))
        out.append((llr, mask, fval))
    return out


def oracle_many(frames, boxplus=False):
    """Oracle u-hat for many frames, one frame per host thread."""
    if not frames:
        return []
    n = frames[0][0].size
    if all(f[0].size == n for f in frames):
        llr = np.stack([f[0] for f in frames])
        fval = np.stack([f[2] for f in frames])
        masks = np.stack([f[1] for f in frames])
        u = oracle.sc_decode_batch(llr, masks, fval, boxplus=boxplus)
        return [u[k] for k in range(len(frames))]
    return [oracle.sc_decode(f[0], f[1], f[2], boxplus=boxplus)[0] for f in frames]


def host_threads() -> int:
    """Worker threads for oracle runs: the CPUs this process may use, at most
    16 (one GPU's share of the host)."""
    import os

    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def magnitude_scale(llr):
    """S_i: leaf values with every g replaced by |a| + |b| and every f by
    min(|a|, |b|): the size of the terms whose rounding errors reach leaf i
    (a ±-sum tree's condition magnitude)."""
    n = llr.size
    return oracle.sc_decode(np.abs(llr), np.ones(n, np.uint8), np.zeros(n, np.uint8), want_leaf=True)[1]


def boxplus_teacher(frame, u_gpu):
    """The FP64 box-plus oracle re-run with the GPU's decisions as partial
    sums (teacher forcing), so that one tolerated disagreement does not
    derail every later LLR.  Returns (oracle decisions, FP64 leaf LLRs)."""
    llr, mask, fval = frame
    u_or, l_ref, _ = oracle.sc_decode(llr, mask, fval, boxplus=True, teacher=u_gpu, want_leaf=True)
    return u_or, l_ref


def check_boxplus_decisions(frames, us, what="", strict=False):
    """Box-plus u-hat against the FP64 oracle in teacher-forcing mode:
    frozen positions hold the frozen values, and an information bit may
    differ from the oracle's decision only where the oracle's leaf LLR lies
    within the LLR tolerance of zero: |L_ref| < 1e-6, or |L_ref| <=
    1e-5 S_i (S_i from magnitude_scale: the leaf is a cancelling sum whose
    terms are S_i large, so FP32 rounding of the terms moves it by about
    that much).  strict: the 1e-6 rule alone.  Oracle runs are spread over
    host threads.  Returns (tolerated disagreements, those that needed the
    S_i band)."""
    import concurrent.futures as cf

    def one(k):
        u_or, l_ref = boxplus_teacher(frames[k], us[k])
        return u_or, l_ref, magnitude_scale(frames[k][0]).astype(np.float64)

    with cf.ThreadPoolExecutor(host_threads()) as ex:
        res = list(ex.map(one, range(len(frames))))
    tolerated = scaled = 0
    for k, ((llr, mask, fval), u, (u_or, l_ref, s)) in enumerate(zip(frames, us, res)):
        fz = mask == 1
        assert np.array_equal(u[fz], fval[fz]), f"{what} frame {k}: frozen positions differ from the frozen values"
        dis = (u_or != u) & ~fz
        a = np.abs(l_ref[dis])
        band = np.full(a.shape, 1e-6) if strict else np.maximum(1e-6, 1e-5 * s[dis])
        assert np.all(a < band) if strict else np.all((a < 1e-6) | (a <= band)), \
            f"{what} frame {k}: {int(dis.sum())} decisions differ, max |L_ref| {a.max()}, band {band[a.argmax()]}"
        tolerated += int(dis.sum())
        scaled += int((a >= 1e-6).sum())
    return tolerated, scaled


def check_boxplus_leaves(frames, us, leaves, what="", computed_only=False, strict=False):
    """Leaf LLRs of box-plus against the teacher-forced FP64 oracle:
    |dL| <= 1e-5 max(|L_ref|, S_i) (S_i from magnitude_scale), plus the
    decision check above.  computed_only: compare only the leaves the kernel
    wrote (NaN marks leaves inside pruned nodes).  Decision disagreements as
    in check_boxplus_decisions.  Returns the number of leaves that pass only
    through S_i."""
    rescued = 0
    for k, (fr, u, lf) in enumerate(zip(frames, us, leaves)):
        llr, mask, fval = fr
        u_or, l_ref = boxplus_teacher(fr, u)
        s = magnitude_scale(llr).astype(np.float64)
        use = ~np.isnan(lf) if computed_only else np.ones(lf.size, bool)
        if not computed_only:
            assert not np.isnan(lf).any(), f"{what} frame {k}: leaves not written"
        err = np.abs(lf.astype(np.float64) - l_ref)
        tol = 1e-5 * np.maximum(np.abs(l_ref), s)
        bad = (err > tol) & use
        assert not bad.any(), f"{what} frame {k}: {int(bad.sum())} leaves out of tolerance, worst {err[bad].max()}"
        rescued += int(((err > 1e-5 * np.abs(l_ref)) & use).sum())
        fz = mask == 1
        assert np.array_equal(u[fz], fval[fz]), f"{what} frame {k}: frozen positions differ from the frozen values"
        dis = (u_or != u) & ~fz
        a = np.abs(l_ref[dis])
        ok = (a < 1e-6) if strict else ((a < 1e-6) | (a <= 1e-5 * s[dis]))
        assert np.all(ok), f"{what} frame {k}: decisions differ at |L_ref| up to {a.max()}"
    return rescued


def random_frames(log2n, g, count):
    """Frames with non-closed random frozen masks of several densities (so the
    kernel's generic node paths run), LLR mixes with many exact zeros, and
    every seventh frame on a Bhattacharyya mask."""
    n = 1 << log2n
    frames = []
    for k in range(count):
        kind = k % 4
        if kind == 0:
            llr = np.where(g.random(n) < 0.1, -1.0, 1.0).astype(np.float32) * np.float32(3.47)
        elif kind == 1:
            llr = (2.0 * ((1 - 2 * g.integers(0, 2, n)) + 0.9 * g.standard_normal(n)) / 0.81).astype(np.float32)
        elif kind == 2:
            llr = g.integers(-2, 3, n).astype(np.float32)   # many exact zeros
        else:
            llr = (g.integers(-3, 4, n) * (0.5 + g.random(n))).astype(np.float32)
        dens = [0.0, 1.0, 0.3, 0.5, 0.7][k % 5]
        if k % 7 == 6:
            mask, _, _ = oracle.frozen_set(log2n, 0.35, n // 2)
        else:
            mask = (g.random(n) < dens).astype(np.uint8)
        fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
        frames.append((llr, mask, fval))
    return frames
