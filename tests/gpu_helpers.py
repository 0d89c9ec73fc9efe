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
