"""GPU tests of the runtime around the decoder, through the C ABI: launch
variants (register-resident subtree 2^10 / 2^11 / 2^12, 4 or 8 wavefronts),
graph replay, the autotuner and its table, and the serving loop (admission
against an arena, continuous batching, cancellation, refusal of oversize
requests).  Every path must give the oracle's u-hat, and a frame's result
must not depend on what it was decoded with."""
import json
import os
import sys
import tempfile
import time

import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import biawgn_frames, bits_host, bsc_frames, decode, frame_items, oracle_many

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


def _mixed_frames(n_frames, lo, hi, seed):
    """Mixed sizes, BSC and BIAWGN, union-bound rates (one mask per frame)."""
    g = np.random.default_rng(seed)
    frames = []
    for f in range(n_frames):
        log2n = int(g.integers(lo, hi + 1))
        if f % 2 == 0:
            p = float(g.uniform(0.01, 0.05))
            mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(p), -1, 0.1)
            _, fval, llr = synth.frame(seed * 1000 + f, log2n, "bsc", p, mask, lambda v: oracle.encode(log2n, v))
        else:
            s = float(g.uniform(0.8, 1.2))
            mask, _, _ = oracle.frozen_set(log2n, synth.biawgn_z0(s), -1, 0.1)
            _, fval, llr = synth.frame(seed * 1000 + f, log2n, "biawgn", s, mask, lambda v: oracle.encode(log2n, v))
        frames.append((llr, mask, fval))
    return frames


# ------------------------------------------------------------ launch variants
@pytest.mark.parametrize("cut", [8, 9, 10, 11])
def test_smaller_cutover_minsum_matches_oracle(cut):
    from paper_1204_5882_amd import polar as lp

    frames = bsc_frames(16, 0.03, 16384, range(7000, 7006)) + bsc_frames(13, 0.02, 1638, range(7100, 7104))
    refs = [oracle.sc_decode(*fr)[0] for fr in frames]
    for waves in (4, 8):
        _say(f"case: cutover {cut}, waves {waves}, min-sum 2^16 and 2^13")
        us, _ = decode(frames, opts={lp.POLAR_OPT_CUTOVER: cut, lp.POLAR_OPT_WG_WAVES: waves})
        for k in range(len(frames)):
            assert np.array_equal(us[k], refs[k]), (cut, waves, k)


@pytest.mark.parametrize("cut", [8, 9, 10, 11])
def test_smaller_cutover_boxplus_equals_cutover_12(cut):
    """Determinism: box-plus results do not depend on where the HBM levels
    end (every f and g sees the same operands).  Agreement with the oracle is
    checked in test_gpu_boxplus.py."""
    from paper_1204_5882_amd import polar as lp

    frames = biawgn_frames(15, 0.97, 18000, range(7200, 7204))
    _say(f"case: box-plus cutover {cut} vs 12")
    ref, _ = decode(frames, f_kind=1, opts={lp.POLAR_OPT_CUTOVER: 12})
    got, _ = decode(frames, f_kind=1, opts={lp.POLAR_OPT_CUTOVER: cut, lp.POLAR_OPT_WG_WAVES: 8})
    for k in range(len(frames)):
        assert np.array_equal(got[k], ref[k]), k


def test_large_frame_on_every_cutover():
    from paper_1204_5882_amd import polar as lp

    frames = bsc_frames(20, 0.03, 262144, [7300])
    ref = oracle.sc_decode(*frames[0])[0]
    for cut in (8, 9, 10, 11, 12):
        _say(f"case: 2^20 min-sum, cutover {cut}")
        us, _ = decode(frames, opts={lp.POLAR_OPT_CUTOVER: cut})
        assert np.array_equal(us[0], ref), cut


# ---------------------------------------------------------------- graphs
def test_graph_replay_equals_eager():
    """Each replay, with eager decodes and synchronisations in between, gives
    the eager result; a batch with other buffers builds another graph."""
    import torch
    from paper_1204_5882_amd import polar as lp

    frames = _mixed_frames(24, 10, 16, seed=81)
    refs = [oracle.sc_decode(*fr)[0] for fr in frames]
    ctx = lp.Ctx(0)
    items = frame_items(frames)
    arr = lp.make_frames(items)
    ctx.ensure_workspace(arr, len(items))
    ctx.set_option(lp.POLAR_OPT_GRAPH, 1)
    other = frame_items(frames[:5])
    for rep in range(4):
        _say(f"case: graph replay {rep}")
        for it in items:
            it["u_hat"].fill_(-1)
        ctx.decode_batch(arr, len(items))
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            assert np.array_equal(bits_host(it["u_hat"], it["llr"].numel()), refs[k]), (rep, k)
        # eager work between replays: a different batch without the graph
        ctx.set_option(lp.POLAR_OPT_GRAPH, 0)
        ctx.decode(other)
        torch.cuda.synchronize()
        for k, it in enumerate(other):
            assert np.array_equal(bits_host(it["u_hat"], it["llr"].numel()), refs[k])
        ctx.set_option(lp.POLAR_OPT_GRAPH, 1)
    _say("case: graph for other buffers")
    ctx.decode(other)
    torch.cuda.synchronize()
    for k, it in enumerate(other):
        assert np.array_equal(bits_host(it["u_hat"], it["llr"].numel()), refs[k])
    ctx.close()


# ---------------------------------------------------------------- autotuner
def test_autotune_picks_a_built_config_and_keeps_results():
    import torch
    from paper_1204_5882_amd import polar as lp

    frames = bsc_frames(16, 0.03, 16384, range(7400, 7408))
    refs = oracle_many(frames)
    ctx = lp.Ctx(0)
    items = frame_items(frames)
    _say("case: autotune 8 x 2^16")
    best = ctx.autotune(items, reps=2)
    assert best["cutover"] in (8, 9, 10, 11, 12) and best["waves"] in (4, 8) and best["slots"] >= 1
    assert best["prune"] in (0, 1) and 1 <= best["fwg"] <= best["waves"]
    assert best["median_ms"] > 0 and best["candidates"] > 20
    q = ctx.query_launch(0, 16, 8)
    assert {k: q[k] for k in ("cutover", "waves", "prune")} == {k: best[k] for k in ("cutover", "waves", "prune")}
    # other sizes keep the defaults
    assert ctx.query_launch(0, 18, 8)["cutover"] == 12
    for it in items:
        it["u_hat"].fill_(-1)
    ctx.decode(items)
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        assert np.array_equal(bits_host(it["u_hat"], 1 << 16), refs[k])
    # explicit options win over the table
    ctx.set_option(lp.POLAR_OPT_CUTOVER, 12)
    assert ctx.query_launch(0, 16, 8)["cutover"] == 12
    ctx.set_option(lp.POLAR_OPT_CUTOVER, 0)
    # save / load round trip
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        ctx.tune_save(path)
        data = json.load(open(path))
        assert data["libpolar_tune"] == 1 and len(data["entries"]) == 1
        ctx2 = lp.Ctx(0)
        ctx2.tune_load(path)
        assert ctx2.query_launch(0, 16, 8) == ctx.query_launch(0, 16, 8)
        ctx2.tune_clear()
        assert ctx2.query_launch(0, 16, 8)["cutover"] == 12
        bad = os.path.join(d, "bad.json")
        with open(bad, "w") as f:
            f.write('{"libpolar_tune": 1, "entries": [{"f_kind": 0, "log2n": 16, "cutover": 13, "waves": 4, "slots": 8}]}')
        with pytest.raises(lp.PolarError):
            ctx2.tune_load(bad)
        ctx2.close()
    ctx.close()


# ---------------------------------------------------------------- serving
def _drain(srv, done, timeout_s=60.0):
    """Poll until nothing is queued, running or unreported; fills done."""
    t0 = time.time()
    while True:
        for rid, st, lat in srv.poll():
            done[rid] = (st, lat)
        if srv.pending() == (0, 0, 0):
            return done
        if time.time() - t0 > timeout_s:
            raise AssertionError(f"serving stalled: {len(done)} done, pending {srv.pending()}")
        time.sleep(0.0005)


def test_serving_results_equal_solo_decodes():
    import torch
    from paper_1204_5882_amd import polar as lp

    frames = _mixed_frames(40, 10, 18, seed=91)
    refs = [oracle.sc_decode(*fr)[0] for fr in frames]
    ctx = lp.Ctx(0)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    srv = lp.Server(ctx, arena, max_slots=16, poll_us=0)
    items = frame_items(frames)
    done = {}
    _say("case: serving 40 mixed requests, staggered")
    for k, it in enumerate(items):
        srv.submit(it, 100 + k)
        if k % 7 == 0:  # start batches while other requests still arrive
            for rid, st, lat in srv.poll():
                done[rid] = (st, lat)
    _drain(srv, done)
    srv.close()
    torch.cuda.synchronize()
    assert sorted(done) == [100 + k for k in range(40)]
    for k, it in enumerate(items):
        assert done[100 + k][0] == lp.POLAR_OK
        u = bits_host(it["u_hat"], it["llr"].numel())
        assert np.array_equal(u, refs[k]), k
    ctx.close()


def test_serving_admission_small_arena_cancel_and_nomem():
    import torch
    from paper_1204_5882_amd import polar as lp

    frames = bsc_frames(18, 0.03, 65536, range(7500, 7506))
    refs = oracle_many(frames)
    ctx = lp.Ctx(0)
    one = ctx.workspace_bytes(lp.make_frames(frame_items(frames[:1])), 1)
    # room for one 2^18 request at a time: batches of one, run one after another
    arena = torch.empty(one + 4096, dtype=torch.uint8, device="cuda")
    srv = lp.Server(ctx, arena, poll_us=0)
    items = frame_items(frames)
    big = frame_items(bsc_frames(20, 0.03, 262144, [7600]))[0]
    _say("case: serving with a one-request arena")
    for k, it in enumerate(items):
        srv.submit(it, k)
    srv.submit(big, 99)  # cannot fit even an empty arena
    # nothing has started yet: request 5 is still queued and can be cancelled
    assert srv.cancel(5) == lp.POLAR_OK
    assert srv.cancel(12345) == lp.POLAR_E_INVAL
    done = {}
    t0 = time.time()
    seen_running = 0
    while len(done) < 7:
        for rid, st, lat in srv.poll():
            done[rid] = (st, lat)
        q, r, c = srv.pending()
        seen_running = max(seen_running, r)
        assert time.time() - t0 < 60, (done, srv.pending())
        time.sleep(0.0002)
    srv.close()
    assert seen_running <= 1  # the arena admits one request at a time
    assert done[5][0] == lp.POLAR_E_CANCELLED
    assert done[99][0] == lp.POLAR_E_NOMEM
    for k in range(5):
        assert done[k][0] == lp.POLAR_OK and done[k][1] > 0
        assert np.array_equal(bits_host(items[k]["u_hat"], 1 << 18), refs[k]), k
    ctx.close()


def test_serving_queue_full_and_cancel_of_running_request():
    import torch
    from paper_1204_5882_amd import polar as lp

    ctx = lp.Ctx(0)
    arena = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    small = frame_items(bsc_frames(8, 0.03, 64, [7700]))[0]
    _say("case: serving queue filled to capacity (no poll, nothing runs)")
    srv = lp.Server(ctx, arena, poll_us=0)
    cap = 65536
    for k in range(cap):
        srv.submit(small, k)
    with pytest.raises(lp.PolarError) as err:
        srv.submit(small, cap)
    assert err.value.code == lp.POLAR_E_BUSY
    assert srv.pending() == (cap, 0, 0)
    srv.close()  # queued requests are dropped, none was started

    _say("case: cancel of a running request")
    frames = bsc_frames(20, 0.03, 262144, [7701])
    ref = oracle_many(frames)[0]
    item = frame_items(frames)[0]
    srv = lp.Server(ctx, arena, poll_us=0)
    srv.submit(item, 1)
    assert srv.poll() == []  # starts the batch; it stays running until a poll reaps it
    assert srv.pending()[1] == 1
    assert srv.cancel(1) == lp.POLAR_E_BUSY
    done = {}
    _drain(srv, done)
    srv.close()
    assert done[1][0] == lp.POLAR_OK
    assert np.array_equal(bits_host(item["u_hat"], 1 << 20), ref)
    ctx.close()


def test_empty_batch_and_refused_frames():
    import torch
    from paper_1204_5882_amd import polar as lp

    frames = bsc_frames(14, 0.03, 4096, [7800])
    ref = oracle_many(frames)[0]
    ctx = lp.Ctx(0)
    _say("case: empty batches")
    ctx.decode_batch(lp.make_frames([]), 0)
    ctx.decode_plain(lp.make_frames([]), 0)
    good = frame_items(frames)[0]
    arr = lp.make_frames([good])
    ctx.ensure_workspace(arr, 1)
    _say("case: invalid frames are refused before any launch")
    bad_frames = [
        dict(good, log2n=0),
        dict(good, log2n=25),
        dict(good, f_kind=7),
        dict(good, llr=good["llr"][1:]),  # not 16-byte aligned
        dict(good, u_hat=good["u_hat"].view(torch.uint8)[1:]),  # not 4-byte aligned
    ]
    for bad in bad_frames:
        with pytest.raises(lp.PolarError) as err:
            ctx.decode_batch(lp.make_frames([good, bad]), 2)
        assert err.value.code == lp.POLAR_E_INVAL
    null_out = lp.make_frames([good])
    null_out[0].u_hat = None
    with pytest.raises(lp.PolarError) as err:
        ctx.decode_batch(null_out, 1)
    assert err.value.code == lp.POLAR_E_INVAL
    torch.cuda.synchronize()
    assert bool((good["u_hat"] == -1).all())  # nothing was decoded
    _say("case: workspace too small")
    small = lp.Ctx(0)
    small.set_workspace(torch.empty(4096, dtype=torch.uint8, device="cuda"))
    with pytest.raises(lp.PolarError) as err:
        small.decode_batch(arr, 1)
    assert err.value.code == lp.POLAR_E_NOMEM
    small.close()
    _say("case: the context decodes normally after refused calls")
    ctx.decode_batch(arr, 1)
    torch.cuda.synchronize()
    assert np.array_equal(bits_host(good["u_hat"], 1 << 14), ref)
    ctx.close()


def test_blocking_serve_with_callbacks():
    import torch
    from paper_1204_5882_amd import polar as lp

    frames = _mixed_frames(16, 10, 16, seed=95)
    refs = [oracle.sc_decode(*fr)[0] for fr in frames]
    items = frame_items(frames)
    ctx = lp.Ctx(0)
    arena = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    queue = list(enumerate(items))
    results = {}

    def next_request():
        if not queue:
            return "end"
        k, it = queue.pop(0)
        return it, 500 + k

    def on_done(rid, status, lat):
        results[rid] = (status, lat)

    _say("case: blocking serve of 16 requests")
    lp.serve(ctx, arena, next_request, on_done, max_slots=8, poll_us=20)
    torch.cuda.synchronize()
    assert sorted(results) == [500 + k for k in range(16)]
    for k, it in enumerate(items):
        assert results[500 + k][0] == lp.POLAR_OK
        assert np.array_equal(bits_host(it["u_hat"], it["llr"].numel()), refs[k]), k
    ctx.close()


# ------------------------------------------------ frames per workgroup (small N)
@pytest.mark.parametrize("fwg", [1, 2, 4, 8])
def test_small_frames_per_wavefront(fwg):
    """Frames of at most 2^cutover leaves decoded one per wavefront, fwg per
    workgroup, behind larger frames of the same launch (the workgroup drops
    to per-wavefront mode when it reaches them): every frame equals the
    oracle, at cutover 12 (LDS caps 2^12 frames at 4 per workgroup) and 10."""
    from paper_1204_5882_amd import polar as lp

    g = np.random.default_rng(1700 + fwg)
    frames = []
    for k in range(300):
        log2n = int(g.integers(1, 13)) if k % 10 else int(g.integers(13, 16))
        p = float(g.uniform(0.01, 0.05))
        mask, _, _ = oracle.frozen_set(log2n, synth.bsc_z0(p), -1, 0.1)
        _, fval, llr = synth.frame(90000 + 1000 * fwg + k, log2n, "bsc", p, mask, lambda v, n=log2n: oracle.encode(n, v))
        frames.append((llr, mask, fval))
    refs = [oracle.sc_decode(*fr)[0] for fr in frames]
    for cut in (12, 10):
        for waves in (4, 8):
            if fwg > waves:
                continue
            _say(f"case: small frames fwg={fwg} cutover={cut} waves={waves}")
            ctx = lp.Ctx(0)
            us, _ = decode(frames, ctx=ctx, opts={lp.POLAR_OPT_FWG: fwg, lp.POLAR_OPT_CUTOVER: cut,
                                                  lp.POLAR_OPT_WG_WAVES: waves, lp.POLAR_OPT_MAX_SLOTS: 24})
            q = ctx.query_launch(0, cut, 300)   # frames of 2^cutover leaves
            assert q["fwg"] == min(fwg, {12: 4, 10: 7}[cut], waves), q
            ctx.close()
            for k in range(len(frames)):
                assert np.array_equal(us[k], refs[k]), (fwg, cut, waves, k)


def test_small_frames_many_per_cu_boxplus_and_dump():
    """Per-wavefront decoding with box-plus and with leaf dumps (2^6 .. 2^12)."""
    from gpu_helpers import check_boxplus_decisions, random_frames

    from paper_1204_5882_amd import polar as lp

    g = np.random.default_rng(1800)
    frames = []
    for lg in (6, 9, 10, 11, 12):
        frames += random_frames(lg, g, 12)
    _say("case: per-wavefront box-plus, 60 frames")
    us, _ = decode(frames, f_kind=1, opts={lp.POLAR_OPT_FWG: 8, lp.POLAR_OPT_MAX_SLOTS: 4})
    check_boxplus_decisions(frames, us, "per-wavefront box-plus")
    _say("case: per-wavefront min-sum with leaf dump")
    us, leaves = decode(frames, prune=False, dump=True, opts={lp.POLAR_OPT_FWG: 8, lp.POLAR_OPT_MAX_SLOTS: 4})
    for k, fr in enumerate(frames):
        ref_u, ref_l, _ = oracle.sc_decode(*fr, want_leaf=True)
        assert np.array_equal(us[k], ref_u), k
        assert np.all(leaves[k] == ref_l), k


def test_launch_respects_occupancy():
    """Workgroups of a launch never exceed what can be resident at once."""
    import torch
    from paper_1204_5882_amd import polar as lp

    ctx = lp.Ctx(0)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    ctx.set_option(lp.POLAR_OPT_MAX_SLOTS, 1 << 20)
    for cut in (8, 9, 10, 11, 12):
        ctx.set_option(lp.POLAR_OPT_CUTOVER, cut)
        q = ctx.query_launch(0, 20, 100000)
        assert 1 <= q["slots"] <= 8 * n_cu, q
        if cut == 12:  # about 127 KiB of LDS per workgroup: one per compute unit
            assert q["slots"] == n_cu, q
    ctx.close()


def test_serving_two_batches_resident_and_per_request_completion():
    """A batch of four 2^22 requests, then a batch of small requests on
    another stream while the first still runs: both batches are on the
    device at once, the small requests complete before the large ones (each
    request completes when its own frame does), and every result equals the
    oracle."""
    import torch
    from paper_1204_5882_amd import polar as lp

    big = bsc_frames(22, 0.03, 1 << 20, range(7900, 7904))
    small = bsc_frames(14, 0.03, 4096, range(7910, 7926))
    refs = oracle_many(big) + oracle_many(small)
    ctx = lp.Ctx(0)
    arena = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    srv = lp.Server(ctx, arena, poll_us=0)
    items = frame_items(big) + frame_items(small)
    _say("case: two resident batches")
    for k in range(4):
        srv.submit(items[k], k)
    assert srv.poll() == []           # starts the 2^22 batch
    for k in range(4, 20):
        srv.submit(items[k], k)
    done, order = {}, []
    max_batches = 0
    t0 = time.time()
    while len(done) < 20:
        for rid, st, lat in srv.poll():
            done[rid] = (st, lat)
            order.append(rid)
        max_batches = max(max_batches, srv.stats()[0])
        assert time.time() - t0 < 60, (done, srv.pending())
    srv.close()
    torch.cuda.synchronize()
    assert max_batches == 2
    assert all(done[k][0] == lp.POLAR_OK for k in range(20))
    first_big = min(order.index(k) for k in range(4))
    assert all(order.index(k) < first_big for k in range(4, 20)), order
    assert max(done[k][1] for k in range(4, 20)) < min(done[k][1] for k in range(4))
    for k, it in enumerate(items):
        assert np.array_equal(bits_host(it["u_hat"], it["llr"].numel()), refs[k]), k
    ctx.close()


def test_serving_waits_for_inputs_on_the_input_stream():
    """Inputs written on the caller's stream right before submit (no host
    synchronisation): the batch must wait for them.  The LLR tensors are
    filled on the stream after a long kernel, so a batch that did not wait
    would read the stale values."""
    import torch
    from paper_1204_5882_amd import polar as lp

    frames = bsc_frames(16, 0.03, 16384, range(8000, 8008))
    refs = oracle_many(frames)
    ctx = lp.Ctx(0)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    items = frame_items(frames)
    srv = lp.Server(ctx, arena, poll_us=0, input_stream=stream)
    host = [torch.from_numpy(fr[0]).pin_memory() for fr in frames]
    torch.cuda.synchronize()
    _say("case: serving inputs produced on the input stream")
    with torch.cuda.stream(stream):
        for it in items:
            it["llr"].fill_(1.0)            # wrong values, then the real ones
        x = torch.randn(4096, 4096, device="cuda")
        for _ in range(8):                  # keep the stream busy for a while
            x = x @ x
            x = x / x.norm()
        for it, h in zip(items, host):
            it["llr"].copy_(h, non_blocking=True)
            it["u_hat"].fill_(-1)
    for k, it in enumerate(items):
        srv.submit(it, k)
    done = {}
    _drain(srv, done)
    srv.close()
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        assert done[k][0] == lp.POLAR_OK
        assert np.array_equal(bits_host(it["u_hat"], 1 << 16), refs[k]), k
    ctx.close()


def test_serving_every_check_update_kind():
    """Requests of all five check updates (FP32 min-sum and box-plus, 16-bit
    saturating min-sum and phi table, 8-bit saturating min-sum) through one
    server: each equals its solo decode, the fixed-point ones the oracle."""
    import torch
    from paper_1204_5882_amd import polar as lp

    frames = _mixed_frames(10, 12, 16, seed=93)
    kinds = [k % 5 for k in range(10)]
    inputs = []
    for fr, fk in zip(frames, kinds):
        llr = fr[0]
        if fk in (2, 3):
            llr = oracle.quantize(llr).astype(np.float32)
        elif fk == 4:
            llr = oracle.quantize(llr, 2, oracle.FIXED8_MAX).astype(np.float32)
        inputs.append((llr, fr[1], fr[2]))
    items = []
    for fr, fk in zip(inputs, kinds):
        items += frame_items([fr], fk)
    ctx = lp.Ctx(0)
    arena = torch.empty(128 << 20, dtype=torch.uint8, device="cuda")
    srv = lp.Server(ctx, arena, max_slots=4, poll_us=0)
    done = {}
    _say("case: serving ten requests of five check-update kinds")
    for k, it in enumerate(items):
        srv.submit(it, 300 + k)
    _drain(srv, done)
    srv.close()
    torch.cuda.synchronize()
    fixed = {2: oracle.FIXED_MINSUM, 3: oracle.FIXED_PHI, 4: oracle.FIXED_MINSUM8}
    for k, (it, fr, fk) in enumerate(zip(items, inputs, kinds)):
        assert done[300 + k][0] == lp.POLAR_OK
        u = bits_host(it["u_hat"], it["llr"].numel())
        solo, _ = decode([fr], f_kind=fk)
        assert np.array_equal(u, solo[0]), k
        if fk in fixed:
            assert np.array_equal(u, oracle.sc_decode_fixed(fr[0].astype(np.int32), fr[1], fr[2], fixed[fk])[0]), k
        elif fk == 0:
            assert np.array_equal(u, oracle.sc_decode(*fr)[0]), k
    ctx.close()


def test_serving_small_request_passes_large_batches():
    """Three 2^22 requests fill the server's general streams; a 2^16 request
    submitted after them runs on the stream kept for small requests and
    completes while they still decode.  Every result equals its solo decode."""
    import torch
    from paper_1204_5882_amd import polar as lp

    big = bsc_frames(22, 0.03, 1 << 20, [9800, 9801, 9802])
    small = bsc_frames(16, 0.03, 1 << 14, [9803])
    frames = big + small
    ctx = lp.Ctx(0)
    arena = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    srv = lp.Server(ctx, arena, poll_us=0)
    items = frame_items(frames)
    torch.cuda.synchronize()
    _say("case: one 2^16 request behind three 2^22 requests")
    order = []
    for k, it in enumerate(items[:3]):
        srv.submit(it, 500 + k)
        for rid, st, _ in srv.poll():  # start each large request in its own batch
            order.append(rid)
    srv.submit(items[3], 503)
    done = {}
    t0 = time.time()
    while srv.pending() != (0, 0, 0):
        for rid, st, lat in srv.poll():
            done[rid] = (st, lat)
            order.append(rid)
        assert time.time() - t0 < 60.0, "serving stalled"
        time.sleep(0.0002)
    srv.close()
    torch.cuda.synchronize()
    assert sorted(order) == [500, 501, 502, 503]
    assert order[0] == 503, order  # the small request finished first
    assert done[503][1] < min(done[k][1] for k in (500, 501, 502))
    refs = oracle_many(frames)
    for k, it in enumerate(items):
        assert done[500 + k][0] == lp.POLAR_OK
        assert np.array_equal(bits_host(it["u_hat"], it["llr"].numel()), refs[k]), k
    ctx.close()


def test_serving_random_sweep_matches_oracle():
    """60 seeded trials: 1..39 requests of FP32 min-sum and the fixed-point
    kinds, N = 2^1 .. 2^18, submitted with random interleaved polls into
    arenas of 1 MiB to 256 MiB with several batch limits.  Every request is
    reported once; those that fit the arena equal the oracle, the others
    (2^18 in 1 MiB) complete with POLAR_E_NOMEM."""
    import torch
    from paper_1204_5882_amd import polar as lp

    kinds = {2: oracle.FIXED_MINSUM, 3: oracle.FIXED_PHI, 4: oracle.FIXED_MINSUM8}
    ctx = lp.Ctx(0)
    for seed in range(60):
        g = np.random.default_rng(20_000 + seed)
        nreq = int(g.integers(1, 40))
        arena_mb = int(g.choice([1, 4, 16, 64, 256]))
        max_slots = int(g.choice([0, 1, 2, 4, 16]))
        _say(f"case: serving sweep seed {seed}: {nreq} requests, arena {arena_mb} MiB, max_slots {max_slots}")
        arena = torch.empty(arena_mb << 20, dtype=torch.uint8, device="cuda")
        srv = lp.Server(ctx, arena, max_slots=max_slots, poll_us=0)
        reqs = []
        for _ in range(nreq):
            fk = int(g.choice([0, 2, 3, 4]))
            log2n = int(g.integers(1, 19))
            n = 1 << log2n
            mask = np.asarray(oracle.frozen_set(log2n, float(g.uniform(0.05, 0.5)), int(g.integers(0, n + 1)))[0],
                              np.uint8)
            fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
            if fk == 0:
                llr = (g.standard_normal(n) * 2).astype(np.float32)
            else:
                lim = oracle.FIXED8_MAX if fk == 4 else oracle.FIXED_MAX
                llr = (g.integers(-lim, lim + 1, n) if g.integers(0, 2) else g.integers(-3, 4, n)).astype(np.float32)
            reqs.append((fk, llr, mask, fval, frame_items([(llr, mask, fval)], fk)[0]))
        done = {}
        for k, r in enumerate(reqs):
            srv.submit(r[4], k)
            if g.integers(0, 3) == 0:
                for rid, st, lat in srv.poll():
                    done[rid] = (st, lat)
        _drain(srv, done)
        srv.close()
        torch.cuda.synchronize()
        assert sorted(done) == list(range(nreq)), seed
        for k, (fk, llr, mask, fval, it) in enumerate(reqs):
            if arena_mb == 1 and it["log2n"] == 18:
                assert done[k][0] == lp.POLAR_E_NOMEM, (seed, k)
                continue
            assert done[k][0] == lp.POLAR_OK, (seed, k, done[k][0])
            u = bits_host(it["u_hat"], llr.size)
            ref = (oracle.sc_decode(llr, mask, fval)[0] if fk == 0
                   else oracle.sc_decode_fixed(llr.astype(np.int32), mask, fval, kinds[fk])[0])
            assert np.array_equal(u, ref), (seed, k)
        del arena
    ctx.close()
