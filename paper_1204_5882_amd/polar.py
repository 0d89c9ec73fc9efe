"""Thin Python binding of libpolar (include/polar.h) over ctypes.

Argument marshalling only: every step of encoding and decoding runs in the
library's HIP kernels.  PyTorch provides device memory and streams.  Bit
vectors are torch.int32 tensors holding the packed uint32 words (bit i in
word i >> 5 at position i & 31).

If libpolar.so has not been built, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpolar.so")

POLAR_OK = 0
POLAR_E_INVAL = -1
POLAR_E_NOMEM = -2
POLAR_E_DEVICE = -3
POLAR_E_BUSY = -4
POLAR_E_CANCELLED = -5

POLAR_F_MINSUM = 0
POLAR_F_BOXPLUS = 1
POLAR_F_MINSUM_Q16 = 2
POLAR_F_PHI_Q16 = 3
POLAR_F_MINSUM_Q8 = 4
POLAR_FIXED_FRAC = 4
POLAR_FIXED_MAX = 32767
POLAR_FIXED8_MAX = 127
POLAR_FIXED8_FRAC = 2
POLAR_MAX_LOG2N = 24

POLAR_OPT_PRUNE = 1
POLAR_OPT_CUTOVER = 2
POLAR_OPT_WG_WAVES = 3
POLAR_OPT_MAX_SLOTS = 4
POLAR_OPT_TIMING = 5
POLAR_OPT_GRAPH = 6
POLAR_OPT_FWG = 7
POLAR_OPT_HELPERS = 8
POLAR_STATIC_SCRATCH_BYTES = 256 << 20
POLAR_STATIC_MAX_FRAMES = 16384
POLAR_CONSTRUCT_MAX_MU = 64
POLAR_SCL_MAX_LIST = 16
POLAR_SCL_MAX_NL = 32768
POLAR_CONSTRUCT_MAX_OUTPUTS = 65536

# every symbol declared in include/polar.h
EXPORTED = [
    "polar_last_error", "polar_version", "polar_build_frozen_set", "polar_encode",
    "polar_ctx_create", "polar_ctx_destroy", "polar_ctx_set_workspace", "polar_ctx_set_option",
    "polar_ctx_get_option", "polar_workspace_bytes", "polar_sc_decode_batch",
    "polar_sc_decode_plain", "polar_sc_decode_batch_static", "polar_autotune", "polar_query_launch", "polar_tune_clear",
    "polar_tune_save", "polar_tune_load", "polar_serve_open", "polar_serve_submit", "polar_serve_poll",
    "polar_serve_pending", "polar_serve_stats", "polar_serve_cancel", "polar_serve_close", "polar_serve",
    "polar_debug_lane_selftest", "polar_debug_phi_table", "polar_fer_generate_bsc", "polar_fer_workspace_bytes", "polar_fer_bsc",
    "polar_construct_workspace_bytes", "polar_construct_degrade", "polar_frozen_from_pe",
    "polar_scl_workspace_bytes", "polar_scl_decode_batch",
]


class PolarError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpolar error {code}: {msg}")
        self.code = code


class polar_frame(ctypes.Structure):
    _fields_ = [
        ("log2n", ctypes.c_int32),
        ("f_kind", ctypes.c_int32),
        ("llr", ctypes.c_void_p),
        ("frozen_mask", ctypes.c_void_p),
        ("frozen_vals", ctypes.c_void_p),
        ("u_hat", ctypes.c_void_p),
        ("leaf_llr", ctypes.c_void_p),
    ]


class polar_serve_cfg(ctypes.Structure):
    _fields_ = [
        ("arena_bytes", ctypes.c_size_t),
        ("arena", ctypes.c_void_p),
        ("max_slots", ctypes.c_int),
        ("poll_us", ctypes.c_int),
        ("input_stream", ctypes.c_void_p),
    ]


class polar_fer_cfg(ctypes.Structure):
    _fields_ = [
        ("log2n", ctypes.c_int32),
        ("f_kind", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("frozen_mask", ctypes.c_void_p),
        ("seed", ctypes.c_uint64),
        ("frame0", ctypes.c_int64),
        ("n_frames", ctypes.c_int64),
        ("batch", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class polar_fer_result(ctypes.Structure):
    _fields_ = [
        ("frames", ctypes.c_int64),
        ("frame_errors", ctypes.c_int64),
        ("bit_errors", ctypes.c_int64),
    ]


class polar_completion(ctypes.Structure):
    _fields_ = [
        ("req_id", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("latency_s", ctypes.c_double),
    ]


NEXT_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(polar_frame), ctypes.POINTER(ctypes.c_uint64))
DONE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_double)

_lib = None


def load():
    """Load libpolar.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python -m paper_1204_5882_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "polar_last_error": ([], ctypes.c_char_p),
        "polar_version": ([], ctypes.c_char_p),
        "polar_build_frozen_set": ([I, ctypes.c_double, I64, ctypes.c_double, P, P, P], I),
        "polar_encode": ([I, I, P, P, P], I),
        "polar_ctx_create": ([P, I, P, SZ], I),
        "polar_ctx_destroy": ([P], I),
        "polar_ctx_set_workspace": ([P, P, SZ], I),
        "polar_ctx_set_option": ([P, I, I64], I),
        "polar_ctx_get_option": ([P, I, P], I),
        "polar_workspace_bytes": ([P, P, I], SZ),
        "polar_sc_decode_batch": ([P, P, I, P], I),
        "polar_sc_decode_plain": ([P, P, I, P], I),
        "polar_sc_decode_batch_static": ([P, P, I, P], I),
        "polar_autotune": ([P, P, I, I, P, P, P, P, P, P, P, P], I),
        "polar_query_launch": ([P, I, I, I, P, P, P, P, P], I),
        "polar_tune_clear": ([P], I),
        "polar_tune_save": ([P, ctypes.c_char_p], I),
        "polar_tune_load": ([P, ctypes.c_char_p], I),
        "polar_serve_open": ([P, P, P], I),
        "polar_serve_submit": ([P, P, ctypes.c_uint64], I),
        "polar_serve_poll": ([P, P, I, P], I),
        "polar_serve_pending": ([P, P, P, P], I),
        "polar_serve_stats": ([P, P, P], I),
        "polar_serve_cancel": ([P, ctypes.c_uint64], I),
        "polar_serve_close": ([P], I),
        "polar_serve": ([P, P, NEXT_FN, DONE_FN, P], I),
        "polar_debug_lane_selftest": ([P, P], I),
        "polar_debug_phi_table": ([P, P], I),
        "polar_fer_generate_bsc": ([I, ctypes.c_double, I, P, ctypes.c_uint64, I64, I, P, P, P, P, P], I),
        "polar_fer_workspace_bytes": ([P, P], SZ),
        "polar_fer_bsc": ([P, P, P, SZ, P, P, P], I),
        "polar_construct_workspace_bytes": ([I, I, I], SZ),
        "polar_construct_degrade": ([I, P, I, I, P, SZ, P, P], I),
        "polar_frozen_from_pe": ([I, P, I64, ctypes.c_double, P, P], I),
        "polar_scl_workspace_bytes": ([I], SZ),
        "polar_scl_decode_batch": ([P, P, I, I, P, P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != POLAR_OK:
        raise PolarError(rc, load().polar_last_error().decode())


def last_error() -> str:
    return load().polar_last_error().decode()


def version() -> str:
    return load().polar_version().decode()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def n_words(log2n: int) -> int:
    return max(1, (1 << log2n) // 32)


def build_frozen_set(log2n: int, z0: float, n_frozen: int = -1, fer_bound: float = 0.1,
                     want_r: bool = False):
    """Host-side Bhattacharyya frozen set.  Returns (mask words uint32, n_frozen, r or None)."""
    mask = np.zeros(n_words(log2n), np.uint32)
    r = np.empty(1 << log2n, np.float64) if want_r else None
    nf = ctypes.c_int64(0)
    _check(load().polar_build_frozen_set(int(log2n), float(z0), int(n_frozen), float(fer_bound),
                                         mask.ctypes.data, None if r is None else r.ctypes.data,
                                         ctypes.addressof(nf)))
    return mask, int(nf.value), r


def construct_workspace_bytes(log2n: int, mu: int, m0: int) -> int:
    return int(load().polar_construct_workspace_bytes(int(log2n), int(mu), int(m0)))


def construct_degrade(log2n: int, w0, mu: int, pe=None, workspace=None, stream=None):
    """Error probabilities of the N synthetic channels by channel degradation
    on the device.  w0: (m0, 2) array of output pairs (a, b) of the channel.
    Returns pe, a float64 torch tensor of N values on the current device."""
    import torch

    w0 = np.ascontiguousarray(np.asarray(w0, np.float64).reshape(-1, 2))
    m0 = w0.shape[0]
    if pe is None:
        pe = torch.empty(1 << log2n, dtype=torch.float64, device="cuda")
    need = construct_workspace_bytes(log2n, mu, m0)
    if need == 0:
        _check(load().polar_construct_degrade(int(log2n), w0.ctypes.data, int(m0), int(mu), None, 0, None, None))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=pe.device)
    _check(load().polar_construct_degrade(int(log2n), w0.ctypes.data, int(m0), int(mu), _ptr(workspace),
                                          int(workspace.numel()), _ptr(pe), _stream_handle(stream)))
    return pe


def frozen_from_pe(log2n: int, pe, n_frozen: int = -1, fer_bound: float = 0.1):
    """Host-side frozen set from per-channel error probabilities.  Returns
    (mask words uint32, n_frozen)."""
    pe = np.ascontiguousarray(np.asarray(pe, np.float64))
    if pe.shape != (1 << log2n,):
        raise ValueError("pe must hold N values")
    mask = np.zeros(n_words(log2n), np.uint32)
    nf = ctypes.c_int64(0)
    _check(load().polar_frozen_from_pe(int(log2n), pe.ctypes.data, int(n_frozen), float(fer_bound),
                                       mask.ctypes.data, ctypes.addressof(nf)))
    return mask, int(nf.value)


def encode(log2n: int, u, x=None, n_frames: Optional[int] = None, stream=None):
    """x = u G_N for packed frames (torch int32 tensors on the GPU); returns x."""
    import torch

    if x is None:
        x = torch.empty_like(u)
    w = n_words(log2n)
    if n_frames is None:
        n_frames = u.numel() // w
    if u.numel() < n_frames * w or x.numel() < n_frames * w:
        raise ValueError("buffers too small")
    _check(load().polar_encode(int(log2n), int(n_frames), _ptr(u), _ptr(x), _stream_handle(stream)))
    return x


def fer_generate_bsc(log2n: int, p: float, frozen_mask, seed: int, frame0: int, n_frames: int, fixed_point=0,
                     stream=None):
    """Synthetic BSC frames on the device (the harness's generator): returns
    (u words, frozen-value words, LLRs) as torch tensors of shapes
    (n_frames, W), (n_frames, W), (n_frames, N).  fixed_point: 0 FP32 LLRs,
    1 (or True) integers in units of 2^-4, 2 integers in units of 2^-2
    capped at 127 (the 8-bit kind)."""
    import torch

    dev = frozen_mask.device
    w = n_words(log2n)
    u = torch.empty((n_frames, w), dtype=torch.int32, device=dev)
    vals = torch.empty_like(u)
    x = torch.empty_like(u)
    llr = torch.empty((n_frames, 1 << log2n), dtype=torch.float32, device=dev)
    _check(load().polar_fer_generate_bsc(int(log2n), float(p), int(fixed_point), _ptr(frozen_mask),
                                         int(seed), int(frame0),
                                         int(n_frames), _ptr(u), _ptr(vals), _ptr(x), _ptr(llr),
                                         _stream_handle(stream)))
    return u, vals, llr


def phi_table(stream=None):
    """The phi table of POLAR_F_PHI_Q16 as the device builds it (256 floats)."""
    import torch

    out = torch.empty(256, dtype=torch.float32, device="cuda")
    _check(load().polar_debug_phi_table(_ptr(out), _stream_handle(stream)))
    return out


def lane_selftest(stream=None):
    import torch

    out = torch.zeros(1024, dtype=torch.int32, device="cuda")
    _check(load().polar_debug_lane_selftest(_ptr(out), _stream_handle(stream)))
    return out


def fill_frame(fr: polar_frame, it: dict) -> None:
    fr.log2n = int(it["log2n"])
    fr.f_kind = int(it.get("f_kind", POLAR_F_MINSUM))
    fr.llr = _ptr(it["llr"])
    fr.frozen_mask = _ptr(it["frozen_mask"])
    fr.frozen_vals = _ptr(it["frozen_vals"])
    fr.u_hat = _ptr(it["u_hat"])
    fr.leaf_llr = _ptr(it.get("leaf_llr"))


def make_frames(items: Sequence[dict]) -> ctypes.Array:
    """items: dicts with log2n, f_kind, llr, frozen_mask, frozen_vals, u_hat,
    optional leaf_llr (torch tensors on the device)."""
    arr = (polar_frame * max(1, len(items)))()
    for i, it in enumerate(items):
        fill_frame(arr[i], it)
    return arr


class Ctx:
    """A polar_ctx plus a workspace tensor it grows on demand."""

    def __init__(self, device: int = 0):
        self._lib = load()
        self._h = ctypes.c_void_p()
        _check(self._lib.polar_ctx_create(ctypes.addressof(self._h), int(device), None, 0))
        self.device = device
        self.workspace = None

    def close(self):
        if self._h:
            self._lib.polar_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, opt: int, value: int):
        _check(self._lib.polar_ctx_set_option(self._h, int(opt), int(value)))

    def get_option(self, opt: int) -> int:
        v = ctypes.c_int64(0)
        _check(self._lib.polar_ctx_get_option(self._h, int(opt), ctypes.addressof(v)))
        return int(v.value)

    def workspace_bytes(self, frames: ctypes.Array, n: int) -> int:
        return int(self._lib.polar_workspace_bytes(self._h, frames, int(n)))

    def set_workspace(self, tensor):
        self.workspace = tensor
        _check(self._lib.polar_ctx_set_workspace(self._h, _ptr(tensor),
                                                 0 if tensor is None else tensor.numel() * tensor.element_size()))

    def ensure_workspace(self, frames: ctypes.Array, n: int):
        import torch

        need = self.workspace_bytes(frames, n)
        have = 0 if self.workspace is None else self.workspace.numel()
        if need > have:
            # torch's caching allocator returns 512-byte aligned blocks
            self.set_workspace(torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}"))

    def scl_decode(self, items: Iterable[dict], list_size: int, path_metric=None, stream=None):
        """SC list decoding of min-sum frames (polar_scl_decode_batch); the
        chosen path's metric goes to path_metric (device float32) if given."""
        import torch

        items = list(items)
        frames = make_frames(items)
        need = int(self._lib.polar_scl_workspace_bytes(len(items)))
        have = 0 if self.workspace is None else self.workspace.numel()
        if need > have:
            self.set_workspace(torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}"))
        self.scl_decode_frames(frames, len(items), list_size, path_metric, stream)

    def scl_decode_frames(self, frames: ctypes.Array, n: int, list_size: int, path_metric=None, stream=None):
        """polar_scl_decode_batch on a prepared frame array (make_frames); the
        workspace must already hold the descriptor table."""
        _check(self._lib.polar_scl_decode_batch(self._h, frames, int(n), int(list_size), _ptr(path_metric),
                                                _stream_handle(stream)))

    def decode_batch(self, frames: ctypes.Array, n: int, stream=None):
        _check(self._lib.polar_sc_decode_batch(self._h, frames, int(n), _stream_handle(stream)))

    def fer_bsc(self, log2n: int, p: float, frozen_mask, n_frames: int, seed: int = 1, frame0: int = 0,
                f_kind: int = POLAR_F_MINSUM, batch: int = 0, stream=None):
        """Monte-Carlo FER on BSC(p), everything on the device.  Returns
        (result dict, per-frame bit errors as a torch int32 tensor)."""
        import torch

        cfg = polar_fer_cfg(int(log2n), int(f_kind), float(p), _ptr(frozen_mask), int(seed), int(frame0),
                            int(n_frames), int(batch), 0)
        need = self._lib.polar_fer_workspace_bytes(self._h, ctypes.addressof(cfg))
        if need == 0:
            raise PolarError(POLAR_E_INVAL, "invalid FER configuration")
        ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
        bit_err = torch.empty(max(1, int(n_frames)), dtype=torch.int32, device=f"cuda:{self.device}")
        res = polar_fer_result()
        _check(self._lib.polar_fer_bsc(self._h, ctypes.addressof(cfg), _ptr(ws), need, _ptr(bit_err),
                                       ctypes.addressof(res), _stream_handle(stream)))
        return ({"frames": res.frames, "frame_errors": res.frame_errors, "bit_errors": res.bit_errors},
                bit_err[: int(n_frames)])

    def decode_batch_static(self, frames: ctypes.Array, n: int, stream=None):
        """polar_sc_decode_batch_static: the library's static device buffer as
        workspace, no allocation (calls on one device must not overlap)."""
        _check(self._lib.polar_sc_decode_batch_static(self._h, frames, int(n), _stream_handle(stream)))

    def decode_plain(self, frames: ctypes.Array, n: int, stream=None):
        _check(self._lib.polar_sc_decode_plain(self._h, frames, int(n), _stream_handle(stream)))

    def decode(self, items: Iterable[dict], plain: bool = False, stream=None):
        items = list(items)
        frames = make_frames(items)
        self.ensure_workspace(frames, len(items))
        (self.decode_plain if plain else self.decode_batch)(frames, len(items), stream)

    # autotuner -----------------------------------------------------------
    def autotune(self, items: Sequence[dict], reps: int = 3, stream=None) -> dict:
        """Time the built launch configurations on these frames, keep the best
        for their (f_kind, largest log2n); returns the launch a batch of these
        frames now gets."""
        import torch

        items = list(items)
        frames = make_frames(items)
        # room for the largest candidate (every resident workgroup, any cutover)
        need = 0
        saved = {o: self.get_option(o) for o in (POLAR_OPT_CUTOVER, POLAR_OPT_MAX_SLOTS, POLAR_OPT_WG_WAVES)}
        for cut in (8, 9, 10, 11, 12):
            for waves in (4, 8):
                self.set_option(POLAR_OPT_CUTOVER, cut)
                self.set_option(POLAR_OPT_WG_WAVES, waves)
                self.set_option(POLAR_OPT_MAX_SLOTS, 1 << 20)
                need = max(need, self.workspace_bytes(frames, len(items)))
        for o, v in saved.items():
            self.set_option(o, v)
        if self.workspace is None or self.workspace.numel() < need:
            self.set_workspace(torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}"))
        c, w, sl, fw, pr, n = (ctypes.c_int() for _ in range(6))
        ms = ctypes.c_double()
        _check(self._lib.polar_autotune(self._h, frames, len(items), int(reps), _stream_handle(stream),
                                        ctypes.addressof(c), ctypes.addressof(w), ctypes.addressof(sl),
                                        ctypes.addressof(fw), ctypes.addressof(pr), ctypes.addressof(ms),
                                        ctypes.addressof(n)))
        return {"cutover": c.value, "waves": w.value, "slots": sl.value, "fwg": fw.value, "prune": pr.value,
                "median_ms": ms.value, "candidates": n.value}

    def query_launch(self, f_kind: int, log2n: int, n_frames: int) -> dict:
        c, w, sl, fw, pr = (ctypes.c_int() for _ in range(5))
        _check(self._lib.polar_query_launch(self._h, int(f_kind), int(log2n), int(n_frames), ctypes.addressof(c),
                                            ctypes.addressof(w), ctypes.addressof(sl), ctypes.addressof(fw),
                                            ctypes.addressof(pr)))
        return {"cutover": c.value, "waves": w.value, "slots": sl.value, "fwg": fw.value, "prune": pr.value}

    def tune_clear(self):
        _check(self._lib.polar_tune_clear(self._h))

    def tune_save(self, path: str):
        _check(self._lib.polar_tune_save(self._h, path.encode()))

    def tune_load(self, path: str):
        _check(self._lib.polar_tune_load(self._h, path.encode()))


class Server:
    """Non-blocking serving API over a caller-provided device arena (a torch
    uint8 tensor).  Frames are dicts as for make_frames; the tensors must stay
    alive until their request completes (the server keeps a reference)."""

    def __init__(self, ctx: Ctx, arena, max_slots: int = 0, poll_us: int = 50, input_stream=None):
        """input_stream: the stream request inputs are produced on (default:
        torch's current stream); every batch waits for the work enqueued on it."""
        self._lib = load()
        self.ctx = ctx
        self.arena = arena
        self._h = ctypes.c_void_p()
        cfg = polar_serve_cfg(arena.numel() * arena.element_size(), _ptr(arena), int(max_slots), int(poll_us),
                              _stream_handle(input_stream))
        _check(self._lib.polar_serve_open(ctx._h, ctypes.addressof(cfg), ctypes.addressof(self._h)))
        self._keep = {}
        self._buf = (polar_completion * 1024)()

    def submit(self, item: dict, req_id: int):
        fr = polar_frame()
        fill_frame(fr, item)
        _check(self._lib.polar_serve_submit(self._h, ctypes.addressof(fr), int(req_id)))
        self._keep[int(req_id)] = item

    def poll(self) -> list:
        """[(req_id, status, latency_s)] of requests completed since the last poll."""
        n = ctypes.c_int(0)
        rc = self._lib.polar_serve_poll(self._h, self._buf, len(self._buf), ctypes.addressof(n))
        out = [(int(self._buf[k].req_id), int(self._buf[k].status), float(self._buf[k].latency_s))
               for k in range(n.value)]
        for rid, _, _ in out:
            self._keep.pop(rid, None)
        _check(rc)
        return out

    def pending(self) -> tuple:
        q, r, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.polar_serve_pending(self._h, ctypes.addressof(q), ctypes.addressof(r), ctypes.addressof(c)))
        return q.value, r.value, c.value

    def stats(self) -> tuple:
        """(batches on the device, arena bytes they hold)."""
        nb, used = ctypes.c_int(), ctypes.c_size_t()
        _check(self._lib.polar_serve_stats(self._h, ctypes.addressof(nb), ctypes.addressof(used)))
        return nb.value, used.value

    def cancel(self, req_id: int) -> int:
        """POLAR_OK, or the error code (POLAR_E_BUSY if running, POLAR_E_INVAL if unknown)."""
        return int(self._lib.polar_serve_cancel(self._h, int(req_id)))

    def close(self):
        if self._h:
            rc = self._lib.polar_serve_close(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()
            _check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve(ctx: Ctx, arena, next_request, on_done, max_slots: int = 0, poll_us: int = 50, input_stream=None):
    """Blocking serving loop.  next_request() -> (item, req_id) | None (none
    yet) | StopIteration-like sentinel "end"; on_done(req_id, status, latency_s)."""
    lib = load()
    keep = {}

    def _next(user, fr_ptr, id_ptr):
        try:
            r = next_request()
        except Exception:  # a failing producer ends the stream
            return 2
        if r is None:
            return 1
        if r == "end":
            return 2
        item, rid = r
        fill_frame(fr_ptr.contents, item)
        id_ptr[0] = int(rid)
        keep[int(rid)] = item
        return 0

    def _done(user, rid, status, lat):
        keep.pop(int(rid), None)
        on_done(int(rid), int(status), float(lat))

    nf, df = NEXT_FN(_next), DONE_FN(_done)
    cfg = polar_serve_cfg(arena.numel() * arena.element_size(), _ptr(arena), int(max_slots), int(poll_us),
                          _stream_handle(input_stream))
    _check(lib.polar_serve(ctx._h, ctypes.addressof(cfg), nf, df, None))
