"""CPU oracle for SC decoding of polar codes.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the CPU
baseline leg of the benchmark.  The GPU library never imports, links or calls
anything here, and nothing here imports the GPU library.

The arithmetic lives in ``sc_oracle.c`` (plain C, compiled with gcc
``-O2 -ffp-contract=off -fno-fast-math``) and in ``naive.py`` (pure Python,
small sizes only).  Bits are passed one byte per bit, in natural index order.

Parity status of each function (what pins it is listed in the tests):
  encode            pinned: Kronecker matrix (N <= 64), involution G.G = I
  bhattacharyya     pinned: 50-digit mpmath recursion (N <= 2^12), sum rule,
                    hand values, partial-order monotonicity
  frozen_set        pinned: as above plus tie-free boundary checks
  sc_decode minsum  pinned: naive per-bit SC (N <= 64), closed forms at scale
  sc_decode boxplus pinned: brute-force likelihood SC (N <= 16), mpmath f
  phi_table         pinned: 60-digit mpmath phi, involution, monotonicity
  scl_decode        pinned: L = 1 equals sc_decode; a per-bit list decoder
                    built on naive.py's re-encoding SC (N <= 32); the final
                    metric equals the codeword's correlation discrepancy
                    sum |L_j| [x_j != hard_j] (max-log ML metric) at any N;
                    with L >= 2^K it returns a discrepancy minimiser (brute
                    force over all codewords)
  sc_decode_fixed   pinned: naive per-bit SC in the same integer arithmetic
                    (N <= 64), FP32 min-sum equality without saturation,
                    saturation at the int16 bounds, phi-table LLRs within the
                    quantization error of the exact FP64 update
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread"]


def build(force: bool = True) -> str:
    """Compile sc_oracle.c into liboracle.so with gcc (CPU only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    lib.oracle_encode.argtypes = [ctypes.c_int, P, P]
    lib.oracle_encode.restype = ctypes.c_int
    lib.oracle_bhattacharyya.argtypes = [ctypes.c_int, ctypes.c_double, P, P]
    lib.oracle_bhattacharyya.restype = ctypes.c_int
    lib.oracle_frozen_set.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                      ctypes.c_double, P, P]
    lib.oracle_frozen_set.restype = ctypes.c_int64
    lib.oracle_sc_decode.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P]
    lib.oracle_sc_decode.restype = ctypes.c_int
    lib.oracle_sc_decode_batch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, P, P, P, P, ctypes.c_int]
    lib.oracle_sc_decode_batch.restype = ctypes.c_int
    lib.oracle_f_minsum.argtypes = [ctypes.c_float, ctypes.c_float]
    lib.oracle_f_minsum.restype = ctypes.c_float
    lib.oracle_g_f32.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_int]
    lib.oracle_g_f32.restype = ctypes.c_float
    lib.oracle_f_boxplus.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_f_boxplus.restype = ctypes.c_double
    lib.oracle_phi_table.argtypes = [ctypes.c_int, ctypes.c_int, P]
    lib.oracle_phi_table.restype = ctypes.c_int
    lib.oracle_sc_decode_fixed.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, ctypes.c_int]
    lib.oracle_sc_decode_fixed.restype = ctypes.c_int
    lib.oracle_f_fixed.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int]
    lib.oracle_f_fixed.restype = ctypes.c_int32
    lib.oracle_scl_decode.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    lib.oracle_scl_decode.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _bits(a, n) -> np.ndarray:
    b = np.ascontiguousarray(np.asarray(a, dtype=np.uint8))
    if b.shape != (n,):
        raise ValueError(f"expected {n} bits, got shape {b.shape}")
    if b.size and b.max() > 1:
        raise ValueError("bit arrays must hold 0/1")
    return b


def encode(log2n: int, u) -> np.ndarray:
    """x = u G_N over GF(2), natural order (Section 3, Arikan's construction)."""
    n = 1 << log2n
    u = _bits(u, n)
    x = np.empty(n, np.uint8)
    if _load().oracle_encode(log2n, _ptr(u), _ptr(x)) != 0:
        raise ValueError("oracle_encode failed")
    return x


def bhattacharyya(log2n: int, z0: float):
    """(ln Z_i, ln(1 - Z_i)) for the N synthetic channels (Section 3)."""
    n = 1 << log2n
    lz = np.empty(n, np.float64)
    lw = np.empty(n, np.float64)
    if _load().oracle_bhattacharyya(log2n, float(z0), _ptr(lz), _ptr(lw)) != 0:
        raise ValueError("oracle_bhattacharyya failed")
    return lz, lw


def frozen_set(log2n: int, z0: float, n_frozen: int = -1, fer_bound: float = 0.1):
    """Frozen mask (1 = frozen), number frozen, reliabilities r_i = ln((1-Z)/Z).

    n_frozen >= 0 freezes that many least reliable channels; n_frozen = -1
    applies the union-bound rule sum_{info} Z_i <= fer_bound (Section 3)."""
    n = 1 << log2n
    mask = np.empty(n, np.uint8)
    r = np.empty(n, np.float64)
    nf = _load().oracle_frozen_set(log2n, float(z0), int(n_frozen), float(fer_bound),
                                   _ptr(mask), _ptr(r))
    if nf < 0:
        raise ValueError("oracle_frozen_set failed")
    return mask, int(nf), r


def sc_decode(llr, frozen, fval, boxplus: bool = False, teacher=None, want_leaf: bool = False,
              want_beta: bool = False):
    """SC-decode one frame (Section 4).

    Returns (u_hat, leaf_llr or None, beta or None).  Min-sum runs in FP32 and
    its leaf LLRs are float32; box-plus runs in FP64 and its leaf LLRs are
    float64.  With ``teacher`` the partial sums use the teacher's bits."""
    llr = np.ascontiguousarray(np.asarray(llr, dtype=np.float32))
    n = llr.shape[0]
    log2n = n.bit_length() - 1
    if (1 << log2n) != n:
        raise ValueError("N must be a power of two")
    frozen = _bits(frozen, n)
    fval = _bits(fval, n)
    t = _bits(teacher, n) if teacher is not None else None
    u = np.empty(n, np.uint8)
    leaf = np.empty(n, np.float64 if boxplus else np.float32) if want_leaf else None
    beta = np.empty(n, np.uint8) if want_beta else None
    rc = _load().oracle_sc_decode(log2n, 1 if boxplus else 0, _ptr(llr), _ptr(frozen),
                                  _ptr(fval), _ptr(t), _ptr(u), _ptr(leaf), _ptr(beta))
    if rc != 0:
        raise ValueError("oracle_sc_decode failed")
    return u, leaf, beta


def sc_decode_batch(llr, frozen, fval, boxplus: bool = False, n_threads: int | None = None):
    """Decode frames llr[k] (shape (F, N)) with one frame per host thread.

    ``frozen`` is either one mask of shape (N,) shared by all frames or (F, N)."""
    llr = np.ascontiguousarray(np.asarray(llr, dtype=np.float32))
    nfr, n = llr.shape
    log2n = n.bit_length() - 1
    frozen = np.ascontiguousarray(np.asarray(frozen, dtype=np.uint8))
    shared = 1 if frozen.ndim == 1 else 0
    fval = np.ascontiguousarray(np.asarray(fval, dtype=np.uint8))
    u = np.empty((nfr, n), np.uint8)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    _load().oracle_sc_decode_batch(log2n, 1 if boxplus else 0, nfr, shared, _ptr(llr),
                                   _ptr(frozen), _ptr(fval), _ptr(u), int(n_threads))
    return u


# Fixed point (Section 4): LLRs as integers in units of 2^-FIXED_FRAC,
# saturated to +-FIXED_MAX; the phi table has FIXED_TABLE_LEN entries.
FIXED_FRAC = 4
FIXED_MAX = 32767
FIXED_TABLE_LEN = 256
FIXED_MINSUM, FIXED_PHI = 0, 1
# Saturating min-sum on 8-bit integers: |L| <= FIXED8_MAX in any units.
FIXED_MINSUM8 = 2
FIXED8_MAX = 127


def phi_table(frac: int = FIXED_FRAC, length: int = FIXED_TABLE_LEN) -> np.ndarray:
    """T[i] = round(phi(i 2^-frac) 2^frac), phi(x) = -ln tanh(x/2) (Section 4's
    table), T[0] = FIXED_MAX."""
    out = np.empty(length, np.int32)
    if _load().oracle_phi_table(int(frac), int(length), _ptr(out)) != 0:
        raise ValueError("oracle_phi_table failed")
    return out


def quantize(llr, frac: int = FIXED_FRAC, limit: int = FIXED_MAX) -> np.ndarray:
    """Channel LLRs to fixed point: round(L 2^frac) (round half to even),
    saturated to +-limit."""
    q = np.round(np.asarray(llr, np.float64) * (1 << frac))
    return np.clip(q, -limit, limit).astype(np.int32)


def sc_decode_fixed(llr_q, frozen, fval, kind: int = FIXED_MINSUM, teacher=None, want_leaf: bool = False,
                    table=None):
    """Fixed-point SC (Section 4): kind FIXED_MINSUM (saturating min-sum) or
    FIXED_PHI (phi-table exact update).  llr_q: N integers.  Returns (u_hat,
    leaf LLRs int32 or None)."""
    llr = np.ascontiguousarray(np.asarray(llr_q, dtype=np.int32))
    n = llr.shape[0]
    log2n = n.bit_length() - 1
    if (1 << log2n) != n:
        raise ValueError("N must be a power of two")
    frozen = _bits(frozen, n)
    fval = _bits(fval, n)
    t = _bits(teacher, n) if teacher is not None else None
    tab = np.ascontiguousarray(table if table is not None else phi_table(), np.int32)
    u = np.empty(n, np.uint8)
    leaf = np.empty(n, np.int32) if want_leaf else None
    rc = _load().oracle_sc_decode_fixed(log2n, int(kind), _ptr(llr), _ptr(frozen), _ptr(fval), _ptr(t),
                                        _ptr(u), _ptr(leaf), _ptr(tab), int(tab.size))
    if rc != 0:
        raise ValueError("oracle_sc_decode_fixed failed")
    return u, leaf


def f_fixed(kind: int, a: int, b: int, table=None) -> int:
    tab = np.ascontiguousarray(table if table is not None else phi_table(), np.int32)
    return int(_load().oracle_f_fixed(int(kind), int(a), int(b), _ptr(tab), int(tab.size)))


def scl_decode(llr, frozen, fval, list_size: int):
    """SC list decoding with FP32 min-sum updates and the LLR path metric
    (Section 4 names list decoders as the improvement of SC).  Returns
    (u_hat of the path of least metric, that metric as float32)."""
    llr = np.ascontiguousarray(np.asarray(llr, dtype=np.float32))
    n = llr.shape[0]
    log2n = n.bit_length() - 1
    if (1 << log2n) != n:
        raise ValueError("N must be a power of two")
    frozen = _bits(frozen, n)
    fval = _bits(fval, n)
    u = np.empty(n, np.uint8)
    pm = ctypes.c_float(0.0)
    if _load().oracle_scl_decode(log2n, int(list_size), _ptr(llr), _ptr(frozen), _ptr(fval), _ptr(u),
                                 ctypes.addressof(pm)) != 0:
        raise ValueError("oracle_scl_decode failed")
    return u, np.float32(pm.value)


def f_minsum(a: float, b: float) -> float:
    return float(_load().oracle_f_minsum(a, b))


def g_f32(a: float, b: float, u: int) -> float:
    return float(_load().oracle_g_f32(a, b, int(u)))


def f_boxplus(a: float, b: float) -> float:
    return float(_load().oracle_f_boxplus(a, b))
