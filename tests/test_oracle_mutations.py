"""The pins are sharp: each plausible slip planted in a copy of the oracle's C
source (dropped term, wrong sign, transposed operand, wrong tie rule, swapped
children) makes one of the independent references disagree.  Everything here
runs on the CPU; the real oracle is untouched."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import naive

SRC = os.path.join(os.path.dirname(oracle.__file__), "sc_oracle.c")

MUTATIONS = {
    "combine_drops_xor": ("beta[j] = (uint8_t)(bl[j] ^ br[j]);", "beta[j] = (uint8_t)(bl[j]);"),
    "g_sign_flipped": ("static float g_f32(float a, float b, int u) { return u ? b - a : b + a; }",
                       "static float g_f32(float a, float b, int u) { return u ? b + a : b - a; }"),
    "g_operands_transposed": ("a[j] = g_f32(alpha[j], alpha[j + h], bl[j]);",
                              "a[j] = g_f32(alpha[j + h], alpha[j], bl[j]);"),
    "decision_zero_as_one": ("int u = c->frozen[off] ? c->fval[off] : (L < 0.0f);",
                             "int u = c->frozen[off] ? c->fval[off] : (L <= 0.0f);"),
    "f_uses_max": ("float m = fminf(fabsf(a), fabsf(b));", "float m = fmaxf(fabsf(a), fabsf(b));"),
    "encode_drops_xor": ("a[j] = (uint8_t)(u[j] ^ u[j + h]);", "a[j] = (uint8_t)(u[j]);"),
    "bhatt_children_swapped": ("bz[2 * j] = mz;", "bz[2 * j] = pz;"),
    "boxplus_log_sign": ("return s * (m + log1p(exp(-(A + B))) - log1p(exp(-fabs(A - B))));",
                         "return s * (m - log1p(exp(-(A + B))) - log1p(exp(-fabs(A - B))));"),
    "fixed_g_unsaturated": ("return sat_to(u ? b - a : b + a, c->max); }", "return u ? b - a : b + a; }"),
    "fixed8_saturates_at_int16": ("const int32_t lim = kind == 2 ? FIXED8_MAX : FIXED_MAX;",
                                  "const int32_t lim = FIXED_MAX;"),
    "fixed_phi_sum_drops_term": ("int32_t s = fx_phi(c, A) + fx_phi(c, B);", "int32_t s = fx_phi(c, A);"),
    "fixed_phi_drops_min_clamp": ("r = t < m ? t : m;", "r = t;"),
    "phi_table_shifted": ("double v = log1p(2.0 / expm1(i * step)) / step;",
                          "double v = log1p(2.0 / expm1((i + 1) * step)) / step;"),
}


def _build_mutant(tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    src = src.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    c.write_text(src)
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, str(c), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    lib.oracle_sc_decode.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P]
    lib.oracle_encode.argtypes = [ctypes.c_int, P, P]
    lib.oracle_bhattacharyya.argtypes = [ctypes.c_int, ctypes.c_double, P, P]
    lib.oracle_sc_decode_fixed.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, ctypes.c_int]
    lib.oracle_phi_table.argtypes = [ctypes.c_int, ctypes.c_int, P]
    return lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _decode(lib, llr, mask, fval, boxplus=False):
    n = llr.size
    u = np.empty(n, np.uint8)
    leaf = np.empty(n, np.float64 if boxplus else np.float32)
    lib.oracle_sc_decode(n.bit_length() - 1, int(boxplus), _p(llr), _p(mask), _p(fval), None,
                         _p(u), _p(leaf), None)
    return u, leaf


def _minsum_pin_catches(lib):
    g = np.random.default_rng(4)
    for log2n in (3, 5, 6):
        n = 1 << log2n
        for _ in range(6):
            llr = g.integers(-2, 3, n).astype(np.float32)
            mask = (g.random(n) < 0.4).astype(np.uint8)
            fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
            u, leaf = _decode(lib, llr, mask, fval)
            un, ln = naive.naive_sc(llr, mask, fval)
            if not (np.array_equal(u, un) and np.array_equal(leaf.view(np.uint32), ln.view(np.uint32))):
                return True
    return False


def _boxplus_pin_catches(lib):
    g = np.random.default_rng(8)
    for log2n in (2, 3, 4):
        n = 1 << log2n
        for _ in range(4):
            llr = (3.0 * g.standard_normal(n)).astype(np.float32)
            mask = (g.random(n) < 0.3).astype(np.uint8)
            fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
            _, leaf = _decode(lib, llr, mask, fval, boxplus=True)
            _, lb = naive.brute_sc(llr, mask, fval)
            if not np.allclose(leaf, lb, rtol=1e-11, atol=1e-11):
                return True
    return False


def _encode_pin_catches(lib):
    g = np.random.default_rng(2)
    u = g.integers(0, 2, 64).astype(np.uint8)
    x = np.empty(64, np.uint8)
    lib.oracle_encode(6, _p(u), _p(x))
    return not np.array_equal(x, naive.encode_matrix(u))


def _bhatt_pin_catches(lib):
    lz = np.empty(4)
    lw = np.empty(4)
    lib.oracle_bhattacharyya(2, ctypes.c_double(0.5), _p(lz), _p(lw))
    return not np.allclose(np.exp(lz), [0.9375, 0.5625, 0.4375, 0.0625])


def _fixed_pin_catches(lib):
    """The fixed-point decoder against the per-bit naive decoder in the same
    integer arithmetic (saturation exercised), every check update."""
    g = np.random.default_rng(12)
    table = oracle.phi_table()
    tab = np.ascontiguousarray(table, np.int32)
    for kind in (0, 1, 2):
        lim = 127 if kind == 2 else 32767
        for log2n in (2, 4, 5):
            n = 1 << log2n
            for trial in range(6):
                llr = (g.integers(-lim, lim + 1, n) if trial % 2 else g.integers(-90, 91, n)).astype(np.int32)
                mask = (g.random(n) < 0.4).astype(np.uint8)
                fval = (g.integers(0, 2, n) & mask).astype(np.uint8)
                u = np.empty(n, np.uint8)
                leaf = np.empty(n, np.int32)
                lib.oracle_sc_decode_fixed(log2n, kind, _p(llr), _p(mask), _p(fval), None, _p(u), _p(leaf),
                                           _p(tab), int(tab.size))
                un, ln = naive.naive_sc_fixed(llr, mask, fval, kind, table)
                if not (np.array_equal(u, un) and np.array_equal(leaf, ln)):
                    return True
    return False


def _phi_table_pin_catches(lib):
    """The table against phi = -ln tanh(x/2) at 60 digits."""
    import mpmath

    mpmath.mp.dps = 60
    out = np.empty(oracle.FIXED_TABLE_LEN, np.int32)
    lib.oracle_phi_table(oracle.FIXED_FRAC, oracle.FIXED_TABLE_LEN, _p(out))
    step = mpmath.mpf(1) / (1 << oracle.FIXED_FRAC)
    for i in range(1, out.size):
        v = -mpmath.log(mpmath.tanh(i * step / 2)) / step
        if out[i] != min(oracle.FIXED_MAX, int(mpmath.floor(v + mpmath.mpf("0.5")))):
            return True
    return False


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    lib = _build_mutant(tmp_path, name)
    caught = {
        "encode_drops_xor": _encode_pin_catches,
        "bhatt_children_swapped": _bhatt_pin_catches,
        "boxplus_log_sign": _boxplus_pin_catches,
        "fixed_g_unsaturated": _fixed_pin_catches,
        "fixed8_saturates_at_int16": _fixed_pin_catches,
        "fixed_phi_sum_drops_term": _fixed_pin_catches,
        "fixed_phi_drops_min_clamp": _fixed_pin_catches,
        "phi_table_shifted": _phi_table_pin_catches,
    }.get(name, _minsum_pin_catches)(lib)
    assert caught, f"mutation {name} was not detected by its pin"


def test_unmutated_source_passes_the_same_pins(tmp_path):
    src = open(SRC).read()
    c = tmp_path / "clean.c"
    c.write_text(src)
    so = tmp_path / "clean.so"
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, str(c), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    lib.oracle_sc_decode.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P]
    lib.oracle_encode.argtypes = [ctypes.c_int, P, P]
    lib.oracle_bhattacharyya.argtypes = [ctypes.c_int, ctypes.c_double, P, P]
    lib.oracle_sc_decode_fixed.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, ctypes.c_int]
    lib.oracle_phi_table.argtypes = [ctypes.c_int, ctypes.c_int, P]
    assert not _fixed_pin_catches(lib)
    assert not _phi_table_pin_catches(lib)
    assert not _minsum_pin_catches(lib)
    assert not _boxplus_pin_catches(lib)
    assert not _encode_pin_catches(lib)
    assert not _bhatt_pin_catches(lib)
