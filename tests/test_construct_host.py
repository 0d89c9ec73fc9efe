"""Host side of the degrading construction, no GPU needed: the frozen-set
rule on per-channel error probabilities (polar_frozen_from_pe) against the
oracle's rule, bit-exact, and the argument checks of the device entry point
(all rejected before any device call)."""
import numpy as np
import pytest

from oracle import construct as C


def _lp():
    from paper_1204_5882_amd import polar as lp

    lp.load()
    return lp


def _mask_bits(words, n):
    from paper_1204_5882_amd import polar as lp

    return ((words[np.arange(n) >> 5] >> (np.arange(n) & 31).astype(np.uint32)) & 1).astype(np.uint8)


@pytest.mark.parametrize("log2n", [0, 3, 8, 14])
@pytest.mark.parametrize("ties", [False, True])
def test_frozen_from_pe_matches_oracle_rule(log2n, ties):
    lp = _lp()
    n = 1 << log2n
    g = np.random.default_rng(40 + log2n)
    pe = 10.0 ** (-12 * g.random(n)) / 2
    if ties:  # many exact ties, as a BEC or a coarse merge gives
        pe = np.round(pe, 3)
    for nf_req, bound in [(-1, 0.1), (-1, 1e-3), (-1, 0.0), (0, 0.1), (n // 3, 0.1), (n, 0.1)]:
        ref_mask, ref_nf = C.frozen_from_pe(pe, nf_req, bound)
        words, nf = lp.frozen_from_pe(log2n, pe, nf_req, bound)
        assert nf == ref_nf, (nf_req, bound)
        assert np.array_equal(_mask_bits(words, n), ref_mask), (nf_req, bound)


def test_frozen_from_pe_rejects_bad_input():
    lp = _lp()
    with pytest.raises(lp.PolarError):
        lp.frozen_from_pe(4, np.full(16, 1.5))
    with pytest.raises(lp.PolarError):
        lp.frozen_from_pe(4, np.full(16, 0.1), n_frozen=17)
    with pytest.raises(lp.PolarError):
        lp.frozen_from_pe(4, np.full(16, 0.1), n_frozen=-1, fer_bound=-1.0)


def test_construct_argument_checks():
    """Every argument error is caught on the host; the fake workspace and
    output pointers are never dereferenced."""
    import ctypes

    lp = _lp()
    lib = lp.load()
    fake = 1 << 20  # 256-byte aligned, never touched

    def call(log2n, w0, mu, ws_bytes=1 << 40, ws=fake, pe=fake):
        w0 = np.ascontiguousarray(np.asarray(w0, np.float64).reshape(-1, 2))
        return lib.polar_construct_degrade(log2n, w0.ctypes.data, w0.shape[0], mu, ws, ws_bytes, pe, None)

    bsc = [[0.98, 0.02]]
    assert call(-1, bsc, 16) == lp.POLAR_E_INVAL
    assert call(25, bsc, 16) == lp.POLAR_E_INVAL
    assert call(10, bsc, 1) == lp.POLAR_E_INVAL
    assert call(10, bsc, 65) == lp.POLAR_E_INVAL
    assert call(10, [[0.02, 0.98]], 16) == lp.POLAR_E_INVAL          # a < b
    assert call(10, [[0.9, 0.05]], 16) == lp.POLAR_E_INVAL           # sums to 0.95
    assert call(10, [[1.02, -0.02]], 16) == lp.POLAR_E_INVAL         # b < 0
    assert call(10, bsc, 16, ws=fake + 8) == lp.POLAR_E_INVAL        # misaligned workspace
    assert call(10, bsc, 16, ws=None) == lp.POLAR_E_INVAL
    need = lp.construct_workspace_bytes(10, 16, 1)
    assert need > 0
    assert call(10, bsc, 16, ws_bytes=need - 1) == lp.POLAR_E_NOMEM
    assert lp.construct_workspace_bytes(10, 65, 1) == 0
    assert lp.construct_workspace_bytes(25, 16, 1) == 0
    # n = 24, mu = 64: 2^23 + 2^22 channels of 64 pairs of doubles, plus counts
    assert lp.construct_workspace_bytes(24, 64, 1) >= (3 << 22) * 64 * 16
