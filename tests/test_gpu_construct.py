"""GPU parity of the degrading construction (polar_construct_degrade) with
the oracle (oracle/construct.py): every synthetic channel's error
probability on codes the oracle builds whole, sampled channels (each built
by the oracle along its own path) at N = 2^20 and 2^24, the BEC against the
Bhattacharyya closed form, and the frozen sets taken from the device's
values.  Both sides merge in the same order with the same double-precision
products and sums, so the values agree to the last bit unless a binning
decision falls within an ulp of a bin edge (the entropy's log2 may differ
by an ulp between the host library and the device); the tests require
agreement to 1e-12 relative and report how many values are bit-identical."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import construct as C

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


def _gpu_pe(log2n, w0, mu):
    import torch

    from paper_1204_5882_amd import polar as lp

    pe = lp.construct_degrade(log2n, w0, mu)
    torch.cuda.synchronize()
    return pe.cpu().numpy()


def _compare(got, ref, what):
    assert got.shape == ref.shape, what
    same = int((got == ref).sum())
    _say(f"  {what}: {same}/{ref.size} bit-identical")
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=0, err_msg=what)


CHANNELS = {
    "bsc0.02": C.bsc(0.02),
    "bsc0.11": C.bsc(0.11),
    "bec0.3": C.bec(0.3),
    "biawgn0.97": synth.biawgn_channel(0.97, 300),
}


@pytest.mark.parametrize("name", sorted(CHANNELS))
@pytest.mark.parametrize("log2n,mu", [(0, 16), (1, 2), (3, 4), (6, 64), (9, 16), (10, 64)])
def test_every_channel_matches_oracle(name, log2n, mu):
    w0 = CHANNELS[name]
    _say(f"case: construct {name} log2n={log2n} mu={mu}")
    got = _gpu_pe(log2n, w0, mu)
    ref = C.synthetic_error_probabilities(log2n, w0, mu)
    _compare(got, ref, f"{name} n={log2n} mu={mu}")


def test_many_outputs_root_merge():
    """A start channel of 5000 outputs (several 64-lane chunks and a ragged
    tail) merged at the root."""
    w0 = synth.biawgn_channel(1.2, 5000)
    _say("case: construct biawgn 5000 outputs log2n=5 mu=32")
    _compare(_gpu_pe(5, w0, 32), C.synthetic_error_probabilities(5, w0, 32), "biawgn 5000 outputs")


@pytest.mark.parametrize("log2n,mu,name", [(20, 32, "bsc0.02"), (20, 16, "biawgn0.97"), (24, 16, "bsc0.02")])
def test_full_size_sampled_channels(log2n, mu, name):
    w0 = CHANNELS[name]
    _say(f"case: construct {name} log2n={log2n} mu={mu} (sampled)")
    got = _gpu_pe(log2n, w0, mu)
    n = 1 << log2n
    g = np.random.default_rng(log2n * 100 + mu)
    idx = np.unique(np.concatenate([[0, 1, n // 2, n - 2, n - 1], g.integers(0, n, 24)]))
    ref = np.array([C.channel_error_probability(log2n, int(i), w0, mu) for i in idx])
    _compare(got[idx], ref, f"{name} n={log2n} sampled")
    # each step squares a channel's total mass, so w0's rounding (a few ulps
    # off 1) grows to about 2^n ulps at level n
    assert np.all((got >= 0) & (got <= 0.5 * (1 + 2.0 ** (log2n - 40))))


@pytest.mark.parametrize("log2n", [16, 20])
def test_bec_equals_bhattacharyya_closed_form(log2n):
    """On the BEC the construction is exact: P_e = Z / 2, Z from the pinned
    (ln Z) recursion."""
    eps = 0.4
    _say(f"case: construct bec log2n={log2n}")
    got = _gpu_pe(log2n, C.bec(eps), 8)
    lz, _ = oracle.bhattacharyya(log2n, eps)
    half_z = np.exp(lz) / 2
    big = half_z > 1e-280
    np.testing.assert_allclose(got[big], half_z[big], rtol=1e-10)
    assert np.all(got[~big] < 1e-279)


def test_frozen_set_from_device_values():
    """The library's frozen set from the device's values equals the oracle's
    rule on the same values, and beats (or ties) the Bhattacharyya rule's
    information set at the FER-0.1 union bound."""
    from paper_1204_5882_amd import polar as lp

    log2n, p = 16, 0.02
    _say("case: frozen set from device construction, BSC 2%, N=2^16")
    pe = _gpu_pe(log2n, C.bsc(p), 32)
    words, nf = lp.frozen_from_pe(log2n, pe, -1, 0.1)
    ref_mask, ref_nf = C.frozen_from_pe(pe, -1, 0.1)
    n = 1 << log2n
    bits = ((words[np.arange(n) >> 5] >> (np.arange(n) & 31).astype(np.uint32)) & 1).astype(np.uint8)
    assert nf == ref_nf and np.array_equal(bits, ref_mask)
    _, nf_z, _ = lp.build_frozen_set(log2n, 2 * np.sqrt(p * (1 - p)), -1, 0.1)
    assert nf <= nf_z


def test_two_calls_share_nothing():
    """Back-to-back calls with different sizes and mu on one workspace give
    the same values as fresh calls."""
    import torch

    from paper_1204_5882_amd import polar as lp

    ws = torch.empty(lp.construct_workspace_bytes(12, 64, 300), dtype=torch.uint8, device="cuda")
    _say("case: construct reusing one workspace")
    a = lp.construct_degrade(12, CHANNELS["biawgn0.97"], 64, workspace=ws)
    b = lp.construct_degrade(8, C.bsc(0.05), 4, workspace=ws)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), _gpu_pe(12, CHANNELS["biawgn0.97"], 64))
    assert np.array_equal(b.cpu().numpy(), _gpu_pe(8, C.bsc(0.05), 4))
