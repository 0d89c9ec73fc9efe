"""The oracle reproduces the committed fixtures in tests/golden (written by
tests/golden/make_golden.py from the oracle itself): a guard against silent
changes to the oracle's arithmetic."""
import glob
import json
import os

import numpy as np
import pytest

import oracle
import synth

# decoding fixtures (the generator's known-answer vectors are checked in test_oracle_fer.py)
GOLDEN = sorted(p for p in glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.json"))
                if not os.path.basename(p).startswith("philox"))


def load_fixture(path):
    d = json.load(open(path))
    n = 1 << d["log2n"]

    def bits(key):
        return synth.unpack_bits(np.array([int(w, 16) for w in d[key]], np.uint32), n)

    llr = np.array([int(w, 16) for w in d["llr_f32_hex"]], np.uint32).view(np.float32)
    return d, bits("frozen_mask"), bits("frozen_vals"), bits("u"), llr, bits("u_hat")


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p) for p in GOLDEN])
def test_oracle_reproduces_fixture(path):
    d, mask, fval, u, llr, uh_ref = load_fixture(path)
    bp = d["f_kind"] == "boxplus"
    m2, nf, _ = oracle.frozen_set(d["log2n"], d["z0"], d["n_frozen"])
    assert np.array_equal(m2, mask) and nf == int(mask.sum())
    u2, fv2, llr2 = synth.frame(d["seed"], d["log2n"], d["channel"], d["param"], mask,
                                lambda v: oracle.encode(d["log2n"], v))
    assert np.array_equal(u2, u) and np.array_equal(fv2, fval)
    assert np.array_equal(llr2.view(np.uint32), llr.view(np.uint32))
    uh, leaf, _ = oracle.sc_decode(llr, mask, fval, boxplus=bp, want_leaf=True)
    assert np.array_equal(uh, uh_ref)
    if bp:
        np.testing.assert_allclose(leaf, np.array(d["leaf_llr"]), rtol=1e-14, atol=1e-300)
    else:
        ref = np.array([int(w, 16) for w in d["leaf_llr"]], np.uint32)
        assert np.array_equal(leaf.view(np.uint32), ref)
