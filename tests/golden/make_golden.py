"""Write the small regression fixtures in this folder.

Calls only the CPU oracle (``oracle/``) and the seeded input generator
(``synth``).  Run from the repository root:  python tests/golden/make_golden.py

Each fixture records the section of the paper its arithmetic follows:
SC decoding (Section 4, recursive decoder of [Ari08]) on frozen sets chosen
from the synthetic-channel reliabilities (Section 3), with the frozen values
revealed as in Section 1.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = [
    # name, log2n, channel, param, z0, n_frozen, boxplus, seed
    ("minsum_bsc_n256", 8, "bsc", 0.05, synth.bsc_z0(0.05), 96, False, 31),
    ("minsum_biawgn_n128", 7, "biawgn", 0.9, synth.biawgn_z0(0.9), 70, False, 32),
    ("boxplus_biawgn_n64", 6, "biawgn", 0.97, synth.biawgn_z0(0.97), 35, True, 33),
]


def _hex_words(bits):
    return [f"{w:08x}" for w in synth.pack_bits(bits).tolist()]


def main():
    for name, log2n, ch, prm, z0, nf, bp, seed in CASES:
        mask, got, _ = oracle.frozen_set(log2n, z0, nf)
        u, fval, llr = synth.frame(seed, log2n, ch, prm, mask, lambda v: oracle.encode(log2n, v))
        uh, leaf, _ = oracle.sc_decode(llr, mask, fval, boxplus=bp, want_leaf=True)
        doc = {
            "cite": "SC decoding, Section 4 (recursive decoder, [Ari08]); frozen set by "
                    "Bhattacharyya reliability, Section 3; frozen values revealed, Section 1",
            "writer": "tests/golden/make_golden.py (oracle/ and synth only)",
            "log2n": log2n, "channel": ch, "param": prm, "z0": z0, "n_frozen": got,
            "f_kind": "boxplus" if bp else "minsum", "seed": seed,
            "frozen_mask": _hex_words(mask), "frozen_vals": _hex_words(fval),
            "u": _hex_words(u),
            "llr_f32_hex": [f"{v:08x}" for v in llr.view(np.uint32).tolist()],
            "u_hat": _hex_words(uh),
            "leaf_llr": ([float(v) for v in leaf] if bp else
                         [f"{v:08x}" for v in leaf.astype(np.float32).view(np.uint32).tolist()]),
        }
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(doc, fh, indent=0)
            fh.write("\n")
        print("wrote", name)


if __name__ == "__main__":
    main()
