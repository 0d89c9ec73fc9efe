"""Checks on the generated gfx950 code (no GPU needed): every kernel runs
without scratch memory (the register-resident decoder does not spill), and
nothing writes through the scalar data cache (stores go through vector
memory instructions)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ISA = os.path.join(ROOT, "paper_1204_5882_amd", "_build", "sc_device-gfx950.s")


@pytest.mark.skipif(not os.path.exists(ISA), reason="device assembly not built")
def test_kernels_do_not_spill():
    text = open(ISA).read()
    sizes = [int(m.group(1)) for m in re.finditer(r"\.private_segment_fixed_size:\s+(\d+)", text)]
    assert sizes and all(s == 0 for s in sizes), "a kernel uses scratch memory"
    assert "scratch_store" not in text and "buffer_store_dword" not in text.replace("buffer_store_dword v", "")


@pytest.mark.skipif(not os.path.exists(ISA), reason="device assembly not built")
def test_no_scalar_cache_writes():
    text = open(ISA).read()
    bad = re.findall(r"^\s*(s_store_\w+|s_buffer_store\w*|s_scratch_store\w*|s_atomic\w*|s_buffer_atomic\w*|"
                     r"s_dcache_wb\w*|s_dcache_discard\w*)", text, flags=re.M)
    assert not bad, sorted(set(bad))
