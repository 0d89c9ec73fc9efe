"""Checks on the generated gfx950 code (no GPU needed): every kernel runs
without scratch memory (the register-resident decoder does not spill), and
nothing writes through the scalar data cache (stores go through vector
memory instructions)."""
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ISA_FILES = sorted(glob.glob(os.path.join(ROOT, "paper_1204_5882_amd", "_build", "*.gfx950.isa")))


def _isa():
    return "\n".join(open(f).read() for f in ISA_FILES)


@pytest.mark.skipif(not ISA_FILES, reason="device assembly not built")
def test_every_decoder_variant_has_device_code():
    names = {os.path.basename(f).split(".")[0] for f in ISA_FILES}
    variants = {os.path.splitext(os.path.basename(f))[0]
                for f in glob.glob(os.path.join(ROOT, "paper_1204_5882_amd", "csrc", "variants", "*.hip"))}
    assert variants and variants <= names
    assert "sc_device" in names


@pytest.mark.skipif(not ISA_FILES, reason="device assembly not built")
def test_kernels_do_not_spill():
    text = _isa()
    sizes = [int(m.group(1)) for m in re.finditer(r"\.private_segment_fixed_size:\s+(\d+)", text)]
    assert sizes and all(s == 0 for s in sizes), "a kernel uses scratch memory"
    assert "scratch_store" not in text and "buffer_store_dword" not in text.replace("buffer_store_dword v", "")


@pytest.mark.skipif(not ISA_FILES, reason="device assembly not built")
def test_no_scalar_cache_writes():
    text = _isa()
    bad = re.findall(r"^\s*(s_store_\w+|s_buffer_store\w*|s_scratch_store\w*|s_atomic\w*|s_buffer_atomic\w*|"
                     r"s_dcache_wb\w*|s_dcache_discard\w*)", text, flags=re.M)
    assert not bad, sorted(set(bad))
