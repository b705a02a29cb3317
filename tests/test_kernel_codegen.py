"""The gfx950 code of the hot BF16 kernels, compiled here (no GPU needed):
the properties that their speed rests on, checked in the assembly hipcc
writes for this repository's own sources.

* Grouped 3x3 kernels load and store through global instructions, not flat
  ones: a flat access also counts as an LDS operation, so every wait for an
  LDS fragment would wait for the loads in flight as well.
* The weight gradient loads its tiles straight into LDS and, per step,
  waits only for the tile two steps old (`s_waitcnt vmcnt(6)`), behind
  barriers that wait for LDS traffic only.
* The data gradient's grouped kernel uses counted buffer loads and stores.
* None of the 3x3 kernels spills registers, except the grouped first-layer
  kernel's known 3."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2108_10209_amd import build as B


def device_asm(src):
    with tempfile.TemporaryDirectory(prefix="n2f_asm_") as tmp:
        out = os.path.join(tmp, os.path.basename(src) + ".s")
        cmd = [B.HIPCC, *B.FLAGS, "-I", os.path.join(B.ROOT, "include"), "-I", B.CSRC, "-x", "hip",
               "--cuda-device-only", "-S", os.path.join(B.CSRC, src), "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return open(out).read()


def kernels(asm):
    """name -> (body text, vgpr spill count)"""
    bodies = {}
    for m in re.finditer(r"^(_Z\w+):", asm, re.M):
        end = asm.find(".Lfunc_end", m.end())
        bodies[m.group(1)] = asm[m.end():end]
    spills = {m.group(1): int(m.group(2))
              for m in re.finditer(r"\.name:\s+(\S+)\n(?:.*\n){0,20}?\s+\.vgpr_spill_count:\s+(\d+)", asm)}
    return {k: (v, spills.get(k)) for k, v in bodies.items()}


@pytest.fixture(scope="module")
def conv():
    return kernels(device_asm("n2f_conv.hip"))


def find(ks, pattern):
    names = [k for k in ks if re.search(pattern, k)]
    assert names, pattern
    return names


def test_grouped_3x3_kernels_use_global_instructions(conv):
    for name in find(conv, r"k_conv_bf16_groupILi|k_wgrad_bf16_group"):
        body, _ = conv[name]
        flat = re.findall(r"^\s+(flat_\w+)", body, re.M)
        assert not flat, (name, flat[:5])


def test_weight_gradient_loads_tiles_into_lds_with_exact_waits(conv):
    for name in find(conv, r"k_wgrad_bf16(ENS0_9WgradArgs|_group)"):
        body, _ = conv[name]
        dma = re.findall(r"^\s+buffer_load_dwordx4\s.*\blds\b", body, re.M)
        assert len(dma) >= 6, name
        assert re.search(r"s_waitcnt vmcnt\(6\)", body), name
        # an LDS-only barrier: lgkmcnt(0) then s_barrier, with no vmcnt(0) between
        assert re.search(r"s_waitcnt lgkmcnt\(0\)\n\s+s_barrier", body), name


def test_grouped_data_gradient_uses_buffer_accesses(conv):
    body, _ = conv[find(conv, r"k_conv_bf16_groupILi1E")[0]]
    assert re.search(r"^\s+buffer_load_dwordx4\s(?!.*\blds\b)", body, re.M)
    assert re.search(r"^\s+buffer_store_dwordx2\s", body, re.M)


def test_3x3_kernels_do_not_spill(conv):
    for name in find(conv, r"k_conv_bf16|k_wgrad_bf16"):
        _, spill = conv[name]
        limit = 3 if re.search(r"k_conv_bf16_groupILi4E", name) else 0
        assert spill is not None and spill <= limit, (name, spill)
