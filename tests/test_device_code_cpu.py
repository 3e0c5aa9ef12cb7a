"""CPU: the library's device code writes memory only through vector stores.

Compiles each translation unit of liblbtr for gfx950 to assembly (as the
build does, without linking) and checks that no instruction writes through
the scalar data cache: no scalar stores or atomics, no scalar-cache
write-back or discard. This file only reads assembly built here from this
repository's sources.
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_03933_amd", "csrc")
FORBIDDEN = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic_|s_buffer_atomic|s_dcache_wb|s_dcache_discard)", re.M)

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")


def _asm(src, defines):
    from paper_2603_03933_amd import build as B

    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        cmd = [B._hipcc(), *B._flags(), "--cuda-device-only", "-S", *defines, "-o", out, os.path.join(CSRC, src)]
        subprocess.run(cmd, check=True, capture_output=True, cwd=CSRC)
        return open(out).read()


@pytest.mark.parametrize("src,defines", [("lb_lib.hip", []), ("inst.hip", ["-DLB_N=128"]), ("inst.hip", ["-DLB_N=64"]), ("inst.hip", ["-DLB_N=256"])])
def test_no_scalar_cache_writes(src, defines):
    asm = _asm(src, defines)
    assert "amdgcn" in asm or ".amdhsa" in asm
    bad = FORBIDDEN.findall(asm)
    assert not bad, sorted(set(bad))
