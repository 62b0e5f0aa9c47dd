"""Every kernel of the library, compiled for gfx950, is free of scalar-cache writes: no scalar
memory stores or atomics and no scalar-cache write-back or discard instructions (all device writes
go through vector memory instructions).  CPU only: hipcc emits the device assembly here."""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_21459_amd", "csrc")
FORBIDDEN = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic_|s_buffer_atomic_|"
                       r"s_dcache_wb|s_dcache_discard|s_dcache_inv)", re.M)


def _sources():
    import sys

    sys.path.insert(0, ROOT)
    from paper_2511_21459_amd import build

    return build.SOURCES, build.FLAGS, build.HIPCC


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_no_scalar_cache_writes():
    sources, flags, hipcc = _sources()
    with tempfile.TemporaryDirectory() as tmp:
        procs = []
        for src in sources:
            out = os.path.join(tmp, src + ".s")
            cmd = [hipcc, *[f for f in flags if f != "-fPIC"], "--cuda-device-only", "-S",
                   os.path.join(CSRC, src), "-o", out]
            procs.append((src, out, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE)))
        for src, out, p in procs:
            _, err = p.communicate()
            assert p.returncode == 0, err.decode()[-2000:]
            asm = open(out).read()
            if "__global__" in open(os.path.join(CSRC, src)).read():  # else host code only
                assert "v_" in asm, f"{src}: no device code emitted"
            bad = FORBIDDEN.findall(asm)
            assert not bad, f"{src}: {sorted(set(bad))}"
