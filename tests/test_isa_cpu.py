"""Compiled-code checks of the compositing kernels (CPU: hipcc cross-compiles
gfx950 here).

The persistent compositing kernels pop work items for the whole wave; their
item loop and entry loop must stay wave-uniform.  A lane-dependent branch
around the pop once let the compiler drop lane 0 from EXEC at the loop's back
edge, after which the wave re-read a stale item id and never finished.  The
signature of a divergent loop exit in gfx9 code is ``s_andn2_b64 exec, exec,
...`` before the back edge; these kernels must contain none.  The check also
asserts that no scalar memory store or scalar atomic is emitted anywhere."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_16144_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


def _asm(src, tmp_path):
    out = str(tmp_path / (os.path.basename(src) + ".s"))
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-S", "--cuda-device-only", os.path.join(CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return open(out).read()


def _kernels(asm, pattern):
    out = {}
    for name in re.findall(r"^(_ZN\w*" + pattern + r"\w*):", asm, re.M):
        body = asm[asm.index(name + ":"):]
        body = body[:body.index(".Lfunc_end")]
        out[name] = [l.strip() for l in body.splitlines() if l.strip() and not l.strip().startswith((";", "."))]
    return out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_persistent_compositing_loops_are_wave_uniform(tmp_path):
    asm = _asm("raster.hip", tmp_path)
    ks = _kernels(asm, "k_raster_(?:fwd|bwd)")
    # (fwd x {f32, bf16} + bwd x {f32, bf16} x {upstream, fused L1, colour given})
    # x {timed, counting}
    assert len(ks) == 16
    for name, lines in ks.items():
        bad = [l for l in lines if l.startswith("s_andn2_b64 exec, exec")]
        assert not bad, (name, bad)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", sorted(f for f in os.listdir(CSRC) if f.endswith(".hip")))
def test_no_scalar_memory_writes(src, tmp_path):
    asm = _asm(src, tmp_path)
    bad = re.findall(r"^\s+(s_(?:store|buffer_store|atomic|buffer_atomic|dcache_wb|dcache_discard|scratch_store)\w*)",
                     asm, re.M)
    assert not bad, bad
