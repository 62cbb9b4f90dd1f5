"""Compiled-code checks of the compositing kernels (CPU: hipcc cross-compiles
gfx950 here).

The persistent compositing kernels pop work items for the whole wave; their
item loop and entry loop must stay wave-uniform.  A lane-dependent branch
around the pop once let the compiler drop lane 0 from EXEC at the loop's back
edge, after which the wave re-read a stale item id and never finished.  The
signature of a divergent loop exit in gfx9 code is ``s_andn2_b64 exec, exec,
...`` before the back edge; these kernels must contain none.  The check also
asserts that no scalar memory store or scalar atomic is emitted anywhere.

A vector instruction may read a matrix-core (MFMA) result only some cycles
after the MFMA writes it; the compiler pads its own readers with wait states
but not the instructions of an asm statement.  An asm statement that read an
MFMA result first once took stale values (the decoder's sign clamp, whose
signs then disagreed with the loss), so every asm instruction whose source
register was last written by an MFMA must come after a compiler-issued
reader of that MFMA's result in the same block."""
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
    # (fwd x {f32, bf16} x {contributor counts, none} + bwd x {f32, bf16} x
    # {upstream, fused L1, colour given}) x {timed, counting}
    assert len(ks) == 20
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


def _vregs(op):
    m = re.fullmatch(r"v\[(\d+):(\d+)\]", op)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.fullmatch(r"\|?-?v(\d+)\|?", op)
    return {int(m.group(1))} if m else set()


def _operands(line):
    return [o.strip() for o in line.split(None, 1)[1].split(",")] if " " in line else []


def asm_reads_of_mfma_results(asm):
    """Instructions inside asm statements (;;#ASMSTART .. ;;#ASMEND) with a
    source VGPR whose last writer in the same basic block is an MFMA and
    with no compiler-issued vector read of that MFMA's result in between."""
    lines = [l.strip() for l in asm.splitlines()]
    out, in_asm = [], False
    for k, t in enumerate(lines):
        if t.startswith(";;#ASMSTART"):
            in_asm = True
            continue
        if t.startswith(";;#ASMEND"):
            in_asm = False
            continue
        if not in_asm or not t.startswith("v_"):
            continue
        ops = _operands(t)
        for r in set().union(set(), *[_vregs(o) for o in ops[1:]]):
            for kk in range(k - 1, -1, -1):
                u = lines[kk]
                if re.match(r"^\.LBB\w+:", u) or u.startswith(("s_cbranch", "s_branch")):
                    break
                if not u.startswith("v_"):
                    continue
                uo = _operands(u)
                if not uo or r not in _vregs(uo[0]):
                    continue
                if u.startswith("v_mfma"):
                    dst, inner, guarded = _vregs(uo[0]), False, False
                    for b in lines[kk + 1:k]:
                        if b.startswith(";;#ASMSTART"):
                            inner = True
                        elif b.startswith(";;#ASMEND"):
                            inner = False
                        elif not inner and b.startswith("v_") and not b.startswith("v_mfma") and \
                                any(_vregs(o) & dst for o in _operands(b)[1:]):
                            guarded = True
                            break
                    if not guarded:
                        out.append(t)
                break
    return out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", ["decoder.hip", "raster.hip"])
def test_asm_does_not_read_fresh_mfma_results(src, tmp_path):
    asm = _asm(src, tmp_path)
    assert "v_mfma" in asm
    bad = asm_reads_of_mfma_results(asm)
    assert not bad, bad[:5]


def test_mfma_read_check_flags_an_unguarded_asm_read():
    bad = """
\tv_mfma_f32_16x16x32_bf16 v[118:121], v[114:117], v[62:65], v[26:29]
\ts_nop 6
\t;;#ASMSTART
\tv_med3_i32 v207, v118, -1, 1
\t;;#ASMEND
"""
    good = """
\tv_mfma_f32_16x16x32_bf16 v[118:121], v[114:117], v[62:65], v[26:29]
\ts_nop 7
\tv_add_f32_e64 v211, v211, |v118|
\t;;#ASMSTART
\tv_med3_i32 v207, v119, -1, 1
\t;;#ASMEND
"""
    assert asm_reads_of_mfma_results(bad) == ["v_med3_i32 v207, v118, -1, 1"]
    assert asm_reads_of_mfma_results(good) == []
