"""CPU guard over the device code this repository builds: the gfx950
assembly of every kernel source must write memory through vector memory
instructions only (no scalar-unit stores, scalar atomics, or scalar-cache
write-back/discard).  The resident-key kernel must read its key with vector
loads into scalar registers (never through the scalar cache), and its loops
must all be wave-uniform: a loop whose exit depends on the exec mask could
leave some lanes of a worker behind, looping on a stale ring position and
never reading the stop flag."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
CSRC = os.path.join(ROOT, "paper_2004_09252_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
SOURCES = ["page_cipher.hip", "mlp_kernels.hip", "resident.hip"]
FORBIDDEN = re.compile(
    r"^\s*(s_(?:buffer_|scratch_)?(?:store|atomic)\w*|s_dcache_(?:wb|discard)\w*)\b",
    re.M)


def _asm(src, tmp_path):
    out = tmp_path / (src + ".s")
    r = subprocess.run(
        [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
         "--cuda-device-only", "-S", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", INCLUDE, "-I", CSRC,
         os.path.join(CSRC, src), "-o", str(out)],
        capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out.read_text()


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not present")
@pytest.mark.parametrize("src", SOURCES)
def test_no_scalar_memory_writes(src, tmp_path):
    text = _asm(src, tmp_path)
    assert "s_endpgm" in text
    bad = sorted(set(m.group(1) for m in FORBIDDEN.finditer(text)))
    assert not bad, bad


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not present")
def test_resident_key_loads_bypass_scalar_cache(tmp_path):
    text = _asm("resident.hip", tmp_path)
    for name in ("ms_resident_pages_r20:", "ms_resident_pages_s20:"):
        body = text[text.index(name):]
        body = body[:body.index(".Lfunc_end")]
        # the eight key words: system-scope vector loads, then readfirstlane
        by_base = {}
        for base, off in re.findall(r"global_load_dword v\d+, v\d+, "
                                    r"(s\[\d+:\d+\])(?: offset:(\d+))? "
                                    r"sc0 sc1", body):
            by_base.setdefault(base, set()).add(int(off or 0))
        key = set(range(0, 32, 4))
        assert any(key <= offs for offs in by_base.values()), (name, by_base)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not present")
def test_resident_loops_are_wave_uniform(tmp_path):
    text = _asm("resident.hip", tmp_path)
    for name in ["ms_resident_pages_%s%d:" % (c, r)
                 for c in "rs" for r in (20, 12, 8)]:
        rounds = name
        body = text[text.index(name):]
        body = body[:body.index(".Lfunc_end")]
        assert "s_cbranch_execnz" not in body, rounds
        assert not re.search(r"s_andn2_b64 exec, exec", body), rounds
        assert not re.search(r"s_xor_b64 exec, exec", body), rounds
