"""CPU-only checks of the C ABI library: it loads, exports every entry point
the public headers declare, its host-only calls behave, the headers compile
as C, and no cipher kernel uses scratch memory (the paper's section 4.4
requirement that the key and cipher state never leave registers)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
CSRC = os.path.join(ROOT, "paper_2004_09252_amd", "csrc")


def _declared():
    names = set()
    for h in os.listdir(INCLUDE):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(ms_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2004_09252_amd import build, memshield
    if not os.path.exists(memshield.LIB_PATH):
        build.build()
    return memshield.load_library()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 20
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2004_09252_amd import memshield
    assert _declared() <= set(memshield.exported_symbols())


def test_host_only_calls(lib):
    from paper_2004_09252_amd import memshield as ms
    cfg = ms.ms_config_default()
    assert cfg.max_keys == 64 and cfg.rounds == 20
    assert cfg.admission_cap_bytes == 8 << 30
    assert ms.ms_status_str(ms.MS_EAGAIN).startswith("queue full")
    assert ms.ms_status_str(12345) == "unknown status"
    # null context is rejected, not dereferenced
    assert ms.ms_key_destroy(None, 1) == ms.MS_EINVAL
    assert ms.ms_shutdown(None) == ms.MS_OK


def test_bad_config_rejected_before_device_use(lib):
    from paper_2004_09252_amd import memshield as ms
    cfg = ms.ms_config_default()
    cfg.rounds = 7
    st, _ = ms.ms_init(0, cfg)
    assert st == ms.MS_EINVAL
    cfg = ms.ms_config_default()
    cfg.queue_depth = 1000   # not a power of two
    st, _ = ms.ms_init(0, cfg)
    assert st == ms.MS_EINVAL
    for field, value in (("host_stage_slots", 1), ("host_stage_slots", 17),
                         ("host_chunk_pages", 65537)):
        cfg = ms.ms_config_default()
        setattr(cfg, field, value)
        st, _ = ms.ms_init(0, cfg)
        assert st == ms.MS_EINVAL, field


def test_host_path_defaults_and_null_context(lib):
    from paper_2004_09252_amd import memshield as ms
    cfg = ms.ms_config_default()
    assert cfg.host_chunk_pages == 16384 and cfg.host_stage_slots == 3
    assert cfg.host_mapped_waves == 128
    n = ms.linear_nonce(0, 1, 0)
    assert ms.ms_encrypt_host_pages(None, 1, None, None, 1, n, 0) == \
        ms.MS_EINVAL
    assert ms.ms_host_alloc(None, 4096)[0] == ms.MS_EINVAL
    assert ms.ms_host_free(None, None) == ms.MS_EINVAL
    assert ms.ms_probe_link(None, None, None, 16, 0) == ms.MS_EINVAL


def test_headers_compile_as_c(tmp_path):
    c = tmp_path / "t.c"
    incs = "".join('#include "%s"\n' % h for h in sorted(os.listdir(INCLUDE))
                   if h.endswith(".h"))
    # layout checks at compile time (a negative array size fails the build)
    c.write_text(incs +
                 'typedef char req_is_80[sizeof(ms_request) == 80 ? 1 : -1];\n'
                 'typedef char cfg_is_64[sizeof(ms_config) == 64 ? 1 : -1];\n'
                 'typedef char nonce_is_32[sizeof(ms_nonce) == 32 ? 1 : -1];\n'
                 'int main(void){ ms_config c; req_is_80 a; cfg_is_64 b;'
                 ' nonce_is_32 d; (void)a; (void)b; (void)d;'
                 ' ms_config_default(&c); return 0; }\n')
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror",
                           "-I", INCLUDE, "-c", str(c), "-o",
                           str(tmp_path / "t.o")])


def test_struct_layouts_match_binding():
    from paper_2004_09252_amd import memshield as ms
    import ctypes
    assert ctypes.sizeof(ms.ms_nonce) == 32
    assert ctypes.sizeof(ms.ms_request) == 80
    assert ctypes.sizeof(ms.ms_tuning) == 24
    assert ctypes.sizeof(ms.ms_config) == 64


@pytest.mark.parametrize("source,min_kernels", [("page_cipher.hip", 8),
                                                ("resident.hip", 6)])
def test_cipher_kernels_use_no_scratch(tmp_path, source, min_kernels):
    """Compile the kernels with resource-usage remarks: every kernel must
    report zero scratch bytes per lane (no register spill), so the key and
    the cipher state never reach per-lane memory (section 4.4)."""
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not present")
    r = subprocess.run(
        [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17",
         "--cuda-device-only", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", INCLUDE, "-I", CSRC,
         "-Rpass-analysis=kernel-resource-usage", "-c",
         os.path.join(CSRC, source), "-o", str(tmp_path / "k.o")],
        capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    names = re.findall(r"Function Name: (\S+)", r.stderr)
    scratch = [int(x) for x in
               re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    assert len(names) >= min_kernels and len(names) == len(scratch)
    bad = [n for n, s in zip(names, scratch) if s != 0]
    assert not bad, bad


def test_cipher_kernels_are_not_optimised_away(tmp_path):
    """Every cipher kernel instantiation must keep its rounds and its
    stores: a kernel the compiler reduced to an empty body would silently
    leave its output untouched."""
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not present")
    r = subprocess.run(
        [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17",
         "--cuda-device-only", "-S", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", INCLUDE, "-I", CSRC,
         os.path.join(CSRC, "page_cipher.hip"), "-o", str(tmp_path / "k.s")],
        capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    asm = open(tmp_path / "k.s").read()
    bodies = re.findall(
        r"^(_Z\S*(?:plain|batch)_pages_kernel\S*):(.*?)^\.Lfunc_end",
        asm, flags=re.S | re.M)
    assert len(bodies) >= 18
    for name, body in bodies:
        rounds = 20 if "ILi20E" in name else (12 if "ILi12E" in name else 8)
        assert body.count("v_alignbit_b32") >= 16 * rounds - 40, name
        assert body.count("global_store_dwordx4") >= 4, name


def test_requests_hold_their_tensors_until_reported_finished():
    """An asynchronous request's tensors stay referenced while it is in
    flight (the caching allocator must not reuse them under the kernel):
    `request` and `array_nonce` carry them, and the Engine's table keeps
    them per ticket until poll reports the ticket finished."""
    import gc
    import weakref

    import torch
    from paper_2004_09252_amd import memshield as ms
    src = torch.zeros(4096, dtype=torch.uint8)
    dst = torch.zeros(4096, dtype=torch.uint8)
    arr = torch.zeros(12, dtype=torch.uint8)
    refs = [weakref.ref(t) for t in (src, dst, arr)]
    r = ms.request(1, src, dst, 1, ms.array_nonce(arr))
    del src, dst, arr
    gc.collect()
    assert all(w() is not None for w in refs)
    pending = {}
    # ticket 0 is a dropped prefetch hint: nothing to hold
    ms._hold(pending, [0, 11], [(1,), getattr(r, "_keep")])
    del r
    gc.collect()
    assert list(pending) == [11] and all(w() is not None for w in refs)
    pending[12] = (2,)
    ms._release(pending, [11, 12], [0, 1])   # 11 still running
    assert list(pending) == [11]
    ms._release(pending, [11], [ms.MS_ECANCELED])
    gc.collect()
    assert not pending and all(w() is None for w in refs)
