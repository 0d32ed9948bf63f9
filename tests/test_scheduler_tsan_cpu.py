"""CPU tests of the library's host logic under ThreadSanitizer, built with g++
against mock HIP and HSA runtimes (tests/mock_hip: streams as threads,
kernels ciphering through the C oracle, and a CPU model of the resident-key
kernel's protocol behind a mock HSA queue).  The library's sources are
compiled unchanged.

* The serving path (paper_2004_09252_amd/csrc/engine.cpp: admission, queues,
  tickets, continuous batching, cancellation, prefetch hints, the scheduler
  thread) with 8 submitting threads, a cancelling thread, the scheduler and
  the stream threads.  The driver (tests/mock_hip/sched_stress.cpp) checks
  that every result is the same alone and in the mix and equals the oracle.
* The resident-key engine's host side (resident.cpp with host_pages.cpp:
  start, the key table, multi-producer submission with slot reuse on a
  small ring, polling, the idle exit, stop, shutdown) with 6 producers and
  the model's poller and 23 workers.  The driver
  (tests/mock_hip/resident_stress.cpp) checks every result against the
  oracle.

ThreadSanitizer must report nothing."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MOCK = os.path.join(ROOT, "tests", "mock_hip")
CSRC = os.path.join(ROOT, "paper_2004_09252_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
ORACLE_C = os.path.join(ROOT, "oracle", "chacha20_oracle.c")

COMMON = [os.path.join(CSRC, "engine.cpp"),
          os.path.join(CSRC, "tune_cache.cpp"),
          os.path.join(MOCK, "mock_hip.cpp"),
          os.path.join(MOCK, "mock_kernels.cpp")]
SCHED_SOURCES = COMMON + [os.path.join(MOCK, "sched_stress.cpp")]
RING_SOURCES = COMMON + [os.path.join(CSRC, "host_pages.cpp"),
                         os.path.join(CSRC, "resident.cpp"),
                         os.path.join(MOCK, "mock_hsa.cpp"),
                         os.path.join(MOCK, "sched_stress.cpp")]
KEY_RACE_SOURCES = COMMON + [os.path.join(CSRC, "host_pages.cpp"),
                             os.path.join(MOCK, "key_race.cpp")]
RESIDENT_SOURCES = COMMON + [os.path.join(CSRC, "host_pages.cpp"),
                             os.path.join(CSRC, "resident.cpp"),
                             os.path.join(MOCK, "mock_hsa.cpp"),
                             os.path.join(MOCK, "resident_stress.cpp")]


def _tsan_available(tmp_path):
    if not shutil.which("g++") or not shutil.which("gcc"):
        return False
    probe = tmp_path / "probe.cpp"
    probe.write_text("int main() { return 0; }\n")
    r = subprocess.run(["g++", "-fsanitize=thread", str(probe), "-o",
                        str(tmp_path / "probe")], capture_output=True)
    return r.returncode == 0


def _build(tmp_path, sources, name, defines=()):
    cxx = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread",
           "-include", os.path.join(MOCK, "tsan_prelude.h"),
           "-I", MOCK, "-I", INCLUDE, "-I", CSRC] + \
        ["-D" + d for d in defines]
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in sources]
    jobs = [cxx + ["-c", s, "-o", o] for s, o in zip(sources, objs)]
    jobs.append(["gcc", "-std=c99", "-O2", "-g", "-fsanitize=thread", "-c",
                 ORACLE_C, "-o", str(tmp_path / "oracle.o")])
    with ThreadPoolExecutor(max_workers=6) as ex:
        results = list(ex.map(
            lambda cmd: subprocess.run(cmd, capture_output=True, text=True),
            jobs))
    for cmd, r in zip(jobs, results):
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr
    exe = tmp_path / name
    r = subprocess.run(["g++", "-fsanitize=thread"] + objs +
                       [str(tmp_path / "oracle.o"), "-o", str(exe),
                        "-lpthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run_clean(exe, **extra_env):
    env = dict(os.environ, TSAN_OPTIONS="second_deadlock_stack=1",
               **extra_env)
    r = subprocess.run([str(exe)], capture_output=True, text=True,
                       timeout=600, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert r.stdout.startswith("ok "), r.stdout
    return r.stdout


def test_serving_host_logic_under_thread_sanitizer(tmp_path):
    if not _tsan_available(tmp_path):
        pytest.skip("g++ with ThreadSanitizer not available")
    _run_clean(_build(tmp_path, SCHED_SOURCES, "sched_stress"))


def test_ring_serving_stage_host_logic_under_thread_sanitizer(tmp_path):
    """The same serving driver with the ring stage (ms_submit publishing
    one descriptor per page into the resident kernel's ring, which reads
    each descriptor's key from the context's key table): alone == mix ==
    oracle, with hints and cancellation beside it, on a mock device of 8
    compute units (31 ring workers, each a host thread)."""
    if not _tsan_available(tmp_path):
        pytest.skip("g++ with ThreadSanitizer not available")
    exe = _build(tmp_path, RING_SOURCES, "ring_stress",
                 defines=("RING_STAGE",))
    _run_clean(exe, MOCK_HIP_CUS="8")


def test_resident_engine_host_logic_under_thread_sanitizer(tmp_path):
    if not _tsan_available(tmp_path):
        pytest.skip("g++ with ThreadSanitizer not available")
    out = _run_clean(_build(tmp_path, RESIDENT_SOURCES, "resident_stress"))
    # the small ring must have filled: producers met MS_EAGAIN
    retries = int(out.split("eagain_retries=")[1].split()[0])
    assert retries > 0, out


def test_key_destroy_racing_synchronous_calls(tmp_path):
    """ms_key_destroy + reload of the same key-table row against
    synchronous calls (plain, fused batch, host pages) that keep using the
    destroyed key's newest handle: every call that succeeds must have
    ciphered with that key, and ThreadSanitizer must report nothing."""
    if not _tsan_available(tmp_path):
        pytest.skip("g++ with ThreadSanitizer not available")
    out = _run_clean(_build(tmp_path, KEY_RACE_SOURCES, "key_race"))
    cycles = int(out.split("cycles=")[1].split()[0])
    assert cycles > 0, out
