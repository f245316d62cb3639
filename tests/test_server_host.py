"""Host-side parts of the request server (no GPU): the admission size of a batch, and the
server's scheduling (paper_1811_06127_amd/csrc/server_core.hpp) driven by a host-only
executor whose lanes are threads and whose search is the CPU oracle
(tests/server_host/fake_server.cpp): FIFO admission by bytes and by a read cap, alone ==
mixed, hit-capacity retries, ring back-pressure, a failing search and the size limits, in
a plain build and under ThreadSanitizer."""
import os
import shutil
import subprocess

import pytest

from paper_1811_06127_amd import fm


def al(x):
    return (x + 255) // 256 * 256


def test_batch_bytes_rule():
    o = fm.server_opts(lanes=2, flags=fm.FM_BOTH | fm.FM_DARRAY, zmax=2, hit_reserve=4, arena_bytes=1 << 28)
    prev = 0
    for n, L in [(0, 0), (1, 50), (1000, 150_000), (20_000, 5_000_000)]:
        b = fm.fm_server_bytes(o, n, L)
        assert b % 256 == 0 and b > prev
        prev = b
        # inputs, outputs and the hit reserve are all inside
        floor = al(L) + al(8 * (n + 1)) + al(n) + al(4 * n) + al(8 * (n + 1)) + al(16 * 4 * n * 2)
        assert b >= floor + 256
    # more reads or more symbols never take less memory
    assert fm.fm_server_bytes(o, 10, 1000) <= fm.fm_server_bytes(o, 11, 1000)
    assert fm.fm_server_bytes(o, 10, 1000) <= fm.fm_server_bytes(o, 10, 1300)
    # one strand and no hit reserve take less
    o1 = fm.server_opts(lanes=2, flags=fm.FM_FWD, zmax=2, hit_reserve=0, arena_bytes=1 << 28)
    assert fm.fm_server_bytes(o1, 1000, 150_000) < fm.fm_server_bytes(o, 1000, 150_000)


@pytest.mark.parametrize("kw", [dict(lanes=0), dict(lanes=9), dict(zmax=5), dict(flags=0),
                                dict(flags=fm.FM_BOTH | fm.FM_PLAIN), dict(arena_bytes=1, lanes=2)])
def test_batch_bytes_rejects_bad_options(kw):
    with pytest.raises(fm.FmError) as e:
        fm.fm_server_bytes(fm.server_opts(**kw), 10, 1000)
    assert e.value.status == fm.FM_EINVAL


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "server_host", "fake_server.cpp")
ORACLE_C = os.path.join(ROOT, "oracle", "fm_oracle.c")
ROCM_CLANG = "/opt/rocm/llvm/bin"


def build_and_run(tmp_path, cc, cxx, extra, env=None):
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "fake_server")
    subprocess.run([cc, "-O1", "-g", *extra, "-c", ORACLE_C, "-o", obj], check=True)
    subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-pthread", *extra, "-I", os.path.join(ROOT, "include"),
                    "-o", exe, HARNESS, obj], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-3000:], r.stderr[-6000:])
    return r


def test_scheduler_with_host_executor(tmp_path):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("no gcc/g++")
    r = build_and_run(tmp_path, "gcc", "g++", ["-Wall", "-Wextra"])
    assert r.returncode == 0 and "ok: 0 failed checks" in r.stdout


def test_scheduler_under_thread_sanitizer(tmp_path):
    """The same scenarios with every access of the scheduler, the lanes and the oracle
    instrumented: ThreadSanitizer reports no data race or lock misuse. (The LLVM runtime
    is used: it intercepts pthread_cond_clockwait, through which libstdc++ implements
    timed waits; GCC 11's does not, and reports such waits as double locks.)"""
    cc, cxx = os.path.join(ROCM_CLANG, "clang"), os.path.join(ROCM_CLANG, "clang++")
    if not (os.path.exists(cc) and os.path.exists(cxx)):
        pytest.skip("no LLVM clang with a ThreadSanitizer runtime")
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66 second_deadlock_stack=1")
    r = build_and_run(tmp_path, cc, cxx, ["-fsanitize=thread"], env=env)
    assert r.returncode == 0 and "ok: 0 failed checks" in r.stdout
    assert "ThreadSanitizer" not in r.stderr
