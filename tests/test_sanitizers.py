"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the CPU oracle (tests/sanitize/check_oracle.c linked with oracle/oracle.cpp),
the library's host-side logic (tests/sanitize/check_abi_host.cpp built with
the library's source, sanitizers on the host side only), and the tile-owner
index logic the count kernel runs, checked on the host against brute force
(tests/sanitize/check_tile_owners.cpp).  Each program exits 0
when its checks pass and the sanitizers report nothing."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(SAN, "_build")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout + r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_oracle_under_asan_ubsan():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "check_oracle")
    objc = os.path.join(OUT, "check_oracle.o")
    flags = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off"]
    subprocess.check_call(["gcc", *flags, "-c", os.path.join(SAN, "check_oracle.c"), "-o", objc])
    subprocess.check_call(["g++", *flags, "-std=c++17", objc, os.path.join(ROOT, "oracle", "oracle.cpp"), "-o", exe])
    _run(exe)


HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="no hipcc")
def test_library_host_code_under_asan_ubsan():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "check_abi_host")
    src = os.path.join(ROOT, "paper_2403_10647_amd", "csrc", "gridbuild.hip")
    # the device code is built as usual; the sanitizers apply to the host side only
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           f"-I{os.path.join(ROOT, 'include')}", src, os.path.join(SAN, "check_abi_host.cpp"), "-o", exe]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    _run(exe)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="no hipcc")
def test_tile_owner_index_logic_on_the_host():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "check_tile_owners")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           f"-I{os.path.join(ROOT, 'paper_2403_10647_amd', 'csrc')}", os.path.join(SAN, "check_tile_owners.cpp"), "-o", exe]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    _run(exe)
