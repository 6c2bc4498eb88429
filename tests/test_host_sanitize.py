"""The library's host code (dark-node decomposition, argument checks, path
decision, net-block packing) run under AddressSanitizer and
UndefinedBehaviorSanitizer on the CPU: the library's sources are compiled
with the sanitizers on the host side only (device code is built as usual)
and linked into a host program that exercises them with random and
malformed inputs.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1312_4587_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_sanitize")


def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_1312_4587_amd import build
    srcs = [os.path.join(CSRC, f) for f in build.SOURCES]
    exe = str(tmp_path / "abi_host_check")
    san = []
    for opt in ("-fsanitize=address", "-fsanitize=undefined",
                "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", opt]
    cmd = [hipcc, "-O1", "-g", "-std=c++17", f"--offload-arch={build.ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", *san,
           *srcs, os.path.join(HERE, "abi_host_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "OK" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
