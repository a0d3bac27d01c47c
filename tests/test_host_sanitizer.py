"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): builds _build/san/libccmi_san.so (host code instrumented, device
code as usual), links tests/host_abi_san.c against it with the same
compiler's sanitizer runtimes, and runs it: argument validation of every
entry point, workspace-bound arithmetic over the ABI's size range, and the
router file parser on good and malformed files."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no ROCm clang")
def test_host_code_under_asan_and_ubsan(tmp_path):
    from paper_1607_06156_amd import build as B
    lib = B.build_sanitized()
    exe = tmp_path / "host_abi_san"
    cmd = [CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host_abi_san.c"), lib, "-Wl,-rpath," + os.path.dirname(lib),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ)
    # the HIP runtime keeps allocations until exit; leaks are not what this checks
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    weights = os.path.join(ROOT, "paper_1607_06156_amd", "router_weights.txt")
    r = subprocess.run([str(exe), str(tmp_path), weights], capture_output=True, text=True, env=env,
                       timeout=120)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "host ABI checks passed" in r.stdout
