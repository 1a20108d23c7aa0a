"""The runtime's host paths under AddressSanitizer, UndefinedBehaviorSanitizer and LeakSanitizer.

runtime.cpp is compiled for the host with the sanitizers (hipcc, each -fsanitize= behind
-Xarch_host, so no device code is instrumented) and linked with the library's kernel object and
tests/host_sanitize.cpp, which drives the partition, the sweep levels, theta, the request byte
count and their error paths (no GPU call).  Leaks inside the HIP runtime's own start-up are
suppressed; any report from the runtime's code fails the test.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
KOBJ = os.path.join(ROOT, "paper_2006_14602_amd", "_build", "kernels.hip.o")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    return r.returncode, r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_paths_clean_under_sanitizers(tmp_path):
    if not os.path.exists(KOBJ):
        pytest.skip("the library's kernel object is not built (run the package build first)")
    rt = str(tmp_path / "runtime_san.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "host_sanitize")
    rc, out = run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-w"] + SAN +
                  ["-c", os.path.join(ROOT, "paper_2006_14602_amd", "csrc", "runtime.cpp"), "-o", rt])
    assert rc == 0, out
    rc, out = run([HIPCC, "-O1", "-g", "-std=c++17", "-w", "-I", os.path.join(ROOT, "include")] + SAN +
                  ["-c", os.path.join(ROOT, "tests", "host_sanitize.cpp"), "-o", drv])
    assert rc == 0, out
    rc, out = run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                   "-fsanitize=undefined", drv, rt, KOBJ, "-lpthread", "-o", exe])
    assert rc == 0, out
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               LSAN_OPTIONS=f"suppressions={supp}", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    rc, out = run([exe], env=env, timeout=120)
    assert rc == 0 and "host-sanitize ok" in out, out
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out, out
