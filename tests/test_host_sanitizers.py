"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's host sources (argument checks, plan construction: tau-weight tables, FFT
plans, filter responses, work lists, size classes, the tuner's bookkeeping) are rebuilt
with both sanitizers on their host pass only and linked, with the unchanged device
objects of the library build, into `host_checks` (tests/host_checks.cpp), which drives
every entry point's argument checks and plans many 2D Haar, general-wavelet and volume
configurations.  Without a GPU each valid plan runs all of its host work and stops at
its first device upload.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1911_01234_amd import build as B  # noqa: E402
from paper_1911_01234_amd import filters  # noqa: E402

HOST_SOURCES = [s for s in B.SOURCES if s.endswith(".cpp")]
# the driver is plain C++, built by the same clang as the library so that one sanitizer
# runtime serves both
CLANGXX = os.path.join(os.path.dirname(os.path.realpath(B.HIPCC)), "..", "lib", "llvm", "bin", "clang++")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _device_objects():
    objs = [os.path.join(B.OBJ_DIR, s + ".o") for s in B.SOURCES if not s.endswith(".cpp")]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    return objs


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    dev = _device_objects()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", B.CSRC]
    base = [B.HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
            "-Wno-unused-result"]
    jobs = [(base + SAN + inc + ["-c", os.path.join(B.CSRC, s), "-o", str(tmp_path / (s + ".o"))])
            for s in HOST_SOURCES]
    jobs.append([CLANGXX, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                 "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                 "-c", os.path.join(ROOT, "tests", "host_checks.cpp"), "-o", str(tmp_path / "host_checks.o")])
    with ThreadPoolExecutor(4) as ex:
        res = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), jobs))
    for c, r in zip(jobs, res):
        assert r.returncode == 0, (" ".join(c), r.stderr[-3000:])
    exe = str(tmp_path / "host_checks")
    link = [B.HIPCC, "--offload-arch=gfx950", *SAN, "-o", exe, str(tmp_path / "host_checks.o"),
            *[str(tmp_path / (s + ".o")) for s in HOST_SOURCES], *dev]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]

    flt = tmp_path / "filters.txt"
    with open(flt, "w") as f:
        for n in (1, 2, 3, 4, 6, 8):
            f.write(" ".join(repr(float(v)) for v in filters.daubechies(n)) + "\n")
    env = dict(os.environ)
    # the HIP runtime's own allocations at exit are not the library's leaks
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe, str(flt)], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    print(r.stdout)
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "0 failures" in r.stdout, out[-4000:]
