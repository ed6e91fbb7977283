"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
seeded generator, the host setup of the network arrays and the oracle, built
with gcc/g++ -fsanitize=address,undefined into a small driver
(tests/native/sanitize_driver.cpp) that runs every topology, both weight
types, the setup's error paths and the oracle in both raster modes on small
networks.  Any out-of-bounds access, leak or undefined operation aborts the
driver with a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _have_sanitizers(tmp):
    src = os.path.join(tmp, "probe.c")
    with open(src, "w") as fh:
        fh.write("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", *SAN, src, "-o", os.path.join(tmp, "probe")],
                       capture_output=True)
    return r.returncode == 0


def test_host_code_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("gcc/g++ not found")
    tmp = str(tmp_path)
    if not _have_sanitizers(tmp):
        pytest.skip("this gcc has no ASan/UBSan runtime")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "synth"),
           "-I", os.path.join(ROOT, "oracle")]
    steps = [
        ["gcc", *SAN, "-std=c11", "-fopenmp", "-c", os.path.join(ROOT, "synth", "synth.c"),
         "-o", "synth.o"],
        ["gcc", *SAN, "-std=c11", "-ffp-contract=off", "-c",
         os.path.join(ROOT, "oracle", "oracle.c"), "-o", "oracle.o"],
        ["g++", *SAN, "-std=c++17", "-fopenmp", *inc, "-c",
         os.path.join(ROOT, "paper_2205_07125_amd", "csrc", "snn_setup.cpp"), "-o", "setup.o"],
        ["g++", *SAN, "-std=c++17", *inc, "-c",
         os.path.join(ROOT, "tests", "native", "sanitize_driver.cpp"), "-o", "drv.o"],
        ["g++", *SAN, "-fopenmp", "drv.o", "setup.o", "synth.o", "oracle.o", "-lm", "-o", "drv"],
    ]
    for cmd in steps:
        subprocess.run(cmd, cwd=tmp, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([os.path.join(tmp, "drv")], cwd=tmp, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitize ok" in r.stdout
    assert "runtime error" not in r.stderr
