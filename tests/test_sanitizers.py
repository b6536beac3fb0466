"""AddressSanitizer and UBSan builds of the CPU oracle and of the library's
host runtime (CPU only).  Each is linked into a small driver of its own
(tests/sanitize/), so the sanitizer runtimes come in with the executable;
the HIP library build adds them to the host code only (-Xarch_host before
each -fsanitize=; the device code is built as usual), and the driver calls
only what runs without a GPU (validation, footprint, tile plans, argument
checks)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_asan"
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-std=c11",
                    "-D_DEFAULT_SOURCE", os.path.join(ROOT, "oracle", "rti_oracle.c"),
                    os.path.join(HERE, "oracle_main.c"), "-o", str(exe), "-lm"], check=True)
    r = subprocess.run([str(exe)], env=ENV, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "oracle ok" in r.stdout, r.stderr[-3000:]


@pytest.mark.slow
def test_host_runtime_under_asan_and_ubsan(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not found")
    exe = tmp_path / "host_asan"
    csrc = os.path.join(ROOT, "paper_2408_07609_amd", "csrc")
    srcs = [os.path.join(csrc, n) for n in ("rti_kernels.hip", "rti_fused.hip", "rti_host.cpp", "rti_batch.cpp")]
    cmd = ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-x", "hip", *srcs,
           "-x", "c++", os.path.join(HERE, "host_main.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=1200)
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0")     # the HIP runtime's static state is not the library's
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "host runtime ok" in r.stdout, (r.stdout + r.stderr)[-3000:]
