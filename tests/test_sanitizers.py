"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle (oracle/oracle.c) and the library's host-side code that runs
without a device (the BVH builder, the dense symmetric eigensolvers of the
eigen step) are compiled with gcc/g++ -fsanitize=address,undefined and
driven on small inputs by tests/sanitize/*; any report aborts the test program.
The library's C ABI itself (capi.cpp) needs a device for nearly every call
and is not covered here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env)
    return r.returncode, r.stdout + r.stderr


@pytest.fixture(scope="module")
def outdir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("sanitize"))


def test_oracle_under_sanitizers(outdir):
    exe = os.path.join(outdir, "oracle_driver")
    rc, out = _run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp", *SAN, "-o", exe,
                    os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
                    "-lm"])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    rc, out = _run([exe], env)
    print(out)
    assert rc == 0 and "ok" in out, out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_sanitizers(outdir):
    exe = os.path.join(outdir, "host_driver")
    csrc = os.path.join(ROOT, "paper_2606_05581_amd", "csrc")
    rc, out = _run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *SAN, "-pthread", "-o", exe,
                    os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), os.path.join(csrc, "bvh_build.cpp"),
                    os.path.join(csrc, "symeig_host.cpp")])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env)
    print(out)
    assert rc == 0 and "ok" in out, out
