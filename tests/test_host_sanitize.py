"""Host sanitizer tier: the library's host driver (planner, validation, work
split, aux batching, q chunking, batch planner, every C-ABI entry point and
its error paths) built for the CPU with AddressSanitizer and
UndefinedBehaviorSanitizer, linked against a host stand-in of the HIP runtime
with no-op kernel launchers (tests/host_sanitize/hip_host_stub.cpp), and
driven on the tiny, C1 and C2 inputs by tests/host_sanitize/drive.py.  Any
sanitizer report aborts the driver, which fails the test.  No GPU is used."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
CSRC = os.path.join(ROOT, "paper_2102_02989_amd", "csrc")


def _runtime(name):
    cxx = shutil.which("g++")
    if not cxx:
        return None
    p = subprocess.run([cxx, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    if not _runtime("libasan.so") or not os.path.isdir("/opt/rocm/include/hip"):
        pytest.skip("g++ with libasan and the HIP headers are needed for the host sanitizer build")
    from paper_2102_02989_amd.build import source_hash
    out = str(tmp_path_factory.mktemp("hostsan") / "librsgdf_hostsan.so")
    # built from the tree's capi.cpp, so it carries the tree's source hash
    # (the binding checks it on load)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
           f'-DRSGDF_SOURCE_HASH="{source_hash()}"',
           "-I/opt/rocm/include",
           # the two HIP-compiler spellings the host driver uses, for a plain C++ compiler
           "-D__align__(n)=__attribute__((aligned(n)))", "-DHIP_SYMBOL(x)=x",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fPIC", "-shared",
           "-Wl,-Bsymbolic", "-o", out, os.path.join(CSRC, "capi.cpp"), os.path.join(HERE, "hip_host_stub.cpp"),
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def test_host_driver_under_asan_ubsan(sanitized_lib):
    env = dict(os.environ)
    env["LD_PRELOAD"] = _runtime("libasan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, os.path.join(HERE, "drive.py"), sanitized_lib], capture_output=True,
                       text=True, env=env, timeout=1200)
    log = r.stdout + r.stderr
    assert r.returncode == 0, log[-6000:]
    assert "ERROR: AddressSanitizer" not in log and "runtime error:" not in log, log[-6000:]
    assert log.rstrip().endswith("done"), log[-3000:]
    # every input was planned and built, the batch ran twice, each malformed input was refused
    for case in ("case tiny 2x1x1", "case tiny 1x2x2", "case C1", "case C2", "batch run rc 0",
                 "case release cache rc 0", "case error paths"):
        assert case in log, case
    assert log.count("error path ") == 16
