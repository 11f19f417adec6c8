"""The host C++ of the C ABI (coeffs.cpp, api.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

tests/sanitize/host_paths.cpp drives the host-side paths: the coefficient
solves for N = 2..8, configuration planning and validation of every lattice,
precision and storage form, the invalid-input and cleanup paths of creation
and of batches, and NULL handles.  The two host sources are compiled with the
ROCm clang++ as plain host C++ (no device code on that line) with
-fsanitize=address,undefined and linked against the device objects that the
library build leaves in _build/ (not instrumented; their host stubs only
launch kernels).  Without a GPU, creation takes its device-error path.  Any
sanitizer report aborts the driver, so the test passes only on a clean run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_22214_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
CLANG = "/opt/rocm/llvm/bin/clang++"


def _device_objects():
    from paper_2605_22214_amd import build
    objs = [u[1] for u in build.UNITS if u[2]]
    if not all(os.path.exists(os.path.join(BUILD, o)) for o in objs):
        build.build(verbose=False)
    return [os.path.join(BUILD, o) for o in objs]


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not installed")
def test_host_paths_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_paths")
    cmd = [CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           os.path.join(CSRC, "coeffs.cpp"), os.path.join(CSRC, "api.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "host_paths.cpp")] + _device_objects() + \
          ["-o", exe, "-L/opt/rocm/lib", "-lamdhip64", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    report = run.stdout[-4000:] + run.stderr[-4000:]
    assert run.returncode == 0, report
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, report
    assert "all checks passed" in run.stdout
