"""The host-side logic of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer: the
host ABI tests (test_abi_host.py: argument validation, constraint bookkeeping, sizing, network
shapes) run in a child process against libfftc_hostsan.so, the same sources built with the
sanitizers on the host code only, with the ASan runtime preloaded.  Any report fails the test
(halt_on_error; UBSan without recovery).  No GPU is used."""
import os
import subprocess
import sys

import pytest

import paper_2607_26082_amd.build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    r = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_host_abi_under_sanitizers():
    if not os.path.exists(B.SAN_OUT):
        pytest.skip("libfftc_hostsan.so not built (paper_2607_26082_amd/build.py --hostsan)")
    srcs = [os.path.join(B.HERE, "csrc", f) for f in os.listdir(os.path.join(B.HERE, "csrc"))]
    if max(os.path.getmtime(f) for f in srcs) > os.path.getmtime(B.SAN_OUT):
        pytest.skip("libfftc_hostsan.so is older than its sources (build.py --hostsan -i rebuilds it)")
    rt = _runtime()
    if rt is None:
        pytest.skip("ASan runtime of the ROCm clang not found")
    nm = subprocess.run(["nm", "-D", "--undefined-only", B.SAN_OUT], capture_output=True, text=True)
    assert "__asan_report_load8" in nm.stdout and "__ubsan_handle" in nm.stdout   # instrumented
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, FFTC_LIB=B.SAN_OUT, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_abi_host.py"), "-m", "not gpu"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
