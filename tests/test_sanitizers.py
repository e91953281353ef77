"""Sanitizer runs of the CPU code (no GPU): the oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc) under its pin tests, and the library's host code (argument
validation, workspace arithmetic, the size recurrences) built with clang's sanitizers on the
host side only, under the ABI tests.  Each runs in a child process with the sanitizer runtime
preloaded; any report fails the run."""
import glob
import os
import subprocess
import sys

import pytest

pytestmark = [pytest.mark.cpu, pytest.mark.slow]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env_extra, args, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *args], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer"):
        assert marker not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan():
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    assert os.path.exists(asan), asan
    out = _run({"LD_PRELOAD": asan, "PHFEM_ORACLE_SANITIZE": "1"}, ["-m", "not gpu", "tests/test_oracle_pins.py"],
               timeout=900)
    assert " passed" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    from paper_2509_11133_amd import build as hb

    lib = str(tmp_path / "libphfem_san.so")
    # sanitizers on the host side only: every -fsanitize= follows -Xarch_host
    cmd = ["hipcc", *[f for f in hb.FLAGS if f != "-O3"], "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           *[os.path.join(hb.CSRC, s) for s in hb.SOURCES], "-o", lib]
    subprocess.check_call(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    out = _run({"LD_PRELOAD": rt[-1], "PHFEM_LIB": lib}, ["tests/test_abi.py", "-k", "not bench"], timeout=600)
    assert " passed" in out
