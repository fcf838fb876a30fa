"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Opt-in (SOAP_SANITIZE=1; it rebuilds both libraries, about a minute):
  * the library is rebuilt with -fsanitize=address,undefined on its host
    code (C ABI validation, FP64 table build, direct radial integrals)
    and tests/test_host_library.py runs against it, with clang's ASan
    runtime preloaded into the interpreter;
  * the oracle is compiled with gcc -fsanitize=address,undefined and the
    oracle pins run against it, with gcc's runtimes preloaded.
A sanitizer report, or any failing test, fails this test.  Device code is
built as usual, without sanitizers.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2101_08814_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.skipif(os.environ.get("SOAP_SANITIZE") != "1",
                                reason="opt-in: set SOAP_SANITIZE=1 (rebuilds the libraries with sanitizers)")

SAN_OPTIONS = "detect_leaks=0:detect_odr_violation=0:alloc_dealloc_mismatch=0:halt_on_error=1"
UBSAN_OPTIONS = "print_stacktrace=1:halt_on_error=1"


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def _sanitized_library(out_dir):
    sys.path.insert(0, ROOT)
    from paper_2101_08814_amd import build_lib
    import concurrent.futures

    def compile_one(src):
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + (["-x", "hip"] if src.endswith(".hip") else []) + [
            "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fsanitize=address,undefined",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        _run(cmd)
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, build_lib.SOURCES))
    lib = os.path.join(out_dir, "libsoap_mi355x_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan", "-Xarch_host",
          "-fsanitize=address,undefined", "-o", lib] + objs)
    rt = _run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"]).stdout.strip()
    assert os.path.isabs(rt) and os.path.exists(rt), rt
    return lib, rt


def _check(r):
    text = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in text and "runtime error:" not in text, text[-6000:]
    assert r.returncode == 0, text[-6000:]


def test_library_host_code_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        lib, rt = _sanitized_library(d)
        env = dict(os.environ, SOAP_MI355X_LIBRARY=lib, LD_PRELOAD=rt, ASAN_OPTIONS=SAN_OPTIONS,
                   UBSAN_OPTIONS=UBSAN_OPTIONS, SOAP_SANITIZE="0")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-v", "-s", "-p", "no:cacheprovider", "-m", "not gpu",
                            os.path.join(ROOT, "tests", "test_host_library.py")],
                           capture_output=True, text=True, env=env, cwd=ROOT)
        print(r.stdout[-2000:])
        _check(r)


def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        sys.path.insert(0, ROOT)
        import oracle
        lib = os.path.join(d, "libsoap_oracle_san.so")
        _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fopenmp", "-fPIC",
              "-shared", "-std=c11", "-o", lib, oracle._SRC, "-lm"])
        rts = [_run(["gcc", f"-print-file-name={n}"]).stdout.strip() for n in ("libasan.so", "libubsan.so")]
        env = dict(os.environ, SOAP_ORACLE_LIBRARY=lib, LD_PRELOAD=":".join(rts), ASAN_OPTIONS=SAN_OPTIONS,
                   UBSAN_OPTIONS=UBSAN_OPTIONS, SOAP_SANITIZE="0", OMP_NUM_THREADS="4")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-v", "-s", "-p", "no:cacheprovider", "-m", "not gpu",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                            os.path.join(ROOT, "tests", "test_compression_pins.py")],
                           capture_output=True, text=True, env=env, cwd=ROOT)
        print(r.stdout[-2000:])
        _check(r)
