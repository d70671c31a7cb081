"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The oracle: ``oracle.c`` is rebuilt with ``-fsanitize=address,undefined``
  and the oracle's pin tests run against that build in a child process that
  preloads gcc's sanitizer runtimes; any report aborts the child.
* The C ABI: the library is rebuilt with the sanitizers on its host code
  only (device code is never instrumented), linked into a small driver
  that calls every entry point with arguments the host code must reject,
  and run; it needs no GPU because every call returns before its first HIP
  call.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_00585_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.slow


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_address_and_ub_sanitizers():
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    env = dict(os.environ)
    env.update({
        "FEASM_ORACLE_SANITIZE": "1",
        "LD_PRELOAD": f"{asan}:{ubsan}",
        # the interpreter itself keeps memory until exit: leaks are not the question
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    probe = subprocess.run(
        [sys.executable, "-c",
         "from oracle import oracle; oracle.build(force=True); oracle.lib(); print(oracle._LIB)"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-3000:]
    lib = probe.stdout.strip().splitlines()[-1]
    assert lib.endswith("liboracle_san.so"), lib
    ldd = subprocess.run(["ldd", lib], capture_output=True, text=True).stdout
    assert "libasan" in ldd and "libubsan" in ldd, ldd
    tests = [os.path.join(ROOT, "tests", t) for t in
             ("test_oracle_pins.py", "test_oracle_spmv.py", "test_oracle_hex8.py",
              "test_oracle_random.py")]
    run = subprocess.run(
        [sys.executable, "-m", "pytest", "-p", "no:cacheprovider", "-x", "-q", "--rootdir", ROOT,
         *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert run.returncode == 0, (run.stdout[-3000:], run.stderr[-3000:])
    assert " passed" in run.stdout


def test_abi_host_code_under_address_and_ub_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("ROCm compilers not installed")
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    # sanitizers on the host code only (never on device code)
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all"]

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        r = subprocess.run([HIPCC, *flags, *inc, "-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
        objs = list(pool.map(compile_one, srcs))
    exe = str(tmp_path / "abi_check")
    r = subprocess.run([CLANGXX, "-std=c++17", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I",
                        "/opt/rocm/include", *inc, os.path.join(ROOT, "tests", "sanitize",
                                                                "abi_check.cpp"),
                        *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, (run.stdout[-3000:], run.stderr[-3000:])
    assert "abi ok" in run.stdout
