"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* The oracle (plain C) is built with gcc's sanitizers together with a driver
  (`tests/sanitize/oracle_exercise.c`) that runs every entry point on inputs
  that reach its edge cases; any report aborts the run.
* The host part of liboctax (`octax_host.cpp`, `octax_pool.cpp`: config
  validation, tables, error paths) is built with the sanitizers on the host
  side only (`-Xarch_host`; the device code is the library's own), and the
  C-ABI tests that run without a GPU (`tests/test_abi_cpu.py`) run against it
  in a child process with the sanitizer runtime loaded first.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_01764_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def test_oracle_under_asan_and_ubsan():
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_exercise")
        subprocess.run(["gcc", "-std=c99", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", "-pthread", os.path.join(ROOT, "oracle", "chip8_oracle.c"),
                        os.path.join(ROOT, "tests", "sanitize", "oracle_exercise.c"), "-o", exe],
                       check=True, capture_output=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env={**os.environ, **SAN_ENV})
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "oracle exercised: 12 cases" in r.stdout


def _hip_objects(d):
    """Device sources compiled as the library builds them (reused from the
    build folder when they are newer than every source and header)."""
    from paper_2510_01764_amd import build as B
    srcs = [s for s in B.SOURCES if s.endswith(".hip")]
    newest = max(os.path.getmtime(os.path.join(CSRC, f)) for f in os.listdir(CSRC))
    newest = max(newest, max(os.path.getmtime(os.path.join(ROOT, "include", f))
                             for f in os.listdir(os.path.join(ROOT, "include"))))
    objs = []
    for s in srcs:
        o = os.path.join(B.BUILD_DIR, s + ".o")
        if not (os.path.exists(o) and os.path.getmtime(o) >= newest):
            o = os.path.join(d, s + ".o")
            subprocess.run([HIPCC] + B.FLAGS + ["-c", os.path.join(CSRC, s), "-o", o], check=True,
                           capture_output=True)
        objs.append(o)
    return objs


def test_host_library_under_asan_and_ubsan():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc not available")
    rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("clang's ASan runtime not available")
    from paper_2510_01764_amd import build as B
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for s in ("octax_host.cpp", "octax_pool.cpp"):
            o = os.path.join(d, s + ".o")
            flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"]
            subprocess.run([HIPCC] + flags + san + ["-x", "hip", "-c", os.path.join(CSRC, s), "-o", o],
                           check=True, capture_output=True)
            objs.append(o)
        objs += _hip_objects(d)
        lib = os.path.join(d, "liboctax.so")
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan"] + san +
                       ["-o", lib] + objs, check=True, capture_output=True)
        code = ("import sys; sys.path.insert(0, %r)\n"
                "import paper_2510_01764_amd.octax as X\n"
                "X.LIB_PATH = %r\n"
                "import pytest\n"
                "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', %r]))\n"
                % (ROOT, lib, os.path.join(ROOT, "tests", "test_abi_cpu.py")))
        env = {**os.environ, **SAN_ENV, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1"}
        # the sanitizer runtime must come first among the preloaded libraries
        env["LD_PRELOAD"] = rt + (":" + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600, env=env,
                           cwd=ROOT)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-4000:]
        assert " passed" in r.stdout
