"""The CPU oracle and the host side of the C-ABI library under
AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU needed).

The oracle is compiled with gcc together with a driver that calls every
exported oracle function on small random and ragged inputs; the library's
host code (validation, size queries, batch / serving / no-alloc refusal
paths) is compiled with the sanitizers on its host pass only and linked with
a driver that exercises those paths with no device present.  Both drivers
exit 0 only when every call returned its documented status, and any
sanitizer report aborts them."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(ROOT, "_build", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"


def run(cmd, env=None, timeout=600):
    res = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return res.returncode, res.stdout + res.stderr


def test_oracle_under_asan_ubsan():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    rc, log = run(["gcc", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
                   "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                   "-o", exe, os.path.join(SAN, "oracle_driver.c"),
                   os.path.join(ROOT, "oracle", "styleblit_oracle.c")])
    assert rc == 0, log
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    rc, log = run([exe], env=env)
    assert rc == 0 and "0 failures" in log, log
    assert "ERROR: AddressSanitizer" not in log and "runtime error" not in log, log


HOST_SOURCES = ["capi", "batch", "serve", "noalloc", "style", "change", "jitter", "search"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="the ROCm compilers are not installed")
def test_host_library_under_asan_ubsan():
    from paper_1807_03249_amd import build as b

    # the device-heavy sources link from the ordinary build's objects
    objs = [os.path.join(b.OBJ_DIR, f + ".hip.o") for f in ("stylize", "lut")]
    if not all(os.path.exists(o) for o in objs):
        b.build()
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1807_03249_amd", "csrc")]
    flags = [
        "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # host pass only: the device code stays unsanitized
        "-Xarch_host", "-fsanitize=address",
        "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-sanitize-recover=all",
        "-Xarch_host", "-fno-omit-frame-pointer",
    ]

    def compile_one(name):
        src = os.path.join(ROOT, "paper_1807_03249_amd", "csrc", name + ".hip")
        obj = os.path.join(OUT, name + ".o")
        return run([HIPCC, *flags, *inc, "-c", src, "-o", obj]), obj

    with ThreadPoolExecutor(min(len(HOST_SOURCES), os.cpu_count() or 4)) as ex:
        done = list(ex.map(compile_one, HOST_SOURCES))
    for (rc, log), obj in done:
        assert rc == 0, log
    drv = os.path.join(OUT, "host_driver.o")
    rc, log = run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                   "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", *inc,
                   "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-c",
                   os.path.join(SAN, "host_driver.cpp"), "-o", drv])
    assert rc == 0, log
    exe = os.path.join(OUT, "host_driver")
    rc, log = run([CLANG, "-fsanitize=address,undefined", "-o", exe, drv,
                   *[o for _, o in done], *objs, "-L/opt/rocm/lib", "-lamdhip64",
                   "-Wl,-rpath,/opt/rocm/lib"])
    assert rc == 0, log
    # the HIP runtime's own allocations at exit are not the library's
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    rc, log = run([exe], env=env)
    assert rc == 0 and "0 failures" in log, log
    assert "ERROR: AddressSanitizer" not in log and "runtime error" not in log, log
