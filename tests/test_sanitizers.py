"""Host-code sanitizer runs (CPU only, slow): the oracle built with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer runs every oracle pin, and
libgce.so with its host code built the same way (clang, through hipcc's
-Xarch_host; device code untouched) runs the C-ABI and merge tests.  A
planted heap overflow in a throwaway library checks that each harness does
report errors."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle
from paper_2006_06866_amd import build as gbuild

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer"]
# host-only sanitizer flags for hipcc: each -fsanitize= after -Xarch_host
HIP_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
UBSAN_OPTIONS = "halt_on_error=1:print_stacktrace=1"

_PLANTED = r"""
#include <stdlib.h>
int planted_overflow(int n) {
    int *a = (int *)malloc(4 * sizeof(int));
    a[n] = 1;          /* n = 4: one past the end */
    int v = a[0];
    free(a);
    return v;
}
"""


def _gcc_asan():
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()


def _clang_asan():
    base = "/opt/rocm/llvm/lib/clang"
    for ver in sorted(os.listdir(base)):
        p = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    pytest.skip("clang ASan runtime not found")


def _run_pytest(files, env_extra):
    env = dict(os.environ, **env_extra)
    env["PYTHONDONTWRITEBYTECODE"] = "1"
    return subprocess.run([sys.executable, "-m", "pytest", *files, "-q", "-x",
                           "-p", "no:cacheprovider", "-m", "not gpu and not slow"],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


def _planted_reported(compiler, flags, runtime, tmp):
    """Build a library with a heap overflow under `flags` and call it with
    `runtime` preloaded: the sanitizer must abort the process."""
    src = os.path.join(tmp, "planted.c")
    with open(src, "w") as f:
        f.write(_PLANTED)
    lib = os.path.join(tmp, "libplanted.so")
    subprocess.run([compiler, "-O1", "-fPIC", "-shared", *flags, src, "-o", lib], check=True,
                   capture_output=True)
    code = ("import ctypes, sys; L = ctypes.CDLL(sys.argv[1]); "
            "print(L.planted_overflow(4))")
    r = subprocess.run([sys.executable, "-c", code, lib],
                       env=dict(os.environ, LD_PRELOAD=runtime,
                                ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0"),
                       capture_output=True, text=True, timeout=300)
    return r.returncode != 0 and ("AddressSanitizer" in r.stderr or
                                  "runtime error" in r.stderr)


def test_oracle_pins_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory(prefix="gce_san_") as tmp:
        lib = os.path.join(tmp, "libce_oracle.so")
        subprocess.run(["gcc", *oracle.CFLAGS, *SAN, oracle._SRC, "-o", lib, "-lm"],
                       check=True)
        runtime = _gcc_asan()
        assert _planted_reported("gcc", SAN, runtime, tmp)
        r = _run_pytest(["tests/test_oracle_pins.py"],
                        {"CE_ORACLE_LIB": lib, "LD_PRELOAD": runtime,
                         "ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": UBSAN_OPTIONS})
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
        assert "passed" in r.stdout and "runtime error" not in r.stderr
        assert "ERROR: AddressSanitizer" not in r.stderr


def test_host_library_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory(prefix="gce_san_") as tmp:
        objs, cmds = [], []
        for s in gbuild.SOURCES:
            o = os.path.join(tmp, os.path.splitext(s)[0] + ".o")
            objs.append(o)
            cmds.append([gbuild.HIPCC, *gbuild.FLAGS, *HIP_SAN, "-c",
                         os.path.join(gbuild.CSRC, s), "-o", o])
        with ThreadPoolExecutor(max_workers=min(8, len(cmds))) as ex:
            for f in [ex.submit(gbuild._run, c, False) for c in cmds]:
                f.result()
        lib = os.path.join(tmp, "libgce.so")
        gbuild._run([gbuild.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HIP_SAN,
                     "-shared-libasan", *objs, "-o", lib], False)
        runtime = _clang_asan()
        assert _planted_reported(gbuild.HIPCC, HIP_SAN, runtime, tmp)
        r = _run_pytest(["tests/test_abi.py", "tests/test_merge.py"],
                        {"GCE_LIB": lib, "LD_PRELOAD": runtime,
                         "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0",
                         "UBSAN_OPTIONS": UBSAN_OPTIONS})
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
        assert "passed" in r.stdout and "runtime error" not in r.stderr
        assert "ERROR: AddressSanitizer" not in r.stderr
