"""The host side of libhisv.so under AddressSanitizer + UBSan.

Every source is built as for the library, at -O1 with both sanitizers on the
host pass only (device code is unchanged and never runs here), and
tests/test_host_lib.py runs again in a child process against that build
(the ASan runtime preloaded into the interpreter, leaks not reported).  This
covers what those tests reach on the host: the circuit front end, every
partitioner, the part compiler for both dtypes, the specialized-source
generator, fused-part unitaries, AUTO's cost model and plan validation.
The two tests that cap the child's address space are left out (ASan's
allocator aborts on a failed allocation instead of returning it).
"""

import glob
import os
import subprocess
import sys

import pytest

from paper_2205_06973_amd import build as hbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN_RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
pytestmark = pytest.mark.skipif(not ASAN_RT or not os.path.exists("/opt/rocm/bin/hipcc"),
                                reason="needs hipcc and its ASan runtime")


@pytest.fixture(scope="module")
def asan_library(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("hisv_asan"))
    flags = [f for f in hbuild.COMMON if f not in ("-O3", "-Wall")]
    flags += ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize=vptr", "-Xarch_host", "-fno-sanitize-recover=all"]
    procs, objs = [], []
    for src in hbuild.sources():
        obj = os.path.join(d, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen([hbuild.hipcc(), *flags, "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err[-3000:]
    lib = os.path.join(d, "libhisv_asan.so")
    # the sanitizer runtime comes from the preloaded library at run time
    r = subprocess.run([hbuild.hipcc(), f"--offload-arch={hbuild.ARCH}", "-shared", "-fPIC", "-o", lib,
                        *objs, "-lhiprtc", "-lpthread"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return lib


def test_host_library_tests_pass_under_asan_ubsan(asan_library):
    env = dict(os.environ, PYTHONPATH=ROOT, HISV_TEST_LIBRARY=asan_library, LD_PRELOAD=ASAN_RT[-1],
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_host_lib.py"), "-q", "-x",
           "-m", "not gpu", "-p", "tests.host_san.use_library", "-p", "no:cacheprovider",
           "-k", "not allocation_failure and not threads_cannot_start"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=1200, env=env, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in r.stdout
    assert f"mapped libhisv builds: {asan_library}\n" in r.stdout, r.stdout[-2000:]
