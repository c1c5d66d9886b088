"""The host runtime (api.cpp, server.cpp) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer, linked with the in-tree HIP
objects, and the C ABI's CPU tests (tests/test_abi_cpu.py) run against it in
a child process that preloads the sanitizer runtimes.  Any sanitizer report
aborts the child (undefined behaviour is made fatal)."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2005_06727_amd")
CSRC = os.path.join(PKG, "csrc")
HOST_SOURCES = ("api.cpp", "server.cpp")


def _hip_objects():
    objs = sorted(glob.glob(os.path.join(PKG, "_build", "*.o")))
    return [o for o in objs if os.path.basename(o)[:-2] + ".cpp" not in HOST_SOURCES]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_abi_cpu_tests_under_asan_ubsan(tmp_path):
    objs = _hip_objects()
    if not objs:
        pytest.skip("the library's HIP objects are not built (python -m paper_2005_06727_amd.build)")
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    host = []
    for src in HOST_SOURCES:
        out = str(tmp_path / (src[:-4] + ".o"))
        subprocess.run(["g++", *flags, "-c", os.path.join(CSRC, src), "-o", out], check=True,
                       capture_output=True, text=True)
        host.append(out)
    lib = str(tmp_path / "libwmd_san.so")
    subprocess.run(["g++", "-shared", "-fPIC", "-fsanitize=address,undefined", "-o", lib, *host, *objs,
                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True,
                   capture_output=True, text=True)
    rt = [subprocess.run(["g++", f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
          for n in ("libasan.so", "libubsan.so")]
    env = dict(os.environ, WMD_LIBRARY=lib, LD_PRELOAD=" ".join(rt),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    probe = ("from paper_2005_06727_amd import wmd; import sys; "
             "maps = open('/proc/self/maps').read(); "
             "sys.exit(0 if wmd.LIB_PATH.endswith('libwmd_san.so') and 'libasan' in maps else 3)")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
