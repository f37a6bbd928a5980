"""Host code of libcapred under AddressSanitizer (CPU only; no GPU is touched).

Every unit of the library is compiled with its host half instrumented
(-Xarch_host -fsanitize=address; the device half as usual) into a scratch
directory and linked into a copy of the library; tests/asan/host_checks.cpp
then drives the argument validation of every entry point family, the error
strings, the persistent launch's tile cut, the workspace query and the plan's
error-path cleanup through it.  An out-of-bounds access, use after free or
double free aborts the driver; a wrong status fails it.  The instrumented
build takes one to two minutes.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

from paper_2603_01122_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
INCLUDE = os.path.join(HERE, "..", "include")


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_host_code_under_asan(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    flags = [f"--offload-arch={B.ARCH}", "-O1", "-std=c++17", "-fPIC",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", INCLUDE]

    def compile_unit(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([hipcc, *flags, "-c", os.path.join(B.CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, f"{src}:\n{r.stderr[-2000:]}"
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(B.SOURCES), os.cpu_count() or 2)) as ex:
        objs = list(ex.map(compile_unit, B.SOURCES))
    lib = str(tmp_path / "libcapred_asan.so")
    r = subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC",
                        "-Xarch_host", "-fsanitize=address", "-o", lib, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "host_checks")
    r = subprocess.run([hipcc, "-x", "c++", "-O1", "-g", "-std=c++17",
                        "-Xarch_host", "-fsanitize=address", "-I", INCLUDE,
                        os.path.join(HERE, "asan", "host_checks.cpp"),
                        f"-L{tmp_path}", "-lcapred_asan", f"-Wl,-rpath,{tmp_path}", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    # the HIP runtime frees some of its own state only at process exit
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "host checks passed" in r.stdout, r.stdout + r.stderr[-4000:]
