import ctypes
import os
import subprocess
import sys
import tempfile

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def torch_philox():
    import torch.utils.cpp_extension as ce
    out = os.path.join(tempfile.gettempdir(), f"capred_philox_ref_{os.getuid()}.so")
    src = os.path.join(ROOT, "tests", "philox_ref.cpp")
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        inc = sum((["-I", p] for p in ce.include_paths()), [])
        subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", *inc, "-o", out + ".tmp", src],
                       check=True)
        os.replace(out + ".tmp", out)
    lib = ctypes.CDLL(out)
    lib.ref_philox.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4 + [
        np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")]
    lib.ref_philox.restype = None

    def f(seed, c0, c1, c2, c3):
        o = np.empty(4, np.uint32)
        lib.ref_philox(seed, c0, c1, c2, c3, o)
        return o
    return f


