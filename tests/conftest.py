import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def csr_checker(tmp_path_factory):
    """The network row checker of tests/native/csr_check.cpp (g++, OpenMP):
    test infrastructure, no GPU code."""
    import ctypes
    import subprocess

    so = str(tmp_path_factory.mktemp("csr_check") / "csr_check.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", so,
                           os.path.join(ROOT, "tests", "native", "csr_check.cpp")])
    L = ctypes.CDLL(so)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    L.csr_check_rows.argtypes = [i64, i64, i64, vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.csr_check_rows.restype = i64
    return L
