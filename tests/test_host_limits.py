"""Host-side guards of the library that need no GPU: the work-list size
limits of the WSPD traversal, compiled from the library's own header with
g++ and run as a plain program."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_worklist_limits(tmp_path):
    src = os.path.join(ROOT, "tests", "native", "limits_check.cpp")
    exe = str(tmp_path / "limits_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-o", exe, src])
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "limits: ok" in out.stdout
