"""Range claims of the fast arithmetic policy (estimated Shoup quotient, Cooley-Tukey values
in [0, 16q) with reduction every other stage), checked on the host against unsigned __int128
(no GPU).  The GPU parity tests check the kernels' own code bit for bit."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fast_shoup_bounds(tmp_path):
    exe = tmp_path / "fast_shoup_bounds"
    subprocess.check_call(["g++", "-std=c++17", "-O2", os.path.join(ROOT, "tests", "host", "fast_shoup_bounds.cpp"),
                           "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout
