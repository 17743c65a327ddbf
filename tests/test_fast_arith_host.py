"""Range claims of the fast arithmetic policy (estimated Shoup quotient, Cooley-Tukey values
in [0, 16q) with reduction every other stage, integer quotient estimate in the final
reduction), checked on the host against unsigned __int128 (no GPU).  The GPU parity tests
check the kernels' own code bit for bit."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "fast_shoup_bounds.cpp")


def _run(tmp_path, name, defines=()):
    exe = tmp_path / name
    subprocess.check_call(["g++", "-std=c++17", "-O2", *defines, SRC, "-o", str(exe)])
    return subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)


def test_fast_shoup_bounds(tmp_path):
    out = _run(tmp_path, "fast_shoup_bounds")
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout


@pytest.mark.parametrize("planted", ["-DQSHIFT=2", "-DQEXTRA=7", "-DQROUNDUP=1"])
def test_planted_quotient_mistakes_fail(tmp_path, planted):
    """A shift one bit short, a multiplier of twice the size, or a multiplier rounded up each
    break the quotient estimate's claim, and the check must say so."""
    out = _run(tmp_path, "planted", [planted])
    assert out.returncode != 0 and "0 failures" not in out.stdout, out.stdout
