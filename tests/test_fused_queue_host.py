"""The fused kernel's queue order, compiled for the host from the header the kernel uses."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("flags", [["-O2"], ["-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]],
                         ids=["plain", "asan_ubsan"])
def test_fused_queue_order(tmp_path, flags):
    exe = tmp_path / "fused_queue_check"
    subprocess.check_call(["g++", "-std=c++17", *flags, "-I", os.path.join(ROOT, "paper_2012_01968_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host", "fused_queue_check.cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout
