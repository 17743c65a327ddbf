"""Host checks of the boundary's bookkeeping, compiled with g++ from the headers the library
uses (no GPU): the plan lifetime rules (plans shared by their creator and the batches that
name them) and the reader of the tuner's flat file (use_autotune)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_01968_amd", "csrc")


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.mark.parametrize("sanitize", [False, True], ids=["plain", "asan_ubsan"])
@pytest.mark.parametrize("check", ["plan_life_check", "tune_file_check", "crt_math_check"])
def test_host_check(tmp_path, check, sanitize):
    """Also built with AddressSanitizer and UndefinedBehaviorSanitizer: the headers are the
    library's own host code (reference counts, the tuner file reader, the conversion tables)."""
    exe = tmp_path / check
    subprocess.check_call(["g++", "-std=c++17", "-O1" if sanitize else "-O2", "-Wall", *(SANITIZE if sanitize else []),
                           "-I", CSRC, os.path.join(ROOT, "tests", "host", check + ".cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout


def test_oracle_under_sanitizers(tmp_path):
    """The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer, every entry point on
    N = 2..256, results checked against each other (tests/host/oracle_sanitize_check.c)."""
    exe = tmp_path / "oracle_sanitize_check"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-Wall", *SANITIZE,
                           os.path.join(ROOT, "tests", "host", "oracle_sanitize_check.c"),
                           os.path.join(ROOT, "oracle", "ntt_oracle.c"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout


def test_flat_tune_file_matches_the_json_cache():
    """The committed flat file is the tuner's JSON cache, line for line, in the format the
    library parses (csrc/tune_file.hpp)."""
    pytest.importorskip("torch")
    from paper_2012_01968_amd import autotune
    import json
    with open(autotune.cache_path()) as f:
        cache = json.load(f)
    lines = autotune.flat_lines(cache)
    assert len(lines) == len(cache["entries"])
    with open(autotune.flat_path()) as f:
        assert f.read().splitlines() == lines
    for line in lines:
        fields = line.split()
        assert len(fields) == 14
        assert all(x.lstrip("-").isdigit() for x in fields[2:])
