"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the CPU oracle, driven through every entry point on small random QPs (hard
and soft rows, refinement, absolute formulation, warm starts), and the
serving layer's first-fit device arena against its unit-map model."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe), *args], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok"), res.stdout + res.stderr
    assert "runtime error" not in res.stderr, res.stderr


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_drive"
    subprocess.run(["gcc", "-std=c99", *SAN, "-o", str(exe), os.path.join(HERE, "native", "oracle_drive.c"), "-lm"],
                   check=True)
    _run(exe)


@pytest.mark.parametrize("seed", [1, 2])
def test_arena_under_sanitizers(tmp_path, seed):
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-std=c++17", *SAN, "-o", str(exe), os.path.join(HERE, "native", "arena_check.cpp")],
                   check=True)
    _run(exe, str(seed))
