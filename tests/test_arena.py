"""Host-side check of the serving loop's device-memory arena (first-fit with
merging), compiled with g++ on the CPU: randomised allocations and releases
against a byte map (no overlap, alignment, bounds, no false failures, full
merge when emptied)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2003_07968_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "arena_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_against_byte_map(tmp_path):
    exe = str(tmp_path / "arena_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                    "-I", CSRC, SRC, "-o", exe], check=True)
    for seed in (1, 2, 3):
        res = subprocess.run([exe, str(seed)], capture_output=True, text=True, timeout=120)
        assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout + res.stderr
