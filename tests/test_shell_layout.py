"""The shell of partial moment sums a tile chunk leaves for its neighbours
(the one-pass step) gives every target cell around the chunk its own slot:
the library's slot functions, compiled for the host and checked over every
chunk extent (no GPU needed).  The same program checks that the XCD order of
the tile launches is a bijection onto the tiles with one contiguous run of
each chunk per XCD."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_shell_slots_distinct_and_in_range(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "shell_layout_check"
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17", "-Wno-unused-value",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2508_00577_amd", "csrc"),
                    os.path.join(ROOT, "tests", "shell_layout_check.hip"), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout
