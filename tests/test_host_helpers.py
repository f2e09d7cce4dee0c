"""Host checks of device helpers that have a plain definition (CPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_morton_rank_is_the_rank_of_the_morton_code(tmp_path):
    """The storage sort keys cells by the rank of their Morton code within
    the level grid, computed in closed form; compare with sorting every
    code of random grids (the helper is compiled for the host)."""
    exe = tmp_path / "morton_rank_check"
    src = os.path.join(ROOT, "tests", "morton_rank_check.cpp")
    inc = os.path.join(ROOT, "paper_2501_05300_amd", "csrc")
    r = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I" + inc, src, "-o", str(exe)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_neighbour_rows_cover_every_cell_within_reach(tmp_path):
    """The broad phase's rows at one level (the box of neighbour cells, less
    rows and end cells wholly out of reach) are built on the host from
    random grids: reads stay inside the level's cells, no entry is covered
    twice, every particle within the reach is covered, and with one entry
    per cell the covered cells are exactly those closer than the reach."""
    exe = tmp_path / "cell_rows_check"
    src = os.path.join(ROOT, "tests", "cell_rows_check.cpp")
    inc = os.path.join(ROOT, "paper_2501_05300_amd", "csrc")
    r = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I" + inc, src, "-o", str(exe)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr
