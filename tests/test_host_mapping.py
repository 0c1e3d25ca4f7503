"""Host logic of the operator launch: the XCD-grouped block -> cell-run map
covers every cell of the mesh exactly once, each run inside one contiguous
segment of rows.  Built with hipcc as a host program (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not available")
def test_operator_runs_cover_every_cell_once(tmp_path):
    exe = tmp_path / "op_runs_check"
    cmd = [HIPCC, "-std=c++17", "-I", os.path.join(ROOT, "paper_1910_11239_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "host", "op_runs_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad 0" in out.stdout
