"""Row maps of the padded vector layouts, on the host (no GPU): the device
helpers that map representatives to stored rows and back are host-callable,
so a small program built from the library's own header runs them over every
layout shape the library builds (plain padded, aligned and packed rows,
d_Gamma 1..12, ragged representative counts) and checks that the maps are
inverse, ordered, inside the vectors, and that every other row is a gap."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_padded_row_maps_are_inverse_on_every_layout_shape(tmp_path):
    exe = str(tmp_path / "layout_rows")
    subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-std=c++17",
                    "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2607_17429_amd", "csrc"),
                    os.path.join(ROOT, "tests", "c", "layout_rows.cpp"), "-o", exe], check=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr
    lines = out.stdout.strip().splitlines()
    assert lines[-1] == "fails 0"
    assert int(lines[-2].split()[1]) >= 100          # shapes checked
    shapes = [dict(f.split("=") for f in ln.split()[1:]) for ln in lines if ln.startswith("shape ")]
    assert any(int(sh["rpl"]) > 1 for sh in shapes)                              # packed lines
    assert any(int(sh["rpl"]) == 1 and sh["rpline"] != sh["dg"] for sh in shapes)  # aligned rows
