"""Host-side check of the exact multiply-shift division (Granlund and
Montgomery's round-up method) that the element, tangent and G^T kernels use
to turn element and DOF indices into lattice coordinates.  The check program
includes the library's own kernel header and is built for the host by hipcc."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not available")
def test_fastdiv_matches_integer_division(tmp_path):
    exe = tmp_path / "fastdiv_check"
    src = os.path.join(HERE, "native", "fastdiv_check.cpp")
    inc = os.path.join(ROOT, "paper_2506_00746_amd", "csrc")
    build = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", inc,
                            "-I", os.path.join(ROOT, "include"), src, "-o", str(exe)],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert run.returncode == 0 and run.stdout.startswith("ok"), run.stdout + run.stderr
