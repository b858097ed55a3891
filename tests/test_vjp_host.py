"""The reverse-mode building blocks of the adjoint step (csrc/dg2_vjp.h),
compiled for the host and checked against fourth-order central differences
of their own forward functions: HLL flux in every wave regime (both wet,
supercritical either way, one side dry), physical flux at Gauss points with
the dummy limit, the prescribed-discharge inflow flux (critical depth and
inner depth branches) and the friction split of a planar element, including
the derivative with respect to the Manning coefficient."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2010_02003_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not found")
def test_vjp_building_blocks_vs_central_differences(tmp_path):
    exe = str(tmp_path / "vjp_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(HERE, "vjp_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 failures" in r.stdout
