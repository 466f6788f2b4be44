"""Host-side checks of the sparse-direct full map (no GPU): the plan query
of the C ABI, and tests/cpp/selinv_plan_check.cpp, which drives the
library's symbolic plan through the panel factorisation and Takahashi
recurrence as plain loops against a dense inverse of G."""
import os
import shutil
import subprocess

import pytest

from paper_2607_05818_amd import gen

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2607_05818_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_plan_and_panel_algorithm_match_dense_inverse(tmp_path):
    exe = str(tmp_path / "selinv_plan_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe,
                    os.path.join(HERE, "cpp", "selinv_plan_check.cpp"),
                    os.path.join(CSRC, "selinv_plan.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all ok" in r.stdout


def test_plan_query_on_the_host():
    """reff_selinv_info needs no device.  For the 4 x 512 x 512 stack the
    dissection tree is complete (2^15 - 1 fronts over 15 levels) and the
    largest front is a 256-column separator of a 256 x 512 box with its
    512-column boundary wall, over 4 tiers: (256 + 512) x 4 = 3072."""
    from paper_2607_05818_amd import reff
    info = reff.reff_selinv_info(gen.config2())
    assert info["n_fronts"] == 2 ** 15 - 1
    assert info["n_levels"] == 15
    assert info["max_front"] == 3072
    assert info["flops_factor"] > 1e11 and info["flops_selinv"] > info["flops_factor"]
    assert info["device_bytes"] > 8 * 1048576


def test_plan_query_rejects_bad_descriptors():
    from paper_2607_05818_amd import reff
    d = gen.small_random_desc(3, 2, 6, 5, 2, 1)
    d = dict(d)
    d["pad_xy"] = [[9, 9]]
    with pytest.raises(reff.ReffError):
        reff.reff_selinv_info(d)
