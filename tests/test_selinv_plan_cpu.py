"""Host-side checks of the sparse-direct full map (no GPU): the plan query
of the C ABI, the batch entry point's host-side rejections, and
tests/cpp/selinv_plan_check.cpp, which drives the library's symbolic plan
(single stacks, and several stacks merged into one forest as the batch
does) through the panel factorisation and Takahashi recurrence as plain
loops against dense inverses of G."""
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
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900)
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


@pytest.mark.parametrize("case", ["disconnected", "node_range", "bad_plan", "empty"])
def test_batch_rejections_on_the_host(case):
    """reff_selinv_batch validates and analyses every plan on the host before
    any device work: a plan whose second tier has no TSV column (G
    singular), a node id out of range and an invalid descriptor are
    refused with the plan named; an empty batch is a no-op."""
    import numpy as np
    from paper_2607_05818_amd import reff
    good = gen.small_random_desc(31, 2, 6, 5, 3, 2)
    if case == "empty":
        outs, st = reff.reff_selinv_batch([])
        assert outs == [] and st["n_fronts"] == 0
        return
    other = dict(good)
    nodes = None
    want = reff.REFF_ERR_INVALID_ARG
    if case == "disconnected":
        other["tsv_xy"] = np.zeros((0, 2), dtype=np.int32)
        other["tsv_g"] = np.zeros((0, 1))
        want = reff.REFF_ERR_DISCONNECTED
    elif case == "node_range":
        nodes = [None, [0, gen.n_nodes(good)]]
    else:
        other["pad_xy"] = [[99, 0]]
    with pytest.raises(reff.ReffError) as ei:
        reff.reff_selinv_batch([good, other], nodes)
    assert ei.value.status == want
    assert "plan 1" in reff.reff_last_error()
