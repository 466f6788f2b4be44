"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function include/reff.h declares, and invalid or disconnected
inputs are rejected by host validation before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2607_05818_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(inc, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(reff_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2607_05818_amd import reff
    lib = C.CDLL(reff.LIB_PATH)
    declared = _declared_functions()
    assert {"reff_build_pdn", "reff_solve_diag", "reff_query_pairs", "reff_batch_plans"} <= declared
    for name in sorted(declared):
        assert hasattr(lib, name), name


def test_status_strings():
    from paper_2607_05818_amd import reff
    assert reff.reff_status_string(0) == "ok"
    assert "invalid" in reff.reff_status_string(-1)
    assert "disconnected" in reff.reff_status_string(-2)


def _bad(desc, **kw):
    d = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in desc.items()}
    d.update(kw)
    return d


@pytest.mark.parametrize("case", [
    "gx_zero", "gx_nan", "gy_neg", "tsv_g_inf", "tsv_out", "tsv_dup", "pad_out", "no_pads",
    "dims",
])
def test_invalid_descriptors_rejected_on_host(case):
    from paper_2607_05818_amd import reff
    d = gen.config1()
    if case == "gx_zero":
        d = _bad(d); d["gx"][0, 3, 4] = 0.0
    elif case == "gx_nan":
        d = _bad(d); d["gx"][1, 0, 0] = np.nan
    elif case == "gy_neg":
        d = _bad(d); d["gy"][0, 2, 2] = -1.0
    elif case == "tsv_g_inf":
        d = _bad(d); d["tsv_g"][3, 0] = np.inf
    elif case == "tsv_out":
        d = _bad(d); d["tsv_xy"][0, 0] = 32
    elif case == "tsv_dup":
        d = _bad(d); d["tsv_xy"][1] = d["tsv_xy"][0]
    elif case == "pad_out":
        d = _bad(d); d["pad_xy"][2, 1] = -1
    elif case == "no_pads":
        d = _bad(d, pad_xy=np.zeros((0, 2), dtype=np.int32))
    elif case == "dims":
        d = _bad(d, n_tiers=0)
    with pytest.raises(reff.ReffError) as ei:
        reff.reff_build_pdn(d)
    assert ei.value.status == reff.REFF_ERR_INVALID_ARG


def test_disconnected_tier_rejected():
    """A tier with no TSV column cannot reach the pads: G is singular."""
    from paper_2607_05818_amd import reff
    d = gen.config1()
    d = _bad(d, tsv_xy=np.zeros((0, 2), dtype=np.int32), tsv_g=np.zeros((0, 1)))
    with pytest.raises(reff.ReffError) as ei:
        reff.reff_build_pdn(d)
    assert ei.value.status == reff.REFF_ERR_DISCONNECTED
    assert "no resistive path" in reff.reff_last_error()


@pytest.mark.parametrize("case", ["bad_plan", "disconnected", "node_range", "graphs_flag"])
def test_batch_rejected_on_host(case):
    """reff_batch_plans validates every plan, node list and option before
    any device work (so these run without a GPU)."""
    from paper_2607_05818_amd import reff
    good = gen.config1()
    plans = [good, _bad(good)]
    nodes = [np.array([3, 4], dtype=np.int64), np.array([5], dtype=np.int64)]
    if case == "bad_plan":
        plans[1]["gy"][0, 0, 0] = 0.0
        want = reff.REFF_ERR_INVALID_ARG
    elif case == "disconnected":
        plans[1] = _bad(good, tsv_xy=np.zeros((0, 2), dtype=np.int32), tsv_g=np.zeros((0, 1)))
        want = reff.REFF_ERR_DISCONNECTED
    elif case == "node_range":
        nodes[1] = np.array([gen.n_nodes(good)], dtype=np.int64)
        want = reff.REFF_ERR_INVALID_ARG
    else:
        want = reff.REFF_ERR_INVALID_ARG
    if case == "graphs_flag":
        structs = (reff.reff_pdn_desc * 1)()
        s, keep = reff._desc_struct(good)
        structs[0] = s
        out = np.zeros(2)
        nptr = (C.c_void_p * 1)(nodes[0].ctypes.data)
        cnt = (C.c_int64 * 1)(2)
        optr = (C.c_void_p * 1)(out.ctypes.data)
        bo = reff.reff_batch_opts()
        bo.solve.graphs = 3
        st = reff._lib.reff_batch_plans(structs, 1, nptr, cnt, optr, C.byref(bo), None)
        assert st == want
        return
    with pytest.raises(reff.ReffError) as ei:
        reff.reff_batch_plans(plans, nodes, precision=reff.REFF_PREC_FP64)
    assert ei.value.status == want


@pytest.mark.parametrize("case", ["one_tier", "no_tsv", "dup_tsv", "off_grid", "neg_r"])
def test_reduced_pairs_rejected_on_host(case):
    from paper_2607_05818_amd import reff
    r_t, s_t = np.ones(3), np.ones(3)
    txy = np.array([[1, 1], [2, 3]], dtype=np.int32)
    tr = np.ones((2, 2))
    bxy = np.array([[0, 0]], dtype=np.int32)
    lxy = np.array([[4, 4]], dtype=np.int32)
    if case == "one_tier":
        r_t, s_t, tr = np.ones(1), np.ones(1), np.ones((2, 0))
    elif case == "no_tsv":
        txy, tr = np.zeros((0, 2), dtype=np.int32), np.ones((0, 2))
    elif case == "dup_tsv":
        txy = np.array([[1, 1], [1, 1]], dtype=np.int32)
    elif case == "off_grid":
        lxy = np.array([[5, 0]], dtype=np.int32)
    elif case == "neg_r":
        tr = -np.ones((2, 2))
    with pytest.raises(reff.ReffError) as ei:
        reff.reff_reduced_pairs(5, 5, r_t, s_t, txy, tr, bxy, lxy)
    assert ei.value.status == reff.REFF_ERR_INVALID_ARG


@pytest.mark.parametrize("brhs", [16, 48, 128, -1])
def test_block_rhs_other_than_0_32_64_rejected(brhs):
    """Options are parsed on the host before any device work (a batch call
    parses them before touching its plans' device state)."""
    from paper_2607_05818_amd import reff
    d = gen.config1()
    s, keep = reff._desc_struct(d)
    plans = (reff.reff_pdn_desc * 1)(s)
    nptrs = (C.c_void_p * 1)(None)
    ncount = (C.c_int64 * 1)(gen.n_nodes(d))
    out = np.zeros(gen.n_nodes(d))
    optrs = (C.c_void_p * 1)(out.ctypes.data)
    bo = reff.reff_batch_opts()
    bo.solve = reff._opts(reff.REFF_PREC_FP64, 0.0, 0, 0, None, False, 0, block_rhs=brhs)
    rc = reff._lib.reff_batch_plans(plans, 1, nptrs, ncount, optrs, C.byref(bo), None)
    assert rc == reff.REFF_ERR_INVALID_ARG
    assert "block_rhs" in reff.reff_last_error()
