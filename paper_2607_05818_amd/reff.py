"""Thin ctypes binding of libreff.so (the C ABI in include/reff.h).

The functions keep the C names and only marshal arguments: every step of
the computation runs in the library's HIP kernels.  Buffers may be numpy
arrays (host) or torch CUDA tensors (device); a CUDA output tensor selects
``out_on_device`` and the caller's current torch stream is used unless a
stream is given.  Importing this module raises if the library has not been
built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# REFF_LIBRARY names another build of the library (A/B timing of variants)
LIB_PATH = os.environ.get("REFF_LIBRARY") or os.path.join(_HERE, "libreff.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2607_05818_amd.build` "
        "(HIP for gfx950); there is no CPU fallback")

try:  # share PyTorch's HIP runtime (libreff is linked against it)
    import torch  # noqa: F401
except ImportError:
    torch = None
_lib = C.CDLL(LIB_PATH)

REFF_OK = 0
REFF_ERR_INVALID_ARG = -1
REFF_ERR_DISCONNECTED = -2
REFF_ERR_NO_CONVERGENCE = -3
REFF_ERR_OUT_OF_MEMORY = -4
REFF_ERR_DEVICE = -5
REFF_ERR_UNSUPPORTED = -6

REFF_PREC_FP64 = 0
REFF_PREC_MIXED = 1
REFF_KRYLOV_BLOCK = 0
REFF_KRYLOV_INDEPENDENT = 1
REFF_PAIRS_GROUNDED = 0
REFF_PAIRS_FLOATING = 1

EXPORTED = [
    "reff_build_pdn", "reff_free_pdn", "reff_pdn_num_nodes", "reff_solve_diag",
    "reff_query_pairs", "reff_batch_plans", "reff_status_string", "reff_last_error",
    "reff_surrogate_create", "reff_surrogate_free", "reff_surrogate_num_params",
    "reff_surrogate_get_params", "reff_surrogate_set_params", "reff_surrogate_loss_grad",
    "reff_surrogate_train", "reff_surrogate_predict", "reff_surrogate_save",
    "reff_surrogate_load", "reff_grid_pairs", "reff_grid_pairs_noalloc", "reff_reduced_pairs",
    "reff_ir_drop",
]


class reff_pdn_desc(C.Structure):
    _fields_ = [
        ("n_tiers", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("gx", C.POINTER(C.c_double)), ("gy", C.POINTER(C.c_double)),
        ("n_tsv", C.c_int32), ("tsv_xy", C.POINTER(C.c_int32)),
        ("tsv_g", C.POINTER(C.c_double)),
        ("n_pads", C.c_int32), ("pad_xy", C.POINTER(C.c_int32)),
    ]


class reff_solve_opts(C.Structure):
    _fields_ = [
        ("precision", C.c_int), ("rel_tol", C.c_double), ("max_iters", C.c_int32),
        ("block_rhs", C.c_int32), ("stream", C.c_void_p), ("out_on_device", C.c_int32),
        ("krylov", C.c_int), ("max_ir_steps", C.c_int32), ("timing", C.c_int32),
        ("graphs", C.c_int32), ("progress", C.c_int32), ("precond_degree", C.c_int32),
        ("pairs_resident_blocks", C.c_int32),
    ]


class reff_solve_stats(C.Structure):
    _fields_ = [
        ("n_solved", C.c_int64), ("n_unconverged", C.c_int64), ("iters_max", C.c_int32),
        ("ir_steps", C.c_int32), ("seconds", C.c_double), ("est_max_rel_err", C.c_double),
        ("iters_total", C.c_int64), ("kernel_ms", C.c_double * 5),
        ("kernel_launches", C.c_int64 * 5), ("kernel_rows", C.c_int64 * 5),
        ("screened", C.c_int32), ("spot_max_rel_err", C.c_double),
    ]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if k.startswith("kernel_") else v
        return out


class reff_selinv_stats(C.Structure):
    _fields_ = [
        ("n_fronts", C.c_int64), ("n_levels", C.c_int32), ("reserved", C.c_int32),
        ("max_front", C.c_int64), ("device_bytes", C.c_int64), ("flops_factor", C.c_double),
        ("flops_selinv", C.c_double), ("seconds", C.c_double), ("seconds_plan", C.c_double),
        ("seconds_factor", C.c_double), ("seconds_selinv", C.c_double),
        ("seconds_setup", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class reff_batch_opts(C.Structure):
    _fields_ = [
        ("solve", reff_solve_opts), ("surrogate", C.c_void_p), ("spot_frac", C.c_double),
        ("fallback_rel_err", C.c_double), ("tune_db", C.c_char_p), ("calibrate", C.c_int32),
    ]


_lib.reff_build_pdn.argtypes = [C.POINTER(reff_pdn_desc), C.c_int32, C.POINTER(C.c_void_p)]
_lib.reff_build_pdn.restype = C.c_int
_lib.reff_free_pdn.argtypes = [C.c_void_p]
_lib.reff_free_pdn.restype = None
_lib.reff_pdn_num_nodes.argtypes = [C.c_void_p]
_lib.reff_pdn_num_nodes.restype = C.c_int64
_lib.reff_solve_diag.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                 C.POINTER(reff_solve_opts), C.POINTER(reff_solve_stats)]
_lib.reff_solve_diag.restype = C.c_int
_lib.reff_query_pairs.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                  C.c_int, C.c_void_p, C.POINTER(reff_solve_opts),
                                  C.POINTER(reff_solve_stats)]
_lib.reff_query_pairs.restype = C.c_int
_lib.reff_batch_plans.argtypes = [C.POINTER(reff_pdn_desc), C.c_int32,
                                  C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_void_p), C.POINTER(reff_batch_opts),
                                  C.POINTER(reff_solve_stats)]
_lib.reff_batch_plans.restype = C.c_int
_lib.reff_grid_pairs.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_void_p,
                                 C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]
_lib.reff_grid_pairs.restype = C.c_int
_lib.reff_grid_pairs_noalloc.argtypes = _lib.reff_grid_pairs.argtypes
_lib.reff_reduced_pairs.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                    C.c_int64, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
_lib.reff_reduced_pairs.restype = C.c_int
_lib.reff_ir_drop.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32,
                              C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                              C.POINTER(reff_solve_opts), C.POINTER(reff_solve_stats)]
_lib.reff_ir_drop.restype = C.c_int
_lib.reff_grid_pairs_noalloc.restype = C.c_int
_lib.reff_selinv_diag.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.POINTER(reff_solve_opts), C.POINTER(reff_selinv_stats)]
_lib.reff_selinv_diag.restype = C.c_int
_lib.reff_selinv_info.argtypes = [C.POINTER(reff_pdn_desc), C.POINTER(reff_selinv_stats)]
_lib.reff_selinv_info.restype = C.c_int
_lib.reff_selinv_batch.argtypes = [C.POINTER(reff_pdn_desc), C.c_int32,
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_void_p), C.POINTER(reff_solve_opts),
                                   C.POINTER(reff_selinv_stats)]
_lib.reff_selinv_batch.restype = C.c_int
_lib.reff_release_cached_memory.argtypes = [C.c_int32]
_lib.reff_release_cached_memory.restype = C.c_int
_lib.reff_stream_probe.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                   C.c_void_p]
_lib.reff_stream_probe.restype = C.c_int
_lib.reff_status_string.argtypes = [C.c_int]
_lib.reff_status_string.restype = C.c_char_p
_lib.reff_last_error.argtypes = []
_lib.reff_last_error.restype = C.c_char_p


class ReffError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__(f"{reff_status_string(status)} ({status}): {detail}")


def reff_status_string(status: int) -> str:
    return _lib.reff_status_string(int(status)).decode()


def reff_last_error() -> str:
    return _lib.reff_last_error().decode()


def _check(status, allow=()):
    if status != REFF_OK and status not in allow:
        raise ReffError(status, reff_last_error())
    return status


def _desc_struct(desc):
    """Pack a descriptor dict into the C struct; returns (struct, keepalive)."""
    nt, nx, ny = int(desc["n_tiers"]), int(desc["nx"]), int(desc["ny"])
    arrs = {
        "gx": np.ascontiguousarray(desc["gx"], dtype=np.float64).ravel(),
        "gy": np.ascontiguousarray(desc["gy"], dtype=np.float64).ravel(),
        "tsv_xy": np.ascontiguousarray(desc["tsv_xy"], dtype=np.int32).ravel(),
        "tsv_g": np.ascontiguousarray(desc["tsv_g"], dtype=np.float64).ravel(),
        "pad_xy": np.ascontiguousarray(desc["pad_xy"], dtype=np.int32).ravel(),
    }
    s = reff_pdn_desc()
    s.n_tiers, s.nx, s.ny = nt, nx, ny
    s.gx = arrs["gx"].ctypes.data_as(C.POINTER(C.c_double))
    s.gy = arrs["gy"].ctypes.data_as(C.POINTER(C.c_double))
    s.n_tsv = len(arrs["tsv_xy"]) // 2
    s.tsv_xy = arrs["tsv_xy"].ctypes.data_as(C.POINTER(C.c_int32))
    s.tsv_g = arrs["tsv_g"].ctypes.data_as(C.POINTER(C.c_double))
    s.n_pads = len(arrs["pad_xy"]) // 2
    s.pad_xy = arrs["pad_xy"].ctypes.data_as(C.POINTER(C.c_int32))
    return s, arrs


class PDN:
    """Owner of a reff_pdn handle."""

    def __init__(self, handle, device, n_pads=0):
        self.handle = handle
        self.device = device
        self.n_pads = int(n_pads)   # pad entries of the descriptor

    @property
    def num_nodes(self):
        return int(_lib.reff_pdn_num_nodes(self.handle))

    def close(self):
        if self.handle:
            _lib.reff_free_pdn(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reff_build_pdn(desc, device: int = 0) -> PDN:
    s, keep = _desc_struct(desc)
    h = C.c_void_p()
    _check(_lib.reff_build_pdn(C.byref(s), int(device), C.byref(h)))
    del keep
    return PDN(h, device, np.asarray(desc["pad_xy"]).reshape(-1, 2).shape[0])


def reff_free_pdn(pdn: PDN) -> None:
    pdn.close()


def _is_torch_cuda(x):
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


def _opts(precision, rel_tol, max_iters, krylov, stream, out_dev, max_ir_steps, timing=False,
          graphs=None, progress=False, precond_degree=0, block_rhs=0):
    o = reff_solve_opts()
    o.progress = 1 if progress else 0
    o.precond_degree = int(precond_degree)
    o.timing = 1 if timing else 0
    # None: automatic (graph replay where possible); True: replay; False: plain
    o.graphs = 0 if graphs is None else (1 if graphs else 2)
    o.precision = int(precision)
    o.rel_tol = float(rel_tol)
    o.max_iters = int(max_iters)
    o.block_rhs = int(block_rhs)
    o.krylov = int(krylov)
    o.max_ir_steps = int(max_ir_steps)
    o.out_on_device = 1 if out_dev else 0
    if stream is None and out_dev:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    o.stream = C.c_void_p(int(stream) if stream is not None else 0)
    return o


def reff_solve_diag(pdn: PDN, nodes=None, R_out=None, *, precision=REFF_PREC_FP64,
                    rel_tol=0.0, max_iters=0, krylov=REFF_KRYLOV_BLOCK, stream=None,
                    max_ir_steps=0, allow_unconverged=False, timing=False, graphs=None,
                    progress=False, precond_degree=0, block_rhs=0):
    """R_i = (G^-1)_ii for `nodes` (None = all).  Returns (R_out, stats)."""
    if nodes is None:
        count = pdn.num_nodes
        nodes_arr = None
        nptr = None
    else:
        nodes_arr = np.ascontiguousarray(nodes, dtype=np.int64)
        count = len(nodes_arr)
        nptr = nodes_arr.ctypes.data
    if R_out is None:
        R_out = np.empty(count, dtype=np.float64)
    out_dev = _is_torch_cuda(R_out)
    if out_dev:
        assert R_out.dtype.__repr__().endswith("float64") and R_out.is_contiguous()
        assert R_out.numel() >= count
        optr = R_out.data_ptr()
    else:
        assert R_out.dtype == np.float64 and R_out.flags.c_contiguous and len(R_out) >= count
        optr = R_out.ctypes.data
    o = _opts(precision, rel_tol, max_iters, krylov, stream, out_dev, max_ir_steps, timing, graphs,
              progress, precond_degree, block_rhs)
    st = reff_solve_stats()
    allow = (REFF_ERR_NO_CONVERGENCE,) if allow_unconverged else ()
    _check(_lib.reff_solve_diag(pdn.handle, nptr, count if nodes is not None else 0, optr,
                                C.byref(o), C.byref(st)), allow)
    return R_out, st.as_dict()


def reff_selinv_diag(pdn: PDN, nodes=None, R_out=None, *, stream=None):
    """R_i = (G^-1)_ii for `nodes` (None = all) by sparse-direct selected
    inversion on the GPU.  Returns (R_out, stats)."""
    if nodes is None:
        count, nptr = pdn.num_nodes, None
    else:
        nodes_arr = np.ascontiguousarray(nodes, dtype=np.int64)
        count, nptr = len(nodes_arr), nodes_arr.ctypes.data
    if R_out is None:
        R_out = np.empty(count, dtype=np.float64)
    out_dev = _is_torch_cuda(R_out)
    if out_dev:
        assert R_out.dtype.__repr__().endswith("float64") and R_out.is_contiguous()
        assert R_out.numel() >= count
        optr = R_out.data_ptr()
    else:
        assert R_out.dtype == np.float64 and R_out.flags.c_contiguous and len(R_out) >= count
        optr = R_out.ctypes.data
    o = _opts(REFF_PREC_FP64, 0.0, 0, REFF_KRYLOV_BLOCK, stream, out_dev, 0)
    st = reff_selinv_stats()
    _check(_lib.reff_selinv_diag(pdn.handle, nptr, count if nodes is not None else 0, optr,
                                 C.byref(o), C.byref(st)))
    return R_out, st.as_dict()


def reff_selinv_batch(plans, nodes=None, R_out=None, *, stream=None):
    """reff_selinv_diag for many stack descriptors in one call (no handle).
    Returns (list of R arrays, stats)."""
    k = len(plans)
    structs = (reff_pdn_desc * k)()
    keep = []
    for i, d in enumerate(plans):
        st_, kp = _desc_struct(d)
        structs[i] = st_
        keep.append(kp)
    nptrs = (C.c_void_p * k)()
    ncount = (C.c_int64 * k)()
    optrs = (C.c_void_p * k)()
    outs, node_arrs = [], []
    out_dev = False
    for i, d in enumerate(plans):
        if nodes is None or nodes[i] is None:
            nptrs[i] = None
            cnt = int(d["n_tiers"]) * int(d["nx"]) * int(d["ny"])
        else:
            arr = np.ascontiguousarray(nodes[i], dtype=np.int64)
            node_arrs.append(arr)
            nptrs[i] = arr.ctypes.data
            cnt = len(arr)
        ncount[i] = cnt
        if R_out is not None:
            o = R_out[i]
            out_dev = _is_torch_cuda(o)
            optrs[i] = o.data_ptr() if out_dev else o.ctypes.data
        else:
            o = np.empty(cnt, dtype=np.float64)
            optrs[i] = o.ctypes.data
        outs.append(o)
    o = _opts(REFF_PREC_FP64, 0.0, 0, REFF_KRYLOV_BLOCK, stream, out_dev, 0)
    st = reff_selinv_stats()
    _check(_lib.reff_selinv_batch(structs, k, nptrs, ncount, optrs, C.byref(o), C.byref(st)))
    del keep, node_arrs
    return outs, st.as_dict()


def reff_release_cached_memory(device=0):
    """Return the device memory the sparse-direct path keeps pooled."""
    _check(_lib.reff_release_cached_memory(int(device)))


def reff_stream_probe(kind, src, dst, nbytes, blocks, stream=None):
    """One launch of an HBM bandwidth probe kernel on device tensors (see
    include/reff.h); asynchronous on `stream` (default: torch's current)."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    _check(_lib.reff_stream_probe(int(kind), src.data_ptr() if src is not None else None,
                                  dst.data_ptr(), int(nbytes), int(blocks),
                                  C.c_void_p(int(stream))))


def reff_selinv_info(desc):
    """Plan of reff_selinv_diag for a stack descriptor (host only): fronts,
    levels, largest front, device bytes, flop counts."""
    ds, keep = _desc_struct(desc)
    st = reff_selinv_stats()
    _check(_lib.reff_selinv_info(C.byref(ds), C.byref(st)))
    del keep
    return st.as_dict()


def reff_query_pairs(pdn: PDN, a, b, mode=REFF_PAIRS_GROUNDED, R_out=None, *,
                     precision=REFF_PREC_FP64, rel_tol=0.0, max_iters=0,
                     krylov=REFF_KRYLOV_BLOCK, stream=None, max_ir_steps=0, precond_degree=0,
                     resident_blocks=0):
    """m x n pair resistances R(a_i, b_j).  Returns (R_out, stats).
    resident_blocks: solution blocks kept on the device at once (0 = as many
    as half the free device memory holds)."""
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    m, n = len(a), len(b)
    if R_out is None:
        R_out = np.empty((m, n), dtype=np.float64)
    out_dev = _is_torch_cuda(R_out)
    optr = R_out.data_ptr() if out_dev else R_out.ctypes.data
    o = _opts(precision, rel_tol, max_iters, krylov, stream, out_dev, max_ir_steps,
              precond_degree=precond_degree)
    o.pairs_resident_blocks = int(resident_blocks)
    st = reff_solve_stats()
    _check(_lib.reff_query_pairs(pdn.handle, a.ctypes.data, m, b.ctypes.data, n, int(mode),
                                 optr, C.byref(o), C.byref(st)))
    return R_out, st.as_dict()


def reff_ir_drop(pdn: PDN, load_nodes, load_amps, nodes=None, drop_out=None, *,
                 precision=REFF_PREC_FP64, rel_tol=0.0, max_iters=0, stream=None,
                 precond_degree=0, pad_amps=True):
    """IR drop of load scenarios by superposition of unit-load responses
    (Eq. 4) and the current each pad delivers.  load_amps: (n_scen, n_loads).
    Returns (drop (n_scen, len(nodes) or n), pad currents (n_scen, n_pads) or
    None, stats)."""
    ln = np.ascontiguousarray(load_nodes, dtype=np.int64)
    la = np.ascontiguousarray(np.atleast_2d(load_amps), dtype=np.float64)
    assert la.shape[1] == len(ln)
    n_scen = la.shape[0]
    if nodes is None:
        count, nptr, narr = pdn.num_nodes, None, None
    else:
        narr = np.ascontiguousarray(nodes, dtype=np.int64)
        count, nptr = len(narr), narr.ctypes.data
    if drop_out is None:
        drop_out = np.empty((n_scen, count), dtype=np.float64)
    out_dev = _is_torch_cuda(drop_out)
    optr = drop_out.data_ptr() if out_dev else drop_out.ctypes.data
    npad = pdn.n_pads
    pa = np.empty((n_scen, npad), dtype=np.float64) if (pad_amps and npad) else None
    o = _opts(precision, rel_tol, max_iters, REFF_KRYLOV_BLOCK, stream, out_dev, 0,
              precond_degree=precond_degree)
    st = reff_solve_stats()
    _check(_lib.reff_ir_drop(pdn.handle, ln.ctypes.data, len(ln), la.ctypes.data, n_scen, nptr,
                             count if nodes is not None else 0, optr,
                             pa.ctypes.data if pa is not None else None, C.byref(o),
                             C.byref(st)))
    return drop_out, pa, st.as_dict()


def _grid_pairs_call(fn, M, N, r, s, xy, R_out, stream):
    pts = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    P = len(pts)
    if R_out is None:
        R_out = np.empty((P, P), dtype=np.float64)
    out_dev = _is_torch_cuda(R_out)
    if out_dev:
        assert R_out.dtype.__repr__().endswith("float64") and R_out.is_contiguous()
        assert R_out.numel() >= P * P
        optr = R_out.data_ptr()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
    else:
        assert R_out.dtype == np.float64 and R_out.flags.c_contiguous and R_out.size >= P * P
        optr = R_out.ctypes.data
    _check(fn(int(M), int(N), float(r), float(s), pts.ctypes.data, P, optr, 1 if out_dev else 0,
              C.c_void_p(int(stream) if stream is not None else 0)))
    return R_out


def reff_grid_pairs(M, N, r, s, xy, R_out=None, *, stream=None):
    """Eq. 3 two-point resistances of every pair of points on a uniform
    M x N grid (edges r along x, s along y).  xy: (P, 2) integer points.
    Returns the P x P matrix (R_out if given: numpy or a torch CUDA tensor)."""
    return _grid_pairs_call(_lib.reff_grid_pairs, M, N, r, s, xy, R_out, stream)


def reff_grid_pairs_noalloc(M, N, r, s, xy, R_out=None, *, stream=None):
    """reff_grid_pairs through the entry point that allocates no device
    memory (the library's fixed per-GPU work array)."""
    return _grid_pairs_call(_lib.reff_grid_pairs_noalloc, M, N, r, s, xy, R_out, stream)


def reff_reduced_pairs(nx, ny, r_t, s_t, tsv_xy, tsv_r, bump_xy, load_xy, R_out=None, *,
                       stream=None):
    """Bump (tier 0) to load (last tier) pair resistances of a stack of
    uniform tiers by the reduced system of Sec. III-C/D.  r_t, s_t: per-tier
    edge resistances along x and y; tsv_xy (p, 2); tsv_r (p, d-1) segment
    resistances; bump_xy (m, 2); load_xy (n, 2).  Returns the m x n matrix
    (R_out if given: numpy or a torch CUDA tensor)."""
    r_t = np.ascontiguousarray(r_t, dtype=np.float64)
    s_t = np.ascontiguousarray(s_t, dtype=np.float64)
    d = len(r_t)
    assert len(s_t) == d
    txy = np.ascontiguousarray(tsv_xy, dtype=np.int32).reshape(-1, 2)
    p = len(txy)
    tr = np.ascontiguousarray(tsv_r, dtype=np.float64).reshape(p, max(d - 1, 0))
    bxy = np.ascontiguousarray(bump_xy, dtype=np.int32).reshape(-1, 2)
    lxy = np.ascontiguousarray(load_xy, dtype=np.int32).reshape(-1, 2)
    m, n = len(bxy), len(lxy)
    if R_out is None:
        R_out = np.empty((m, n), dtype=np.float64)
    out_dev = _is_torch_cuda(R_out)
    if out_dev:
        assert R_out.is_contiguous() and R_out.numel() >= m * n
        optr = R_out.data_ptr()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
    else:
        assert R_out.dtype == np.float64 and R_out.flags.c_contiguous and R_out.size >= m * n
        optr = R_out.ctypes.data
    _check(_lib.reff_reduced_pairs(d, int(nx), int(ny), r_t.ctypes.data, s_t.ctypes.data, p,
                                   txy.ctypes.data, tr.ctypes.data, m, bxy.ctypes.data, n,
                                   lxy.ctypes.data, optr, 1 if out_dev else 0,
                                   C.c_void_p(int(stream) if stream is not None else 0)))
    return R_out


def reff_batch_plans(plans, nodes=None, *, precision=REFF_PREC_MIXED, rel_tol=0.0,
                     max_iters=0, krylov=REFF_KRYLOV_BLOCK, stream=None, R_out=None,
                     timing=False, surrogate=None, spot_frac=0.0, fallback_rel_err=0.0,
                     graphs=None, tune_db=None, precond_degree=0, calibrate=False):
    """Solve many plans in one call.  Returns (list of R arrays, list of stats)."""
    k = len(plans)
    structs = (reff_pdn_desc * k)()
    keep = []
    for i, d in enumerate(plans):
        s, kp = _desc_struct(d)
        structs[i] = s
        keep.append(kp)
    node_arrs = []
    nptrs = (C.c_void_p * k)()
    ncount = (C.c_int64 * k)()
    outs = []
    optrs = (C.c_void_p * k)()
    out_dev = False
    for i, d in enumerate(plans):
        if nodes is None or nodes[i] is None:
            nptrs[i] = None
            cnt = int(d["n_tiers"]) * int(d["nx"]) * int(d["ny"])
        else:
            arr = np.ascontiguousarray(nodes[i], dtype=np.int64)
            node_arrs.append(arr)
            nptrs[i] = arr.ctypes.data
            cnt = len(arr)
        ncount[i] = cnt
        if R_out is not None:
            o = R_out[i]
            out_dev = _is_torch_cuda(o)
            optrs[i] = o.data_ptr() if out_dev else o.ctypes.data
            outs.append(o)
        else:
            o = np.empty(cnt, dtype=np.float64)
            optrs[i] = o.ctypes.data
            outs.append(o)
    bo = reff_batch_opts()
    bo.solve = _opts(precision, rel_tol, max_iters, krylov, stream, out_dev, 0, timing, graphs,
                     precond_degree=precond_degree)
    if tune_db is not None:
        bo.tune_db = os.fsencode(tune_db)
    if surrogate is not None:
        bo.surrogate = surrogate.handle
        bo.spot_frac = spot_frac
        bo.fallback_rel_err = fallback_rel_err
        bo.calibrate = 1 if calibrate else 0
    stats = (reff_solve_stats * k)()
    _check(_lib.reff_batch_plans(structs, k, nptrs, ncount, optrs, C.byref(bo), stats))
    return outs, [stats[i].as_dict() for i in range(k)]


# ---------------------------------------------------------------- surrogate

class reff_surrogate_config(C.Structure):
    _fields_ = [("n_tiers", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("base_channels", C.c_int32), ("seed", C.c_uint64)]


class reff_labels(C.Structure):
    _fields_ = [("nodes", C.c_void_p), ("n_nodes", C.c_int64), ("R", C.c_void_p)]


class reff_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("seed", C.c_uint64)]


_lib.reff_surrogate_create.argtypes = [C.POINTER(reff_surrogate_config), C.c_int32,
                                       C.POINTER(C.c_void_p)]
_lib.reff_surrogate_create.restype = C.c_int
_lib.reff_surrogate_free.argtypes = [C.c_void_p]
_lib.reff_surrogate_free.restype = None
_lib.reff_surrogate_num_params.argtypes = [C.c_void_p]
_lib.reff_surrogate_num_params.restype = C.c_int64
_lib.reff_surrogate_get_params.argtypes = [C.c_void_p, C.c_void_p]
_lib.reff_surrogate_get_params.restype = C.c_int
_lib.reff_surrogate_set_params.argtypes = [C.c_void_p, C.c_void_p]
_lib.reff_surrogate_set_params.restype = C.c_int
_lib.reff_surrogate_loss_grad.argtypes = [C.c_void_p, C.POINTER(reff_pdn_desc),
                                          C.POINTER(reff_labels), C.c_int32,
                                          C.POINTER(C.c_double), C.c_void_p]
_lib.reff_surrogate_loss_grad.restype = C.c_int
_lib.reff_surrogate_train.argtypes = [C.c_void_p, C.POINTER(reff_pdn_desc),
                                      C.POINTER(reff_labels), C.c_int32,
                                      C.POINTER(reff_train_opts), C.c_void_p]
_lib.reff_surrogate_train.restype = C.c_int
_lib.reff_surrogate_predict.argtypes = [C.c_void_p, C.POINTER(reff_pdn_desc), C.c_int32,
                                        C.POINTER(C.c_void_p), C.c_int32]
_lib.reff_surrogate_predict.restype = C.c_int
_lib.reff_surrogate_save.argtypes = [C.c_void_p, C.c_char_p]
_lib.reff_surrogate_save.restype = C.c_int
_lib.reff_surrogate_load.argtypes = [C.c_char_p, C.c_int32, C.POINTER(C.c_void_p)]
_lib.reff_surrogate_load.restype = C.c_int


class Surrogate:
    """Owning wrapper of a reff_surrogate handle."""

    def __init__(self, handle, geometry):
        self.handle = handle
        self.geometry = geometry

    def close(self):
        if self.handle:
            _lib.reff_surrogate_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _plan_structs(plans):
    structs = (reff_pdn_desc * max(len(plans), 1))()
    keep = []
    for i, d in enumerate(plans):
        s, kp = _desc_struct(d)
        structs[i] = s
        keep.append(kp)
    return structs, keep


def _label_structs(labels):
    arr = (reff_labels * max(len(labels), 1))()
    keep = []
    for i, (nodes, R) in enumerate(labels):
        n = np.ascontiguousarray(nodes, dtype=np.int64)
        r = np.ascontiguousarray(R, dtype=np.float64)
        assert n.shape == r.shape
        keep += [n, r]
        arr[i] = reff_labels(n.ctypes.data, len(n), r.ctypes.data)
    return arr, keep


def reff_surrogate_create(n_tiers, nx, ny, base_channels=32, seed=0, device=0) -> Surrogate:
    cfg = reff_surrogate_config(n_tiers, nx, ny, base_channels, seed)
    h = C.c_void_p()
    _check(_lib.reff_surrogate_create(C.byref(cfg), device, C.byref(h)))
    return Surrogate(h, (n_tiers, nx, ny))


def reff_surrogate_free(s: Surrogate) -> None:
    s.close()


def reff_surrogate_num_params(s: Surrogate) -> int:
    return int(_lib.reff_surrogate_num_params(s.handle))


def reff_surrogate_get_params(s: Surrogate) -> np.ndarray:
    out = np.empty(reff_surrogate_num_params(s), dtype=np.float32)
    _check(_lib.reff_surrogate_get_params(s.handle, out.ctypes.data))
    return out


def reff_surrogate_set_params(s: Surrogate, params) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == reff_surrogate_num_params(s)
    _check(_lib.reff_surrogate_set_params(s.handle, p.ctypes.data))


def reff_surrogate_loss_grad(s: Surrogate, plans, labels, grad=True):
    """labels: list of (node ids, R values) per plan.  Returns (loss, grad)."""
    structs, keep = _plan_structs(plans)
    lab, keep2 = _label_structs(labels)
    loss = C.c_double()
    g = np.empty(reff_surrogate_num_params(s), dtype=np.float32) if grad else None
    _check(_lib.reff_surrogate_loss_grad(s.handle, structs, lab, len(plans), C.byref(loss),
                                         g.ctypes.data if grad else None))
    return loss.value, g


def reff_surrogate_train(s: Surrogate, plans, labels, *, epochs=1, batch=16, lr=1e-3, seed=0):
    structs, keep = _plan_structs(plans)
    lab, keep2 = _label_structs(labels)
    o = reff_train_opts(epochs, batch, lr, seed)
    hist = np.zeros(max(epochs, 1))
    _check(_lib.reff_surrogate_train(s.handle, structs, lab, len(plans), C.byref(o),
                                     hist.ctypes.data))
    return hist


def reff_surrogate_predict(s: Surrogate, plans, R_out=None):
    structs, keep = _plan_structs(plans)
    nt, nx, ny = s.geometry
    if R_out is None:
        R_out = [np.empty(nt * nx * ny, dtype=np.float64) for _ in plans]
    dev = len(R_out) > 0 and _is_torch_cuda(R_out[0])
    ptrs = (C.c_void_p * max(len(plans), 1))()
    for i, o in enumerate(R_out):
        ptrs[i] = o.data_ptr() if dev else o.ctypes.data
    _check(_lib.reff_surrogate_predict(s.handle, structs, len(plans), ptrs, 1 if dev else 0))
    return R_out


def reff_surrogate_save(s: Surrogate, path: str) -> None:
    _check(_lib.reff_surrogate_save(s.handle, os.fsencode(path)))


def reff_surrogate_load(path: str, device: int = 0) -> Surrogate:
    h = C.c_void_p()
    _check(_lib.reff_surrogate_load(os.fsencode(path), device, C.byref(h)))
    with open(path, "rb") as f:
        hdr = f.read(20)
    nt, nx, ny = (int.from_bytes(hdr[8 + 4 * i:12 + 4 * i], "little", signed=True)
                  for i in range(3))
    return Surrogate(h, (nt, nx, ny))
