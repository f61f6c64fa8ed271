"""Python binding of libbvmv (compressed-graph A.x and PageRank on MI355X).

Argument marshalling only: every step runs in the HIP library.  Function
names are the C-ABI names of include/bvmv.h.  Device vectors are torch
tensors (torch is used for device memory and streams); the library is loaded
after torch so both share one HIP runtime.  If the library is missing this
module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbvmv.so")

BVMV_OK, BVMV_NOT_CONVERGED = 0, 1
BVMV_EINVAL, BVMV_EFORMAT, BVMV_ENOMEM, BVMV_EDEVICE = -1, -2, -3, -4
BVMV_F64, BVMV_F32, BVMV_F32_COMP = 0, 1, 2
PREC_NAMES = {"f64": BVMV_F64, "f32": BVMV_F32, "f32c": BVMV_F32_COMP}

_lib = None


class BvmvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("bvmv error %d: %s" % (code, msg))
        self.code = code


class LoadOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("tile_rows", ctypes.c_int), ("window_cap", ctypes.c_int),
                ("stage_bytes", ctypes.c_int), ("long_row_bytes", ctypes.c_int), ("interval_mode", ctypes.c_int),
                ("autotune", ctypes.c_int),
                ("keep_lists", ctypes.c_int), ("nthreads", ctypes.c_int), ("device_mem_budget", ctypes.c_uint64)]


class PROpts(ctypes.Structure):
    _fields_ = [("damping", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("prec", ctypes.c_int), ("chunk", ctypes.c_int), ("exact_zero_damping", ctypes.c_int),
                ("fallback_check", ctypes.c_int), ("mlp", ctypes.c_void_p), ("restart_every", ctypes.c_int),
                ("max_restarts", ctypes.c_int)]


class PRResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("residual", ctypes.c_double),
                ("used_start", ctypes.c_int), ("products", ctypes.c_int), ("restarts_accepted", ctypes.c_int),
                ("restarts_rejected", ctypes.c_int)]


class BicliqueInfo(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("n", "m", "nbic", "s_ids", "c_ids", "residual", "words",
                                               "layout_bytes")]


NFEAT = 12
MLP_PARAMS = 5057


class Info(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("n", "m", "m_prime", "units", "diff_rows", "direct_rows",
                                               "long_rows", "escapes", "ntiles", "layout_bytes",
                                               "stream_bytes", "n_singles", "n_wide", "n_intervals")] + \
               [(f, ctypes.c_int) for f in ("W", "R", "Lmin", "zeta_k", "tile_rows", "window_cap",
                                            "stage_bytes", "long_row_bytes", "interval_mode", "max_level",
                                            "ngraphs", "autotuned")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def load_library():
    """Load libbvmv.so (after torch, to share its HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (brings in the HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbvmv.so is not built (run __graft_entry__.build() or "
                          "python paper_1708_07271_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int64
    P = ctypes.POINTER
    sigs = {
        "bvmv_load": ([vp, sz, P(LoadOpts), P(vp)], i32),
        "bvmv_multiply": ([vp, vp, vp, i32, vp], i32),
        "bvmv_multiply_batch": ([vp, vp, vp, i32, i64, i32, vp], i32),
        "bvmv_multiply_left": ([vp, vp, vp, i32, vp], i32),
        "bvmv_pagerank": ([vp, P(PROpts), vp, vp, vp, i32, P(PRResult), vp], i32),
        "bvmv_pagerank_noalloc": ([vp, P(PROpts), vp, vp, vp, P(PRResult), vp], i32),
        "bvmv_colblocks_create": ([P(vp), i32, P(vp)], i32),
        "bvmv_colblocks_multiply": ([vp, vp, vp, i32, vp], i32),
        "bvmv_colblocks_free": ([vp], None),
        "bvmv_biclique_load": ([i64, i64, vp, vp, vp, vp, vp, vp, i32, P(vp)], i32),
        "bvmv_biclique_multiply": ([vp, vp, vp, i32, vp], i32),
        "bvmv_biclique_get_info": ([vp, P(BicliqueInfo)], i32),
        "bvmv_biclique_free": ([vp], None),
        "bvmv_group": ([P(vp), i32, P(vp)], i32),
        "bvmv_group_offsets": ([vp, P(i64), P(i32)], i32),
        "bvmv_get_info": ([vp, P(Info)], i32),
        "bvmv_export_csr": ([vp, vp, vp], i32),
        "bvmv_degrees": ([vp, vp, vp], i32),
        "bvmv_decode": ([vp, sz, i32, vp, vp, vp, P(i64), P(i64)], i32),
        "bvmv_csr_create": ([vp, P(vp)], i32),
        "bvmv_csr_create_host": ([i64, vp, vp, i32, P(vp)], i32),
        "bvmv_csr_multiply": ([vp, vp, vp, i32, vp], i32),
        "bvmv_csr_pagerank": ([vp, P(PROpts), vp, vp, vp, P(PRResult), vp], i32),
        "bvmv_csr_bytes": ([vp], i64),
        "bvmv_csr_free": ([vp], None),
        "bvmv_free": ([vp], None),
        "bvmv_layout_selfcheck": ([vp, sz, P(LoadOpts), vp, vp, vp], i32),
        "bvmv_left_selfcheck": ([vp, sz, P(LoadOpts), vp, vp], i32),
        "bvmv_features": ([vp, vp, vp], i32),
        "bvmv_mlp_create": ([i32, vp, P(vp)], i32),
        "bvmv_mlp_params": ([vp, vp], i32),
        "bvmv_mlp_forward": ([vp, vp, i64, vp, vp], i32),
        "bvmv_mlp_gradient": ([vp, vp, vp, i64, vp, vp], i32),
        "bvmv_mlp_train_step": ([vp, vp, vp, i64, ctypes.c_float, vp, vp], i32),
        "bvmv_restart_sample": ([vp, i32, i32, vp, vp, vp, P(ctypes.c_double), vp], i32),
        "bvmv_mlp_free": ([vp], None),
        "bvmv_last_error": ([], ctypes.c_char_p),
        "bvmv_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc, allow=(BVMV_OK,)):
    if rc not in allow:
        raise BvmvError(rc, load_library().bvmv_last_error().decode())
    return rc


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError("tensor too small: %d < %d" % (t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


def _prec(prec):
    return PREC_NAMES[prec] if isinstance(prec, str) else int(prec)


def _vec_dtype(prec):
    import torch
    return torch.float64 if _prec(prec) == BVMV_F64 else torch.float32


class Graph:
    """Handle of a loaded compressed graph (owns the device layout)."""

    def __init__(self, handle, n, members=None):
        self._h = ctypes.c_void_p(handle)
        self.n = n
        self.members = members  # keeps group members alive

    @property
    def handle(self):
        return self._h

    def info(self):
        out = Info()
        _check(load_library().bvmv_get_info(self._h, ctypes.byref(out)))
        return out.as_dict()

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.bvmv_free(self._h)
            self._h = ctypes.c_void_p(None)


class Csr:
    def __init__(self, handle, n):
        self._h = ctypes.c_void_p(handle)
        self.n = n

    def bytes(self):
        return int(load_library().bvmv_csr_bytes(self._h))

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.bvmv_csr_free(self._h)
            self._h = ctypes.c_void_p(None)


def _as_u8(data):
    arr = np.ascontiguousarray(np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray))
                               else np.asarray(data, dtype=np.uint8))
    return arr


def bvmv_load(bitstream, device=0, tile_rows=0, window_cap=0, stage_bytes=0, long_row_bytes=0, interval_mode=0,
              autotune=0, keep_lists=0, nthreads=0, device_mem_budget=0) -> Graph:
    lib = load_library()
    data = _as_u8(bitstream)
    o = LoadOpts(device, tile_rows, window_cap, stage_bytes, long_row_bytes, interval_mode, autotune, keep_lists,
                 nthreads, device_mem_budget)
    h = ctypes.c_void_p()
    _check(lib.bvmv_load(data.ctypes.data, data.size, ctypes.byref(o), ctypes.byref(h)))
    info = Info()
    lib.bvmv_get_info(h, ctypes.byref(info))
    return Graph(h.value, info.n)


def bvmv_multiply(g: Graph, x, y, prec=BVMV_F32_COMP, stream=None):
    p = _prec(prec)
    dt = _vec_dtype(p)
    _check(load_library().bvmv_multiply(g.handle, _dev_ptr(x, dt, g.n), _dev_ptr(y, dt, g.n), p,
                                        _stream_ptr(stream)))


def bvmv_multiply_left(g: Graph, x, y, prec=BVMV_F32_COMP, stream=None):
    """y = x A (the left product) on the loaded rows."""
    p = _prec(prec)
    dt = _vec_dtype(p)
    _check(load_library().bvmv_multiply_left(g.handle, _dev_ptr(x, dt, g.n), _dev_ptr(y, dt, g.n), p,
                                             _stream_ptr(stream)))


def bvmv_multiply_batch(g: Graph, X, Y, prec=BVMV_F32_COMP, stream=None):
    """X, Y: (k, n) device tensors, row c = right-hand side c (the column-major
    n x k blocks of the C interface).  Rows may be views into longer rows:
    both tensors need unit element stride and the same row stride ld >= n,
    which is passed as the leading dimension."""
    import torch
    p = _prec(prec)
    dt = _vec_dtype(p)
    if X.dim() != 2 or X.shape != Y.shape or X.shape[1] != g.n:
        raise ValueError("X and Y must be (k, n)")
    k = X.shape[0]
    ld = X.stride(0) if k > 1 else g.n
    if (k > 1 and Y.stride(0) != ld) or X.stride(1) != 1 or Y.stride(1) != 1 or ld < g.n:
        raise ValueError("X and Y need unit element stride and one row stride >= n")
    for t in (X, Y):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt:
            raise TypeError("expected %s device tensors" % dt)
    _check(load_library().bvmv_multiply_batch(g.handle, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                              k, ld, p, _stream_ptr(stream)))


def _pr_opts(damping, tol, max_iter, prec, chunk, fallback_check=0, mlp=None, restart_every=0, max_restarts=0):
    return PROpts(damping, tol, max_iter, _prec(prec), chunk, 1 if damping == 0.0 else 0, int(fallback_check),
                  mlp.handle if mlp is not None else None, int(restart_every), int(max_restarts))


def bvmv_pagerank_detail(g: Graph, p_out, teleport=None, start=None, damping=0.85, tol=1e-6, max_iter=1000,
                         prec=BVMV_F32_COMP, chunk=16, k=1, fallback_check=0, stream=None, mlp=None,
                         restart_every=0, max_restarts=0):
    """Returns a list of dicts (iters, converged, residual, used_start,
    products, restarts_accepted, restarts_rejected), one per column (or member
    of a group).  With `mlp`, learned warm restarts every `restart_every`
    iterations (0 = 10), at most `max_restarts` (0 = 2)."""
    p = _prec(prec)
    dt = _vec_dtype(p)
    lib = load_library()
    nres = k
    if g.members is not None:
        nres = len(g.members)
    res = (PRResult * max(nres, 1))()
    o = _pr_opts(damping, tol, max_iter, p, chunk, fallback_check, mlp, restart_every, max_restarts)
    tp = _dev_ptr(teleport, dt, g.n * k) if teleport is not None else ctypes.c_void_p(None)
    sp = _dev_ptr(start, dt, g.n * k) if start is not None else ctypes.c_void_p(None)
    _check(lib.bvmv_pagerank(g.handle, ctypes.byref(o), tp, sp, _dev_ptr(p_out, dt, g.n * k), k, res,
                             _stream_ptr(stream)), allow=(BVMV_OK, BVMV_NOT_CONVERGED))
    return [dict(iters=r.iters, converged=bool(r.converged), residual=r.residual, used_start=r.used_start,
                 products=r.products, restarts_accepted=r.restarts_accepted, restarts_rejected=r.restarts_rejected)
            for r in res[:nres]]


def bvmv_pagerank(g: Graph, p_out, teleport=None, start=None, damping=0.85, tol=1e-6, max_iter=1000,
                  prec=BVMV_F32_COMP, chunk=16, k=1, stream=None):
    """Returns a list of (iters, converged, residual), one per column (or member of a group)."""
    out = bvmv_pagerank_detail(g, p_out, teleport, start, damping, tol, max_iter, prec, chunk, k, 0, stream)
    return [(r["iters"], r["converged"], r["residual"]) for r in out]


def bvmv_pagerank_noalloc(g: Graph, p_out, teleport=None, start=None, damping=0.85, tol=1e-6, max_iter=1000,
                          prec=BVMV_F32_COMP, chunk=16, stream=None):
    """PageRank of a single graph (k = 1) that allocates nothing: its working
    set lives in the library's fixed device array.  Returns a dict like
    bvmv_pagerank_detail's entries."""
    p = _prec(prec)
    dt = _vec_dtype(p)
    lib = load_library()
    res = PRResult()
    o = _pr_opts(damping, tol, max_iter, p, chunk)
    tp = _dev_ptr(teleport, dt, g.n) if teleport is not None else ctypes.c_void_p(None)
    sp = _dev_ptr(start, dt, g.n) if start is not None else ctypes.c_void_p(None)
    _check(lib.bvmv_pagerank_noalloc(g.handle, ctypes.byref(o), tp, sp, _dev_ptr(p_out, dt, g.n), ctypes.byref(res),
                                     _stream_ptr(stream)), allow=(BVMV_OK, BVMV_NOT_CONVERGED))
    return dict(iters=res.iters, converged=bool(res.converged), residual=res.residual, used_start=res.used_start,
                products=res.products, restarts_accepted=res.restarts_accepted,
                restarts_rejected=res.restarts_rejected)


class ColBlocks:
    """Handle of column blocks; keeps the member graphs alive."""

    def __init__(self, handle, n, blocks):
        self._h = handle
        self.n = n
        self.blocks = list(blocks)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.bvmv_colblocks_free(self._h)
            self._h = None


def bvmv_colblocks_create(blocks) -> ColBlocks:
    arr = (ctypes.c_void_p * len(blocks))(*[b.handle.value for b in blocks])
    h = ctypes.c_void_p()
    _check(load_library().bvmv_colblocks_create(arr, len(blocks), ctypes.byref(h)))
    return ColBlocks(h, blocks[0].n, blocks)


def bvmv_colblocks_multiply(c: ColBlocks, x, y, prec=BVMV_F32_COMP, stream=None):
    p = _prec(prec)
    dt = _vec_dtype(p)
    _check(load_library().bvmv_colblocks_multiply(c.handle, _dev_ptr(x, dt, c.n), _dev_ptr(y, dt, c.n), p,
                                                  _stream_ptr(stream)))


class Biclique:
    """Handle of a biclique layout (freed with the object)."""

    def __init__(self, handle, n):
        self._h = handle
        self.n = n

    @property
    def handle(self):
        return self._h

    def info(self):
        i = BicliqueInfo()
        _check(load_library().bvmv_biclique_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in BicliqueInfo._fields_}

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.bvmv_biclique_free(self._h)
            self._h = None


def bvmv_biclique_load(bic, device=0) -> Biclique:
    """bic: a decomposition with fields n, sptr, sidx, cptr, cidx, rptr, rcol
    (host arrays; e.g. bvinputs.Bicliques)."""
    lib = load_library()
    u64 = lambda a: np.ascontiguousarray(a, dtype=np.uint64)
    u32 = lambda a: np.ascontiguousarray(a, dtype=np.uint32)
    arrs = [u64(bic.sptr), u32(bic.sidx), u64(bic.cptr), u32(bic.cidx), u64(bic.rptr), u32(bic.rcol)]
    ptrs = [a.ctypes.data if a.size else None for a in arrs]
    h = ctypes.c_void_p()
    _check(lib.bvmv_biclique_load(int(bic.n), int(arrs[0].size - 1), *ptrs, device, ctypes.byref(h)))
    return Biclique(h, int(bic.n))


def bvmv_biclique_multiply(b: Biclique, x, y, prec=BVMV_F32_COMP, stream=None):
    p = _prec(prec)
    dt = _vec_dtype(p)
    _check(load_library().bvmv_biclique_multiply(b.handle, _dev_ptr(x, dt, b.n), _dev_ptr(y, dt, b.n), p,
                                                 _stream_ptr(stream)))


def bvmv_group(graphs) -> Graph:
    lib = load_library()
    arr = (ctypes.c_void_p * len(graphs))(*[gr.handle.value for gr in graphs])
    h = ctypes.c_void_p()
    _check(lib.bvmv_group(arr, len(graphs), ctypes.byref(h)))
    info = Info()
    lib.bvmv_get_info(h, ctypes.byref(info))
    return Graph(h.value, info.n, members=list(graphs))


def bvmv_group_offsets(g: Graph):
    lib = load_library()
    cnt = ctypes.c_int()
    _check(lib.bvmv_group_offsets(g.handle, None, ctypes.byref(cnt)))
    offs = (ctypes.c_int64 * (cnt.value + 1))()
    _check(lib.bvmv_group_offsets(g.handle, offs, ctypes.byref(cnt)))
    return list(offs)


def bvmv_get_info(g: Graph):
    return g.info()


def bvmv_export_csr(g: Graph):
    info = g.info()
    rowptr = np.zeros(info["n"] + 1, dtype=np.uint64)
    col = np.zeros(max(info["m"], 1), dtype=np.uint32)
    _check(load_library().bvmv_export_csr(g.handle, rowptr.ctypes.data, col.ctypes.data))
    return rowptr, col[:info["m"]]


def bvmv_degrees(g: Graph, deg, stream=None):
    import torch
    _check(load_library().bvmv_degrees(g.handle, _dev_ptr(deg, torch.int32, g.n), _stream_ptr(stream)))


def bvmv_decode(bitstream, nthreads=0):
    """Host-only decode: (rowptr uint64, col uint32, refs uint8)."""
    lib = load_library()
    data = _as_u8(bitstream)
    n, m = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.bvmv_decode(data.ctypes.data, data.size, nthreads, None, None, None, ctypes.byref(n),
                           ctypes.byref(m)))
    rowptr = np.zeros(n.value + 1, dtype=np.uint64)
    col = np.zeros(max(m.value, 1), dtype=np.uint32)
    refs = np.zeros(n.value, dtype=np.uint8)
    _check(lib.bvmv_decode(data.ctypes.data, data.size, nthreads, rowptr.ctypes.data, col.ctypes.data,
                           refs.ctypes.data, ctypes.byref(n), ctypes.byref(m)))
    return rowptr, col[:m.value], refs


def bvmv_csr_create(g: Graph) -> Csr:
    h = ctypes.c_void_p()
    _check(load_library().bvmv_csr_create(g.handle, ctypes.byref(h)))
    return Csr(h.value, g.n)


def bvmv_csr_create_host(rowptr, col, device=0) -> Csr:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    h = ctypes.c_void_p()
    n = rowptr.size - 1
    _check(load_library().bvmv_csr_create_host(n, rowptr.ctypes.data, col.ctypes.data, device, ctypes.byref(h)))
    return Csr(h.value, n)


def bvmv_csr_multiply(c: Csr, x, y, prec=BVMV_F32_COMP, stream=None):
    p = _prec(prec)
    dt = _vec_dtype(p)
    _check(load_library().bvmv_csr_multiply(c._h, _dev_ptr(x, dt, c.n), _dev_ptr(y, dt, c.n), p,
                                            _stream_ptr(stream)))


def bvmv_csr_pagerank(c: Csr, p_out, teleport=None, start=None, damping=0.85, tol=1e-6, max_iter=1000,
                      prec=BVMV_F32_COMP, chunk=16, stream=None):
    p = _prec(prec)
    dt = _vec_dtype(p)
    res = (PRResult * 1)()
    o = _pr_opts(damping, tol, max_iter, p, chunk)
    tp = _dev_ptr(teleport, dt, c.n) if teleport is not None else ctypes.c_void_p(None)
    sp = _dev_ptr(start, dt, c.n) if start is not None else ctypes.c_void_p(None)
    _check(load_library().bvmv_csr_pagerank(c._h, ctypes.byref(o), tp, sp, _dev_ptr(p_out, dt, c.n), res,
                                            _stream_ptr(stream)), allow=(BVMV_OK, BVMV_NOT_CONVERGED))
    return (res[0].iters, bool(res[0].converged), res[0].residual)


def bvmv_layout_selfcheck(bitstream, x, tile_rows=0, window_cap=0, stage_bytes=0, long_row_bytes=0):
    """Host interpretation of the device layout (test aid): y = A x in double."""
    data = _as_u8(bitstream)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    stats = np.zeros(9, dtype=np.int64)
    o = LoadOpts(0, tile_rows, window_cap, stage_bytes, long_row_bytes, 0, 0, 0, 0, 0)
    _check(load_library().bvmv_layout_selfcheck(data.ctypes.data, data.size, ctypes.byref(o), x.ctypes.data,
                                                y.ctypes.data, stats.ctypes.data))
    keys = ["ntiles", "units", "diff_rows", "direct_rows", "long_rows", "escapes", "layout_bytes", "m_prime",
            "max_level"]
    return y, dict(zip(keys, stats.tolist()))


def bvmv_left_selfcheck(bitstream, x, tile_rows=0, window_cap=0, stage_bytes=0, long_row_bytes=0, interval_mode=0):
    """Host interpretation of the left product's layout (test aid): y = x A in double."""
    data = _as_u8(bitstream)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    o = LoadOpts(0, tile_rows, window_cap, stage_bytes, long_row_bytes, interval_mode, 0, 0, 0, 0)
    _check(load_library().bvmv_left_selfcheck(data.ctypes.data, data.size, ctypes.byref(o), x.ctypes.data,
                                              y.ctypes.data))
    return y


def bvmv_version():
    return load_library().bvmv_version().decode()


# ------------------------------------------------------------ learned warm start
class Mlp:
    """Handle of a warm-start network (FP32 master parameters, BF16 weight
    copies and Adam state on the device)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.bvmv_mlp_free(self._h)
            self._h = ctypes.c_void_p(None)


def bvmv_features(g: Graph, F, stream=None):
    """Structural inputs into columns 0..7 of F, an (n, 12) float32 device tensor."""
    import torch
    _check(load_library().bvmv_features(g.handle, _dev_ptr(F, torch.float32, g.n * NFEAT), _stream_ptr(stream)))


def bvmv_mlp_create(params, device=0) -> Mlp:
    params = np.ascontiguousarray(params, dtype=np.float32)
    if params.size != MLP_PARAMS:
        raise ValueError("expected %d parameters" % MLP_PARAMS)
    h = ctypes.c_void_p()
    _check(load_library().bvmv_mlp_create(device, params.ctypes.data, ctypes.byref(h)))
    return Mlp(h.value)


def bvmv_mlp_params(m: Mlp):
    out = np.zeros(MLP_PARAMS, dtype=np.float32)
    _check(load_library().bvmv_mlp_params(m.handle, out.ctypes.data))
    return out


def bvmv_mlp_forward(m: Mlp, F, s, stream=None):
    import torch
    n = s.numel()
    _check(load_library().bvmv_mlp_forward(m.handle, _dev_ptr(F, torch.float32, n * NFEAT),
                                           n, _dev_ptr(s, torch.float32, n), _stream_ptr(stream)))


def bvmv_mlp_gradient(m: Mlp, F, target, grad, stream=None):
    """grad: float32 device tensor of MLP_PARAMS + 1 (the gradient, then the loss)."""
    import torch
    n = target.numel()
    _check(load_library().bvmv_mlp_gradient(m.handle, _dev_ptr(F, torch.float32, n * NFEAT),
                                            _dev_ptr(target, torch.float32, n), n,
                                            _dev_ptr(grad, torch.float32, MLP_PARAMS + 1), _stream_ptr(stream)))


def bvmv_mlp_train_step(m: Mlp, F, target, lr, loss=None, stream=None):
    import torch
    n = target.numel()
    lp = _dev_ptr(loss, torch.float32, 1) if loss is not None else ctypes.c_void_p(None)
    _check(load_library().bvmv_mlp_train_step(m.handle, _dev_ptr(F, torch.float32, n * NFEAT),
                                              _dev_ptr(target, torch.float32, n), n, float(lr), lp,
                                              _stream_ptr(stream)))


def bvmv_restart_sample(g: Graph, K, F, T=None, p_star=None, prec=BVMV_F32_COMP, stream=None):
    """K plain iterations from the uniform vector, then the 12 inputs into F
    ((n, 12) float32) and, with p_star, the target into T ((n,) float32).
    Returns delta = ||p_K - p_{K-1}||_1."""
    import torch
    p = _prec(prec)
    if (T is None) != (p_star is None):
        raise ValueError("T and p_star go together")
    d = ctypes.c_double()
    _check(load_library().bvmv_restart_sample(
        g.handle, int(K), p, _dev_ptr(p_star, _vec_dtype(p), g.n) if p_star is not None else ctypes.c_void_p(None),
        _dev_ptr(F, torch.float32, g.n * NFEAT), _dev_ptr(T, torch.float32, g.n) if T is not None else
        ctypes.c_void_p(None), ctypes.byref(d), _stream_ptr(stream)))
    return d.value
