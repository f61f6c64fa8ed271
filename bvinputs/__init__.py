"""Seeded synthetic inputs shared by the CPU oracle and the HIP library.

This module holds none of the method's arithmetic: it generates graphs (as
CSR adjacency lists), encodes them into the project's BV-style bitstream (the
input format of ``bvmv_load``) and draws the vectors the workloads use.  Both
sides decode the bitstream with decoders of their own.

It also produces the input of the biclique product: a decomposition of the
edges into bicliques plus residual edges, mined from a graph
(``biclique_mine``, ``biclique.c``) or planted (``planted_bicliques``).

The native part (``gen.c``, ``biclique.c``) is plain C built with gcc; see
``build()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libbvinputs.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c and biclique.c into libbvinputs.so (host C, gcc -O3,
    pthreads)."""
    if force or not os.path.exists(_SO):
        srcs = [os.path.join(_HERE, "gen.c"), os.path.join(_HERE, "biclique.c")]
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-Wno-unused-variable"] + srcs + ["-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build(force=False)
    lib = ctypes.CDLL(_SO)
    P = ctypes.POINTER
    lib.bvi_web_graph.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, P(P(ctypes.c_uint64)),
                                  P(P(ctypes.c_uint32)), P(ctypes.c_int64)]
    lib.bvi_web_graph.restype = ctypes.c_int
    lib.bvi_social_graph.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.c_double,
                                     ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                     P(P(ctypes.c_uint64)), P(P(ctypes.c_uint32)), P(ctypes.c_int64)]
    lib.bvi_social_graph.restype = ctypes.c_int
    lib.bvi_powerlaw_shift.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_double]
    lib.bvi_powerlaw_shift.restype = ctypes.c_double
    lib.bvi_encode.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                               P(P(ctypes.c_uint8)), P(ctypes.c_int64), ctypes.c_void_p]
    lib.bvi_encode.restype = ctypes.c_int
    lib.bvi_biclique_mine.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int64, ctypes.c_int, P(ctypes.c_int64),
                                      P(P(ctypes.c_uint64)), P(P(ctypes.c_uint32)), P(P(ctypes.c_uint64)),
                                      P(P(ctypes.c_uint32)), P(P(ctypes.c_uint64)), P(P(ctypes.c_uint32))]
    lib.bvi_biclique_mine.restype = ctypes.c_int
    lib.bvi_free.argtypes = [ctypes.c_void_p]
    lib.bvi_free.restype = None
    _lib = lib
    return lib


def _take(ptr, count, dtype):
    lib = _load()
    if count == 0:
        lib.bvi_free(ctypes.cast(ptr, ctypes.c_void_p))
        return np.zeros(0, dtype=dtype)
    arr = np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)
    lib.bvi_free(ctypes.cast(ptr, ctypes.c_void_p))
    return arr


@dataclass
class Graph:
    """Adjacency lists as CSR: row i lists the out-neighbours of node i,
    strictly increasing.  rowptr is uint64 (n+1), col is uint32 (m)."""
    rowptr: np.ndarray
    col: np.ndarray

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.rowptr[-1])

    def row(self, i: int) -> np.ndarray:
        return self.col[int(self.rowptr[i]):int(self.rowptr[i + 1])]

    def transpose(self) -> "Graph":
        """In-link lists: row v lists every u with an edge u -> v."""
        n = self.n
        src = np.repeat(np.arange(n, dtype=np.uint32), np.diff(self.rowptr).astype(np.int64))
        order = np.lexsort((src, self.col))
        col_t = src[order]
        counts = np.bincount(self.col, minlength=n).astype(np.uint64)
        rp = np.zeros(n + 1, dtype=np.uint64)
        np.cumsum(counts, out=rp[1:])
        return Graph(rp, col_t.astype(np.uint32))


def web_graph(n: int, mean_deg: float, seed: int, proto_window: int = 7, p_copy: float = 0.7,
              gap_mean: float = 8.0) -> Graph:
    """Web-like copying-model graph (prototype among the previous
    `proto_window` nodes, copy each link with p_copy, new links at geometric
    gaps near i, half of them runs of >= 4 consecutive ids)."""
    lib = _load()
    rp = ctypes.POINTER(ctypes.c_uint64)()
    cp = ctypes.POINTER(ctypes.c_uint32)()
    m = ctypes.c_int64()
    rc = lib.bvi_web_graph(n, mean_deg, seed, proto_window, p_copy, gap_mean,
                           ctypes.byref(rp), ctypes.byref(cp), ctypes.byref(m))
    if rc != 0:
        raise RuntimeError("bvi_web_graph failed (%d)" % rc)
    return Graph(_take(rp, n + 1, np.uint64), _take(cp, m.value, np.uint32))


def social_graph(n: int, mean_deg: float, max_deg: int, exponent: float, seed: int,
                 proto_window: int = 7, p_copy: float = 0.3, bfs: bool = True) -> Graph:
    """Social-like graph: out-degree P(k) ~ (k+s)^-exponent on [1, max_deg]
    with the shift s solved for the mean, weak copying, uniform random other
    targets, then BFS renumbering."""
    lib = _load()
    rp = ctypes.POINTER(ctypes.c_uint64)()
    cp = ctypes.POINTER(ctypes.c_uint32)()
    m = ctypes.c_int64()
    rc = lib.bvi_social_graph(n, mean_deg, max_deg, exponent, seed, proto_window, p_copy, int(bfs),
                              ctypes.byref(rp), ctypes.byref(cp), ctypes.byref(m))
    if rc != 0:
        raise RuntimeError("bvi_social_graph failed (%d)" % rc)
    return Graph(_take(rp, n + 1, np.uint64), _take(cp, m.value, np.uint32))


def powerlaw_shift(mean_deg: float, max_deg: int, exponent: float) -> float:
    return float(_load().bvi_powerlaw_shift(mean_deg, max_deg, exponent))


@dataclass
class Encoded:
    data: np.ndarray      # uint8 bitstream (header + offsets + body)
    refs: np.ndarray      # uint8 reference gap g_i chosen by the encoder (0 = none)
    W: int
    R: int
    Lmin: int
    zeta_k: int


def encode(g: Graph, W: int = 7, R: int = 3, Lmin: int = 4, zeta_k: int = 3,
           stride: int = 65536, nthreads: int = 8) -> Encoded:
    """Encode adjacency lists into the project's BV-style bitstream."""
    lib = _load()
    rowptr = np.ascontiguousarray(g.rowptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    out = ctypes.POINTER(ctypes.c_uint8)()
    nb = ctypes.c_int64()
    refs = np.zeros(g.n, dtype=np.uint8)
    rc = lib.bvi_encode(g.n, rowptr.ctypes.data, col.ctypes.data, W, R, Lmin, zeta_k, stride, nthreads,
                        ctypes.byref(out), ctypes.byref(nb), refs.ctypes.data)
    if rc != 0:
        raise RuntimeError("bvi_encode failed (%d)" % rc)
    return Encoded(_take(out, nb.value, np.uint8), refs, W, R, Lmin, zeta_k)


def from_lists(lists) -> Graph:
    """CSR from a list of iterables of column ids (sorted, deduplicated here)."""
    rows = [np.unique(np.asarray(list(r), dtype=np.int64)) for r in lists]
    rp = np.zeros(len(rows) + 1, dtype=np.uint64)
    rp[1:] = np.cumsum([r.size for r in rows])
    col = np.concatenate(rows).astype(np.uint32) if rows and rp[-1] > 0 else np.zeros(0, np.uint32)
    return Graph(rp, col)


# ----------------------------------------------------------- structured graphs
def complete_graph(n: int) -> Graph:
    return from_lists([[j for j in range(n) if j != i] for i in range(n)])


def path_graph(n: int) -> Graph:
    """Directed path i -> i+1."""
    return from_lists([[i + 1] if i + 1 < n else [] for i in range(n)])


def cycle_graph(n: int) -> Graph:
    return from_lists([[(i + 1) % n] for i in range(n)])


def star_graph(n: int, center: int = 0, kind: str = "both") -> Graph:
    """kind: 'both' (centre <-> leaves), 'in' (leaves -> centre), 'out' (centre -> leaves)."""
    lists = [[] for _ in range(n)]
    leaves = [j for j in range(n) if j != center]
    if kind in ("both", "out"):
        lists[center] = leaves
    if kind in ("both", "in"):
        for j in leaves:
            lists[j] = [center]
    return from_lists(lists)


def empty_graph(n: int) -> Graph:
    return from_lists([[] for _ in range(n)])


# ------------------------------------------------------------------ vectors
def uniform_x(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    return np.random.default_rng(seed).random(n, dtype=np.dtype(dtype).type)


def integer_x(n: int, seed: int, hi: int, dtype=np.float64) -> np.ndarray:
    """Integers in [0, hi] stored as floating point (all partial sums exact)."""
    return np.random.default_rng(seed).integers(0, hi + 1, size=n).astype(dtype)


def teleport_sets(n: int, k: int, seeds_per_set: int, seed: int) -> np.ndarray:
    """k personalized-teleport vectors, node-major (n x k) float32, each with
    1/seeds_per_set on seeds_per_set distinct uniform random nodes."""
    rng = np.random.default_rng(seed)
    V = np.zeros((n, k), dtype=np.float32)
    for c in range(k):
        s = rng.choice(n, size=seeds_per_set, replace=False)
        V[s, c] = np.float32(1.0 / seeds_per_set)
    return V


# ------------------------------------------------------------------ workloads
WORKLOADS = {
    # tiny web-like copying model, one FP64 product
    "web-n1e4-d15": dict(kind="web", n=10_000, mean=15.0, seed=1),
    # web-like, n = 2^20, mean out-degree 20: product + PageRank
    "web-n2p20-d20": dict(kind="web", n=1 << 20, mean=20.0, seed=2),
    # social-like, n = 4e6, power-law out-degree (exponent 2.1, mean 40, max 50000), BFS order
    "social-n4e6-d40": dict(kind="social", n=4_000_000, mean=40.0, max_deg=50_000, exponent=2.1, seed=3),
    # web-like, n = 8e6, mean out-degree 25 (batched personalized PageRank)
    "web-n8e6-d25": dict(kind="web", n=8_000_000, mean=25.0, seed=4),
}


def workload_graph(name: str, n: int | None = None) -> Graph:
    """Graph of a named workload; `n` overrides the size (same recipe)."""
    w = dict(WORKLOADS[name])
    if n is not None:
        w["n"] = n
    if w["kind"] == "web":
        return web_graph(w["n"], w["mean"], w["seed"])
    return social_graph(w["n"], w["mean"], w["max_deg"], w["exponent"], w["seed"])


# ------------------------------------------------------------ column blocks
def column_blocks(g: Graph, nblocks: int):
    """Split g's columns into nblocks ranges of consecutive ids of (nearly)
    equal width: block b keeps, in every row, the ids in [c_b, c_{b+1}),
    c_b = floor(b n / nblocks).  Each block is an n-row graph with absolute
    column ids (encode it like any graph).  Returns (bounds, [Graph])."""
    n = g.n
    bounds = [(b * n) // nblocks for b in range(nblocks + 1)]
    col = np.asarray(g.col, dtype=np.int64)
    rowid = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.rowptr.astype(np.int64)))
    out = []
    for b in range(nblocks):
        keep = (col >= bounds[b]) & (col < bounds[b + 1])
        cnt = np.bincount(rowid[keep], minlength=n)
        rp = np.zeros(n + 1, dtype=np.uint64)
        np.cumsum(cnt, out=rp[1:])
        out.append(Graph(rp, g.col[keep].copy()))
    return bounds, out


# ----------------------------------------------------- biclique decomposition
@dataclass
class Bicliques:
    """Edges of an n-node graph as bicliques plus residual edges (the input of
    the biclique product).  Biclique r: every node of S_r =
    sidx[sptr[r]:sptr[r+1]] points to every node of C_r =
    cidx[cptr[r]:cptr[r+1]] (both ascending); residual edges as CSR (rptr
    n+1, rcol ascending per row).  Every edge lies in exactly one biclique or
    in the residual."""
    n: int
    sptr: np.ndarray
    sidx: np.ndarray
    cptr: np.ndarray
    cidx: np.ndarray
    rptr: np.ndarray
    rcol: np.ndarray

    @property
    def nbic(self) -> int:
        return int(self.sptr.shape[0] - 1)

    def words(self) -> int:
        """Stored ids: sum |S_r| + |C_r| over bicliques, plus residual edges."""
        return int(self.sidx.size + self.cidx.size + self.rcol.size)

    def biclique(self, r: int):
        return (self.sidx[int(self.sptr[r]):int(self.sptr[r + 1])],
                self.cidx[int(self.cptr[r]):int(self.cptr[r + 1])])


def biclique_mine(g: Graph, window: int = 8, cmin: int = 2, block: int = 4096, nthreads: int = 8) -> Bicliques:
    """Greedy biclique decomposition of g (see biclique.c): rows seed
    bicliques grown from the next `window` rows while |S||C| - |S| - |C|
    grows; independent blocks of `block` rows."""
    lib = _load()
    rowptr = np.ascontiguousarray(g.rowptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    nb = ctypes.c_int64()
    ptrs = [ctypes.POINTER(ctypes.c_uint64)(), ctypes.POINTER(ctypes.c_uint32)(),
            ctypes.POINTER(ctypes.c_uint64)(), ctypes.POINTER(ctypes.c_uint32)(),
            ctypes.POINTER(ctypes.c_uint64)(), ctypes.POINTER(ctypes.c_uint32)()]
    rc = lib.bvi_biclique_mine(g.n, rowptr.ctypes.data, col.ctypes.data, window, cmin, block, nthreads,
                               ctypes.byref(nb), *[ctypes.byref(p) for p in ptrs])
    if rc != 0:
        raise RuntimeError("bvi_biclique_mine failed (%d)" % rc)
    sptr = _take(ptrs[0], nb.value + 1, np.uint64)
    cptr = _take(ptrs[2], nb.value + 1, np.uint64)
    rptr = _take(ptrs[4], g.n + 1, np.uint64)
    return Bicliques(g.n, sptr, _take(ptrs[1], int(sptr[-1]), np.uint32), cptr,
                     _take(ptrs[3], int(cptr[-1]), np.uint32), rptr, _take(ptrs[5], int(rptr[-1]), np.uint32))


def planted_bicliques(n: int, nbic: int, s_range=(2, 8), c_range=(2, 16), res_mean: float = 3.0, seed: int = 0,
                      spread: int = 4):
    """A graph built from planted bicliques plus residual edges, and that
    decomposition.  Biclique r: |S_r|, |C_r| uniform in the given ranges,
    each set a sample of distinct ids from a range of `spread` times its size
    at a uniform offset; a column that one of S_r's rows already points to
    is dropped from C_r (the edges stay a partition), and a biclique left
    with no column is dropped.  Residual: 1 + Poisson(res_mean - 1) targets
    per node near it (geometric gaps, mean 8), edges already present
    skipped.  For small n (Python loops).  Returns (Graph, Bicliques)."""
    rng = np.random.default_rng(seed)
    rows = [set() for _ in range(n)]
    S_l, C_l = [], []
    for _ in range(nbic):
        s = int(rng.integers(s_range[0], s_range[1] + 1))
        c = int(rng.integers(c_range[0], c_range[1] + 1))
        s, c = min(s, n), min(c, n)
        a = int(rng.integers(0, max(1, n - spread * s + 1)))
        b = int(rng.integers(0, max(1, n - spread * c + 1)))
        S = np.sort(rng.choice(np.arange(a, min(n, a + spread * s)), size=s, replace=False))
        C = np.sort(rng.choice(np.arange(b, min(n, b + spread * c)), size=c, replace=False))
        C = np.array([j for j in C if all(int(j) not in rows[int(i)] for i in S)], dtype=np.int64)
        if C.size == 0:
            continue
        for i in S:
            rows[int(i)].update(int(j) for j in C)
        S_l.append(S)
        C_l.append(C)
    res = [[] for _ in range(n)]
    for i in range(n):
        k = 1 + int(rng.poisson(max(res_mean - 1.0, 0.0))) if res_mean > 0 else 0
        j = i - 12 + int(rng.geometric(1.0 / 8.0))
        for _ in range(k):
            jj = j % n
            if jj not in rows[i]:
                rows[i].add(jj)
                res[i].append(jj)
            j += int(rng.geometric(1.0 / 8.0))
    g = from_lists([sorted(r) for r in rows])
    cnt = lambda L: np.concatenate([[0], np.cumsum([len(x) for x in L])]).astype(np.uint64)
    cat = lambda L: (np.concatenate(L) if L else np.zeros(0)).astype(np.uint32)
    res = [sorted(r) for r in res]
    return g, Bicliques(n, cnt(S_l), cat(S_l), cnt(C_l), cat(C_l), cnt(res),
                        cat([np.asarray(r, dtype=np.int64) for r in res]))


# ------------------------------------------------------- network parameters
MLP_SHAPES = [("W1", (64, 12)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("w3", (64,)), ("b3", (1,))]


def mlp_init_params(seed: int) -> np.ndarray:
    """Seeded starting parameters of the 12 -> 64 -> 64 -> 1 warm-restart
    network, in the library's parameter order (W1 row-major (out, in), b1,
    W2, b2, w3, b3): weights uniform on [-a, a] with a = sqrt(6 / (fan_in +
    fan_out)) (Glorot) drawn from numpy's default_rng(seed) in that order,
    biases zero, rounded to float32.  Returned as float32 (5057 values)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in MLP_SHAPES:
        if name[0] == "b":
            parts.append(np.zeros(int(np.prod(shape))))
        else:
            fo, fi = shape if len(shape) == 2 else (1, shape[0])
            a = (6.0 / (fi + fo)) ** 0.5
            parts.append(rng.uniform(-a, a, size=shape).reshape(-1))
    return np.concatenate(parts).astype(np.float32)


def ragged_sizes(count: int = 48, seed: int = 999, lo_exp: float = 4.0, hi_exp: float = 6.0):
    """Graph sizes log-uniform in [10^lo_exp, 10^hi_exp]."""
    u = np.random.default_rng(seed).random(count)
    return [int(round(10 ** (lo_exp + (hi_exp - lo_exp) * v))) for v in u]
