"""CPU tier for the native library: it loads, exports every symbol the header
declares, its host decoder matches the generator's lists and the
hand-written stream, and the device layout (interpreted on the host) gives
the oracle's product.  No compute call touches a device here."""
import os
import re

import numpy as np
import pytest

import bvinputs as B
from oracle import product
from tests.golden_io import pack_stream, read_tiny_stream

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_1708_07271_amd as mod
    mod.load_library()
    return mod


def test_exports_every_declared_symbol(P):
    lib = P.load_library()
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            names |= set(re.findall(r"^\s*(?:[\w\*]+\s+)+\**(bvmv_\w+)\s*\(", text, flags=re.M))
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_decode_golden_stream(P):
    data, lists, refs = read_tiny_stream()
    rowptr, col, got_refs = P.bvmv_decode(data)
    for i, L in enumerate(lists):
        assert col[int(rowptr[i]):int(rowptr[i + 1])].tolist() == L
    assert got_refs.tolist() == refs


@pytest.mark.parametrize("nthreads", [1, 4])
def test_decode_matches_generator(P, nthreads):
    for g in (B.web_graph(150_000, 20.0, 31), B.social_graph(60_000, 20.0, 5000, 2.1, 32)):
        enc = B.encode(g, stride=4096)
        rowptr, col, refs = P.bvmv_decode(enc.data, nthreads=nthreads)
        assert np.array_equal(rowptr, g.rowptr)
        assert np.array_equal(col, g.col)
        assert np.array_equal(refs, enc.refs)


def test_decode_rejects_corruption(P):
    g = B.web_graph(3000, 12.0, 3)
    data = B.encode(g, stride=512).data
    for bad in (data[:100], data[: len(data) - 9]):
        with pytest.raises(P.BvmvError) as ei:
            P.bvmv_decode(bad)
        assert ei.value.code == P.BVMV_EFORMAT
    bad = data.copy()
    bad[16] ^= 4                                  # header edge count
    with pytest.raises(P.BvmvError):
        P.bvmv_decode(bad)
    bad = data.copy()
    bad[64 + 8] ^= 1                              # second segment offset
    with pytest.raises(P.BvmvError):
        P.bvmv_decode(bad)
    # node 1 referencing 2 rows back
    with pytest.raises(P.BvmvError):
        P.bvmv_decode(pack_stream(2, 2, 7, 3, 4, 3, "010" + "1" + "110" + "010" + "001"))
    # flipped body bits must never crash: either an error or a consistent graph
    rng = np.random.default_rng(0)
    body0 = 64 + 8 * ((g.n + 511) // 512)
    for _ in range(40):
        bad = data.copy()
        pos = int(rng.integers(body0, len(data)))
        bad[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        try:
            rp, col, _ = P.bvmv_decode(bad)
            assert rp[-1] == col.size and np.all(col < g.n)
        except P.BvmvError as e:
            assert e.code == P.BVMV_EFORMAT


LAYOUT_CASES = [(64, 1024, 4096, 2048), (16, 64, 512, 16), (64, 8191, 16384, 16384), (32, 256, 1024, 40)]


@pytest.mark.parametrize("tile_rows,window_cap,stage,long_bytes", LAYOUT_CASES)
def test_layout_interpreter_matches_oracle(P, tile_rows, window_cap, stage, long_bytes):
    graphs = [B.web_graph(30_000, 20.0, 41), B.social_graph(20_000, 30.0, 3000, 2.1, 42)]
    for g in graphs:
        enc = B.encode(g)
        x = B.integer_x(g.n, 7, 1000)
        y, st = P.bvmv_layout_selfcheck(enc.data, x, tile_rows, window_cap, stage, long_bytes)
        assert np.array_equal(y, product.matvec(g.rowptr, g.col, x))
        assert st["max_level"] <= 3
        x = B.uniform_x(g.n, 8)
        y, _ = P.bvmv_layout_selfcheck(enc.data, x, tile_rows, window_cap, stage, long_bytes)
        y0 = product.matvec(g.rowptr, g.col, x)
        assert np.max(np.abs(y - y0) / np.maximum(y0, 1e-300)) < 1e-12


def test_layout_crafted_edge_cases(P):
    n = 5000
    rng = np.random.default_rng(5)
    lists = [[] for _ in range(n)]
    lists[0] = [n - 1]
    lists[1] = list(range(0, 300))                     # long interval from 0
    lists[2] = list(range(0, 300))                     # identical to its reference
    lists[3] = [2, 3]                                  # reference almost fully skipped
    lists[4] = [4]                                     # self-loop
    lists[5] = sorted(rng.choice(n, 4000, replace=False).tolist())   # long random row
    lists[6] = sorted(set(lists[5][:3900]) | {n - 1})  # reuses a long row
    lists[n - 1] = list(range(n - 20, n))              # interval touching n-1
    g = B.from_lists(lists)
    enc = B.encode(g)
    x = B.integer_x(n, 1, 1000)
    for case in LAYOUT_CASES:
        y, _ = P.bvmv_layout_selfcheck(enc.data, x, *case)
        assert np.array_equal(y, product.matvec(g.rowptr, g.col, x))


def _chunk_index(a, C, rcp_offset):
    """The tile kernel's chunk index of an entry offset a: floor of one fused
    multiply-add (a + 1/2) * r in single precision, r = 1/C rounded to single
    precision and moved by rcp_offset ulps (the hardware reciprocal is within
    1 ulp).  The product is formed in double (exact to far below the margin)
    and rounded once to single."""
    r = np.float32(1.0 / C)
    r = np.nextafter(r, np.float32(np.inf if rcp_offset > 0 else -np.inf), dtype=np.float32) if rcp_offset else r
    v = (a.astype(np.float64) + 0.5) * np.float64(r)
    return np.floor(v.astype(np.float32)).astype(np.int64)


@pytest.mark.parametrize("C", list(range(1, 131)) + [255, 1000, 4096, 16383])
def test_chunk_index_formula_is_exact(C):
    """floor((a + 1/2) r) = a // C for every entry offset a < 64 C of a flat
    pass, whichever way the reciprocal rounds: (a + 1/2) / C stays at least
    1 / (2C) from every integer, far beyond the single-precision error."""
    a = np.arange(64 * C, dtype=np.int64)
    for off in (-1, 0, 1):
        assert np.array_equal(_chunk_index(a, C, off), a // C), (C, off)


def test_bench_refuses_several_gpus():
    """bench.py is single-GPU: --gpus 2 exits with status 2 and a message,
    before any device work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env=dict(os.environ, WORLD_SIZE="1"))
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_host_decode_and_layout_under_sanitizers(tmp_path):
    """The host decoder, layout builder and layout interpreter built with
    AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only) and
    run on generator graphs, crafted edge cases and damaged streams
    (tests/native/sanitize_host.cpp)."""
    import shutil
    import subprocess
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    csrc = os.path.join(root, "paper_1708_07271_amd", "csrc")
    exe = str(tmp_path / "sanitize_host")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", csrc, "-I", os.path.join(root, "include"),
           os.path.join(root, "tests", "native", "sanitize_host.cpp"), os.path.join(csrc, "bv_decode.cpp"),
           os.path.join(csrc, "bv_layout.cpp"), os.path.join(csrc, "bv_layout_check.cpp"), "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    rng = np.random.default_rng(3)
    graphs = [B.web_graph(3000, 15.0, 91), B.social_graph(2000, 20.0, 1500, 2.1, 92), B.empty_graph(1),
              B.empty_graph(300), B.complete_graph(40), B.from_lists([[0], [0, 1], [1, 2]])]
    n = 6000
    lists = [[] for _ in range(n)]
    lists[1] = list(range(0, 300))
    lists[2] = list(range(0, 300))
    lists[5] = sorted(rng.choice(n, 5000, replace=False).tolist())
    lists[6] = sorted(set(lists[5][:4500]) | {n - 1})
    lists[n - 1] = list(range(n - 20, n))
    for i in range(100, 140):
        lists[i] = sorted(({0, i, i - 50, n - 1} | set(range(i + 5, i + 30))) - {i - 1})
    graphs.append(B.from_lists(lists))
    files = []
    for k, g in enumerate(graphs):
        for W, R, stride in ((7, 3, 64), (1, 1, 65536), (15, 0, 7)):
            f = tmp_path / ("g%d_w%d_r%d.bv" % (k, W, R))
            f.write_bytes(bytes(B.encode(g, W=W, R=R, stride=stride).data))
            files.append(str(f))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe] + files, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.startswith("ok %d" % len(files))


def test_api_rejects_bad_arguments_before_device_work(P):
    """Every argument check that precedes device work answers BVMV_EINVAL with
    a message, also on a machine without a GPU: null handles and buffers,
    load options out of range, malformed host CSR arrays (offsets that do not
    start at 0 or decrease, which would make a row length wrap; column ids out
    of range), empty groups, a null network."""
    import ctypes
    lib = P.load_library()
    h = ctypes.c_void_p()
    data = np.frombuffer(bytes(B.encode(B.web_graph(200, 5.0, 1)).data), dtype=np.uint8)

    def einval(rc, text):
        assert rc == P.BVMV_EINVAL, (rc, text)
        msg = lib.bvmv_last_error().decode()
        assert text in msg, (text, msg)

    einval(lib.bvmv_load(None, 0, None, ctypes.byref(h)), "null argument")
    for field, bad in (("tile_rows", 7), ("tile_rows", 129), ("window_cap", 63), ("window_cap", 8192),
                       ("stage_bytes", 511), ("stage_bytes", 16385), ("long_row_bytes", 15),
                       ("long_row_bytes", 5000), ("interval_mode", 2), ("interval_mode", -1), ("device", -1)):
        with pytest.raises(P.BvmvError) as e:
            P.bvmv_load(data, **{field: bad})
        assert e.value.code == P.BVMV_EINVAL and "load option out of range" in str(e.value), field
    einval(lib.bvmv_multiply(None, None, None, 0, None), "null argument")
    einval(lib.bvmv_multiply_batch(None, None, None, 1, 1, 0, None), "null argument")
    einval(lib.bvmv_pagerank(None, None, None, None, None, 1, None, None), "null argument")
    einval(lib.bvmv_degrees(None, None, None), "null argument")
    einval(lib.bvmv_group(None, 0, ctypes.byref(h)), "bad group arguments")
    einval(lib.bvmv_csr_create(None, ctypes.byref(h)), "null argument")
    einval(lib.bvmv_csr_multiply(None, None, None, 0, None), "null argument")
    einval(lib.bvmv_csr_pagerank(None, None, None, None, None, None, None), "null argument")
    einval(lib.bvmv_features(None, None, None), "null argument")
    einval(lib.bvmv_restart_sample(None, 10, 0, None, None, None, None, None), "null argument")
    einval(lib.bvmv_mlp_create(0, None, ctypes.byref(h)), "null argument")
    einval(lib.bvmv_mlp_forward(None, None, 1, None, None), "bad network arguments")
    einval(lib.bvmv_mlp_gradient(None, None, None, 1, None, None), "bad network arguments")

    def csr(rowptr, col, text):
        rp = np.ascontiguousarray(rowptr, dtype=np.uint64)
        c = np.ascontiguousarray(col if len(col) else [0], dtype=np.uint32)
        einval(lib.bvmv_csr_create_host(rp.size - 1, rp.ctypes.data, c.ctypes.data, 0, ctypes.byref(h)), text)
        assert h.value is None

    csr([0], [], "bad CSR arguments")                        # n = 0
    csr([1, 2, 3], [0, 1, 0], "rowptr[0] must be 0")
    csr([0, 5, 3], [0, 1, 0, 1, 0], "rowptr must be nondecreasing")
    csr([0, 2, 1, 4], [0, 1, 2, 0], "rowptr must be nondecreasing")
    csr([0, 1, 2], [0, 7], "column out of range")
    einval(lib.bvmv_csr_create_host(2, None, None, 0, ctypes.byref(h)), "bad CSR arguments")
    rp = np.array([0, 1, 1], dtype=np.uint64)
    einval(lib.bvmv_csr_create_host(2, rp.ctypes.data, None, 0, ctypes.byref(h)), "bad CSR arguments")


def test_layout_property_random_graphs(P):
    """Property test: for random small graphs (row lengths from empty to dense,
    clustered or scattered ids, runs that become intervals, rows copied from
    earlier rows), random encoder settings and random tile / window / stage
    shapes, the host interpreter of the device layout gives the oracle's
    product exactly on integer x, and the host decoder gives the lists back."""
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies

    @st.composite
    def graph_case(draw):
        n = draw(st.integers(1, 400))
        seed = draw(st.integers(0, 2**31 - 1))
        rng = np.random.default_rng(seed)
        lists = []
        for i in range(n):
            kind = draw(st.sampled_from(["empty", "near", "far", "run", "copy", "dense"]))
            if kind == "empty":
                row = []
            elif kind == "near":
                row = (i + rng.integers(-20, 21, rng.integers(1, 12))) % n
            elif kind == "far":
                row = rng.integers(0, n, rng.integers(1, 30))
            elif kind == "run":
                s = int(rng.integers(0, n))
                row = list(range(s, min(n, s + int(rng.integers(1, 60)))))
            elif kind == "copy" and lists:
                src = lists[max(0, i - int(rng.integers(1, 9)))]
                keep = [c for c in src if rng.random() < 0.8]
                row = keep + list(rng.integers(0, n, rng.integers(0, 4)))
            else:
                row = rng.choice(n, min(n, int(rng.integers(1, 400))), replace=False)
            lists.append(sorted(set(int(c) for c in row)))
        enc = dict(W=draw(st.integers(0, 15)), R=draw(st.integers(0, 15)), Lmin=draw(st.integers(2, 8)),
                   zeta_k=draw(st.integers(1, 5)), stride=draw(st.sampled_from([7, 64, 65536])))
        stage = draw(st.sampled_from([512, 1024, 4096, 16384]))
        lay = (draw(st.sampled_from([8, 16, 32, 64, 96, 128])), draw(st.integers(64, 1024)), stage,
               draw(st.integers(16, stage)))
        return lists, enc, lay

    @hyp.settings(max_examples=150, deadline=None, database=None, derandomize=True)
    @hyp.given(graph_case())
    def check(case):
        lists, enc_opts, lay = case
        g = B.from_lists(lists)
        enc = B.encode(g, **enc_opts)
        rowptr, col, _ = P.bvmv_decode(enc.data)
        assert np.array_equal(rowptr, g.rowptr) and np.array_equal(col, g.col)
        x = B.integer_x(g.n, 3, 1000)
        y, info = P.bvmv_layout_selfcheck(enc.data, x, *lay)
        assert np.array_equal(y, product.matvec(g.rowptr, g.col, x)), (enc_opts, lay)
        assert info["max_level"] <= max(enc_opts["R"], 0)

    check()


def test_missing_library_fails_loudly():
    """With the native library absent, every entry point raises instead of
    computing anything, and the package never loads the oracle (there is no
    CPU fallback).  Run in a child process so that this process keeps its
    loaded library."""
    import subprocess
    import sys
    code = "\n".join([
        "import sys, numpy as np",
        "import paper_1708_07271_amd as P",
        "P.LIB_PATH = '/nonexistent/libbvmv.so'",
        "calls = [lambda: P.load_library(), lambda: P.bvmv_load(np.zeros(64, np.uint8)),",
        "         lambda: P.bvmv_decode(np.zeros(64, np.uint8)), lambda: P.bvmv_csr_create_host([0, 0], [])]",
        "for f in calls:",
        "    try:",
        "        f()",
        "    except ImportError as e:",
        "        assert 'not built' in str(e), e",
        "    else:",
        "        raise SystemExit('an entry point ran without the library')",
        "assert not any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules), 'oracle imported'",
        "print('ok')",
    ])
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:], r.stderr[-2000:])
