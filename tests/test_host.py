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


def _gamma_bits(x):
    """Elias gamma of x + 1 (the format's gamma code of x)."""
    b = (x + 1).bit_length() - 1
    return "0" * b + format(x + 1, "b")


def _zeta_bits(x, k):
    """zeta_k of x + 1: unary bucket h, then the value's offset in the bucket
    [2^(hk), 2^((h+1)k)) in minimal binary."""
    v = x + 1
    h = 0
    while v >= 1 << ((h + 1) * k):
        h += 1
    left = 1 << (h * k)
    zmax = (1 << ((h + 1) * k)) - left
    z = v - left
    s = (zmax - 1).bit_length()
    thr = (1 << s) - zmax
    return "0" * h + "1" + (format(z, "0%db" % (s - 1)) if z < thr else format(z + thr, "0%db" % s))


def _hostile_bodies():
    """Bodies of an 8-node stream (W = 0, L_min = 4, zeta_3) whose node 0
    decodes a value near 2^64 where a length, a gap or a start is expected."""
    huge = (1 << 64) - 2           # the largest gamma value
    zhuge = (1 << 63) - 2           # a zeta_3 value in the last bucket
    return [
        # 10 entries, one interval of length L_min + huge (wraps to a small length unchecked)
        _gamma_bits(10) + _gamma_bits(1) + _gamma_bits(0) + _gamma_bits(huge),
        # one interval whose start offset is huge
        _gamma_bits(10) + _gamma_bits(1) + _gamma_bits(huge) + _gamma_bits(0),
        # two intervals, the second's gap huge
        _gamma_bits(10) + _gamma_bits(2) + _gamma_bits(0) + _gamma_bits(0) + _gamma_bits(huge) + _gamma_bits(0),
        # two residuals, the second's gap huge (prev + 1 + gap would overflow)
        _gamma_bits(2) + _zeta_bits(0, 3) + _zeta_bits(zhuge, 3),
        # a first residual at a huge signed offset
        _gamma_bits(2) + _zeta_bits(zhuge, 3) + _zeta_bits(0, 3),
    ]


def test_zeta_bits_helper_decodes():
    # the test's own encoder of hostile streams, checked against the oracle decoder's reader
    from oracle import bvdecode
    for x in (0, 1, 6, 7, 8, 100, 4095, 123456, (1 << 40) + 3):
        bits = _zeta_bits(x, 3) + _gamma_bits(x)
        br = bvdecode.BitReader(int(bits + "0" * (-len(bits) % 8), 2).to_bytes((len(bits) + 7) // 8, "big"),
                                len(bits))
        assert br.zeta(3) == x and br.gamma() == x


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
    for k, bits in enumerate(_hostile_bodies()):
        f = tmp_path / ("hostile%d.bv" % k)
        f.write_bytes(bytes(pack_stream(8, 12, 0, 0, 4, 3, bits)))
        files.append("reject:" + str(f))
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


def _twosum_lib(tmp_path):
    import ctypes
    import shutil
    import subprocess
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    so = str(tmp_path / "twosum_host.so")
    subprocess.run(["g++", "-std=c++17", "-O2", "-shared", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
                    "-msse2", "-mfpmath=sse", "-I", os.path.join(root, "paper_1708_07271_amd", "csrc"),
                    os.path.join(root, "tests", "native", "twosum_host.cpp"), "-o", so], check=True, timeout=300)
    lib = ctypes.CDLL(so)
    return lib


def _f32_cases(rng, n):
    """Float pairs over many binades, with exact ties, heavy cancellation and
    operands far apart in magnitude."""
    e = rng.integers(-40, 40, size=(n, 2))
    m = rng.random((n, 2)) + 0.5
    v = (np.where(rng.random((n, 2)) < 0.5, -1.0, 1.0) * m * np.exp2(e)).astype(np.float32)
    hard = np.array([[1.0, 2.0 ** -24], [1.0, 3 * 2.0 ** -25], [1.0, -1.0 + 2.0 ** -24], [3 * 2.0 ** 100, 2.0 ** -100],
                     [-2.0 ** 30, 2.0 ** 30 + 1.0], [1e-38, -1e-38 * 0.75], [0.0, 0.0], [65504.0, 2.0 ** -14]],
                    dtype=np.float32)
    near = v[:, :1] * (1 + np.float32(2.0 ** -20) * rng.integers(-8, 8, size=(n, 1))).astype(np.float32)
    return np.concatenate([v, hard, np.concatenate([v[:, :1], -near], axis=1)]).astype(np.float32)


def test_two_sum_exact(tmp_path):
    """O7: TwoSum as the device code computes it (twosum.hpp built for the
    host): s is the rounded float sum and s + e equals a + b exactly, checked
    in rational arithmetic."""
    import ctypes
    from fractions import Fraction
    lib = _twosum_lib(tmp_path)
    v = _f32_cases(np.random.default_rng(17), 3000)
    a, b = np.ascontiguousarray(v[:, 0]), np.ascontiguousarray(v[:, 1])
    s, e = np.empty_like(a), np.empty_like(a)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.host_two_sum(a.ctypes.data_as(fp), b.ctypes.data_as(fp), s.ctypes.data_as(fp), e.ctypes.data_as(fp),
                     len(a))
    assert np.array_equal(s, a + b)             # numpy float32 addition rounds to nearest as well
    for i in range(len(a)):
        assert Fraction(float(s[i])) + Fraction(float(e[i])) == Fraction(float(a[i])) + Fraction(float(b[i])), i


def test_pair_add_error_bound(tmp_path):
    """pair_add on normalised pairs (|lo| <= ulp(hi)/2): the result is
    normalised, and hi + lo is within 4 u^2 (|a| + |b|) of the exact sum of
    the four parts (u = 2^-24), in rational arithmetic."""
    import ctypes
    from fractions import Fraction
    lib = _twosum_lib(tmp_path)
    rng = np.random.default_rng(18)
    v = _f32_cases(rng, 2000)
    hi = v.astype(np.float32)
    lo = (hi.astype(np.float64) * (rng.random(hi.shape) - 0.5) * 2.0 ** -24).astype(np.float32)
    lo = np.where((hi + lo) == hi, lo, np.float32(0))                     # keep the pairs normalised
    ah, al, bh, bl = (np.ascontiguousarray(t) for t in (hi[:, 0], lo[:, 0], hi[:, 1], lo[:, 1]))
    h, l = np.empty_like(ah), np.empty_like(ah)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.host_pair_add(ah.ctypes.data_as(fp), al.ctypes.data_as(fp), bh.ctypes.data_as(fp), bl.ctypes.data_as(fp),
                      h.ctypes.data_as(fp), l.ctypes.data_as(fp), len(ah))
    assert np.array_equal(h + l, h)
    u2 = Fraction(1, 2 ** 48)
    for i in range(len(ah)):
        exact = sum(Fraction(float(t[i])) for t in (ah, al, bh, bl))
        err = abs(Fraction(float(h[i])) + Fraction(float(l[i])) - exact)
        assert err <= 4 * u2 * (abs(Fraction(float(ah[i]))) + abs(Fraction(float(bh[i])))), i


def test_kernel_index_replay(tmp_path):
    """Every global index the tile kernel computes (stream rounds, row-end
    counts, window loads, Z indices, gathered wide and long columns), replayed
    on the host over every tile and lane of layouts in six shapes, stays
    inside the device arrays (tests/native/index_replay.cpp): the bench's
    2^20-node graph, the property-test families and crafted edge cases."""
    import shutil
    import subprocess
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    csrc = os.path.join(root, "paper_1708_07271_amd", "csrc")
    exe = str(tmp_path / "index_replay")
    subprocess.run(["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", csrc,
                    "-I", os.path.join(root, "include"), os.path.join(root, "tests", "native", "index_replay.cpp"),
                    os.path.join(csrc, "bv_decode.cpp"), os.path.join(csrc, "bv_layout.cpp"), "-lpthread", "-o", exe],
                   check=True, timeout=600)
    rng = np.random.default_rng(21)
    graphs = [B.workload_graph("web-n2p20-d20"), B.web_graph(5000, 15.0, 22), B.social_graph(4000, 30.0, 3000, 2.1, 23),
              B.empty_graph(1), B.empty_graph(77), B.complete_graph(300), B.star_graph(5000, 17, "both")]
    n = 3000
    lists = [sorted(rng.choice(n, int(rng.integers(0, 60)), replace=False).tolist()) for _ in range(n)]
    lists[n - 1] = list(range(n))
    graphs.append(B.from_lists(lists))
    files = []
    for k, g in enumerate(graphs):
        for W, R in ((7, 3), (1, 15), (15, 1)):
            f = tmp_path / ("g%d_%d_%d.bv" % (k, W, R))
            f.write_bytes(bytes(B.encode(g, W=W, R=R).data))
            files.append(str(f))
            if k == 0:
                break
    r = subprocess.run([exe] + files, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert r.stdout.startswith("ok")


def test_biclique_load_rejects_bad_decompositions():
    """bvmv_biclique_load validates on the host before any device work: an
    edge listed twice, unsorted or out-of-range ids and bad offsets give
    BVMV_EFORMAT; a null argument BVMV_EINVAL."""
    import paper_1708_07271_amd as P
    g, b = B.planted_bicliques(300, 30, seed=11)

    def bad(**kw):
        d = dict(n=b.n, sptr=b.sptr.copy(), sidx=b.sidx.copy(), cptr=b.cptr.copy(), cidx=b.cidx.copy(),
                 rptr=b.rptr.copy(), rcol=b.rcol.copy())
        d.update(kw)
        with pytest.raises(P.BvmvError) as e:
            P.bvmv_biclique_load(B.Bicliques(**d))
        return e.value.code

    S0, C0 = b.biclique(0)
    # the residual repeats an edge of biclique 0
    i, j = int(S0[0]), int(C0[0])
    rows = [list(b.rcol[int(b.rptr[k]):int(b.rptr[k + 1])]) for k in range(b.n)]
    rows[i] = sorted(set(rows[i]) | {j})
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.uint64)
    rc = np.asarray([v for r in rows for v in r], np.uint32)
    assert bad(rptr=rp, rcol=rc) == P.BVMV_EFORMAT
    cidx = b.cidx.copy()
    cidx[int(b.cptr[0])] = b.n  # out of range
    assert bad(cidx=cidx) == P.BVMV_EFORMAT
    if C0.size >= 2:
        cidx = b.cidx.copy()
        a = int(b.cptr[0])
        cidx[a], cidx[a + 1] = cidx[a + 1], cidx[a]  # unsorted
        assert bad(cidx=cidx) == P.BVMV_EFORMAT
    sptr = b.sptr.copy()
    sptr[1] = sptr[2] + 1  # decreasing offsets
    assert bad(sptr=sptr) == P.BVMV_EFORMAT


@pytest.mark.parametrize("case", range(5))
def test_left_layout_interpreter(case):
    """The left product's column-wise layout, interpreted on the host as the
    two device passes read it (bvmv_left_selfcheck): x A exactly for integer
    x, and within the left product's tolerance (per entry 1e-12 relative plus
    2^-48 of the largest entry: a column's terms cancel where a row skips an
    entry of its reference row) for uniform x; on web-like and social-like
    graphs, 128-row tiles with wide windows, intervals summed entry by entry,
    and long rows (whose entries all leave the windows)."""
    import paper_1708_07271_amd as P
    from oracle import product
    from tests import tolerances as TOL
    g, kw = [(B.web_graph(20000, 15.0, 5), {}), (B.social_graph(20000, 40.0, 5000, 2.1, 6), {}),
             (B.web_graph(5000, 12.0, 7), dict(tile_rows=128, window_cap=512)),
             (B.web_graph(5000, 12.0, 8), dict(interval_mode=1)),
             (B.web_graph(3000, 30.0, 9), dict(long_row_bytes=40))][case]
    enc = B.encode(g)
    xi = B.integer_x(g.n, 3, 1000)
    assert np.array_equal(P.bvmv_left_selfcheck(enc.data, xi, **kw), product.left_matvec(g.rowptr, g.col, xi))
    x = B.uniform_x(g.n, 4)
    ratio, _ = TOL.within(P.bvmv_left_selfcheck(enc.data, x, **kw), product.left_matvec_exact(g.rowptr, g.col, x),
                          TOL.F64, TOL.FLOOR["f64"])
    assert ratio <= 1.0
