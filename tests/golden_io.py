"""Readers for the hand-written fixtures under tests/golden/."""
import os
import struct

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_codes():
    rows = []
    with open(os.path.join(GOLDEN, "codes.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, k, x, bits = line.split()
            rows.append((kind, int(k), int(x), bits))
    return rows


def pack_stream(n, m, W, R, Lmin, zk, bitstr, stride=0, seg_offsets=()):
    """Header + MSB-first body assembled from a '0'/'1' string."""
    nbits = len(bitstr)
    padded = bitstr + "0" * ((-nbits) % 64)
    body = int(padded, 2).to_bytes(len(padded) // 8, "big") if padded else b""
    hdr = b"BVMV" + struct.pack("<IQQIIIIIIQQ", 1, n, m, W, R, Lmin, zk, stride, 0, nbits, len(seg_offsets))
    hdr += b"".join(struct.pack("<Q", o) for o in seg_offsets)
    return np.frombuffer(hdr + body, dtype=np.uint8).copy()


def read_tiny_stream():
    params, bits, lists, refs = {}, {}, {}, {}
    with open(os.path.join(GOLDEN, "tiny_bv_stream.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "param":
                params[tok[1]] = int(tok[2])
            elif tok[0] == "bits":
                bits[int(tok[1])] = "".join(tok[2:])
            elif tok[0] == "list":
                lists[int(tok[1])] = [int(t) for t in tok[2:]]
            elif tok[0] == "ref":
                refs[int(tok[1])] = int(tok[2])
    n = len(lists)
    bitstr = "".join(bits[i] for i in range(n))
    m = sum(len(v) for v in lists.values())
    data = pack_stream(n, m, params["W"], params["R"], params["Lmin"], params["zeta_k"], bitstr)
    return data, [lists[i] for i in range(n)], [refs[i] for i in range(n)]
