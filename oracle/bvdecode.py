"""Oracle decoder of the project's BV-style bitstream (pure Python + numpy).

TEST INFRASTRUCTURE: this package is the CPU oracle.  Only tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never does.

The bitstream realises list referencing as the paper describes it (Section
"Our Approach"): row i is represented against a reference row r_i < i taken
within a window W, by marking which of the reference's entries are kept
(copy blocks) and which are spurious (skip blocks), and by adding the missing
entries, coded with differential compression and codes for natural numbers.
The codes themselves follow their published definitions: unary; Elias gamma;
Boldi-Vigna zeta_k.  Field order and header are this project's own.

Header (little endian, 64 bytes): "BVMV", u32 version, u64 n, u64 m, u32 W,
u32 R, u32 Lmin, u32 zeta_k, u32 stride, u32 0, u64 body_bits, u64 nseg; then
nseg u64 bit offsets of nodes 0, S, 2S, ... (S = stride); then the MSB-first
body.  With a segment table a reference never crosses a multiple of S.
"""
from __future__ import annotations

import struct

import numpy as np


class FormatError(ValueError):
    pass


class BitReader:
    """MSB-first bit reader over a numpy bit array."""

    def __init__(self, body: bytes, nbits: int):
        self.bits = np.unpackbits(np.frombuffer(body, dtype=np.uint8))[:nbits]
        self.ones = np.flatnonzero(self.bits)
        self.nbits = nbits
        self.pos = 0

    def read_bits(self, k: int) -> int:
        if k == 0:
            return 0
        if self.pos + k > self.nbits:
            raise FormatError("read past end of body")
        v = 0
        for b in self.bits[self.pos:self.pos + k]:
            v = (v << 1) | int(b)
        self.pos += k
        return v

    def unary(self) -> int:
        """Number of zeros before the next one bit; consumes the one."""
        k = int(np.searchsorted(self.ones, self.pos))
        if k >= self.ones.size:
            raise FormatError("unary code runs past end of body")
        z = int(self.ones[k]) - self.pos
        self.pos += z + 1
        return z

    def gamma(self) -> int:
        """Elias gamma of x >= 0: unary(b) then the b low bits of x+1, b = floor(log2(x+1))."""
        b = self.unary()
        if b > 63:
            raise FormatError("gamma code too long")
        return ((1 << b) | self.read_bits(b)) - 1

    def zeta(self, k: int) -> int:
        """Boldi-Vigna zeta_k of x >= 0 (coded on v = x+1): unary(h) with
        h = floor(log2(v)/k), then v - 2^(hk) as a minimal binary code over
        the 2^((h+1)k) - 2^(hk) values of that bucket."""
        h = self.unary()
        if (h + 1) * k > 64:
            raise FormatError("zeta code too long")
        left = 1 << (h * k)
        zmax = (1 << ((h + 1) * k)) - left
        s = (zmax - 1).bit_length()          # ceil(log2(zmax)) for zmax >= 2
        if s == 0:                           # a bucket of one value: no bits
            return left - 1
        thr = (1 << s) - zmax
        z = self.read_bits(s - 1)
        if z >= thr:
            z = ((z << 1) | self.read_bits(1)) - thr
        return left + z - 1


def nu_inv(u: int) -> int:
    """Inverse of nu(z) = 2z (z >= 0), 2|z|-1 (z < 0)."""
    return u // 2 if u % 2 == 0 else -((u + 1) // 2)


def parse_header(data):
    data = bytes(data)
    if len(data) < 64 or data[:4] != b"BVMV":
        raise FormatError("bad magic")
    version, n, m, W, R, Lmin, zk, stride, _pad, body_bits, nseg = struct.unpack_from("<IQQIIIIIIQQ", data, 4)
    if version != 1:
        raise FormatError("unsupported version")
    hdr = dict(n=n, m=m, W=W, R=R, Lmin=Lmin, zeta_k=zk, stride=stride, body_bits=body_bits, nseg=nseg)
    off = 64 + 8 * nseg
    if off + (body_bits + 7) // 8 > len(data):
        raise FormatError("truncated stream")
    hdr["seg_offsets"] = list(struct.unpack_from("<%dQ" % nseg, data, 64)) if nseg else []
    return hdr, data[off:]


def decode(data, with_stats=False):
    """Decode a bitstream into (rowptr uint64, col uint32, refs uint8, header).

    refs[i] = g_i = i - r_i (0 = no reference).  Raises FormatError on any
    inconsistency (ids out of range, unsorted or duplicate ids, a reference
    outside the window or deeper than R, counts that do not add up).

    With `with_stats`, also returns an (n, 5) int64 array of how each row is
    coded: reference-chain depth, reference entries skipped, intervals,
    their total length, residuals."""
    hdr, body = parse_header(data)
    n, W, R, Lmin, zk = hdr["n"], hdr["W"], hdr["R"], hdr["Lmin"], hdr["zeta_k"]
    br = BitReader(body, hdr["body_bits"])
    lists: list[list[int]] = []
    refs = np.zeros(n, dtype=np.uint8)
    depth = [0] * n
    stats = np.zeros((n, 5), dtype=np.int64)
    for i in range(n):
        d = br.gamma()
        if d == 0:
            lists.append([])
            continue
        if d > n:
            raise FormatError("degree larger than n at node %d" % i)
        g = br.unary() if W > 0 else 0
        if g > W or g > i:
            raise FormatError("reference outside the window at node %d" % i)
        if g and hdr["stride"] and hdr["nseg"] and (i - g) // hdr["stride"] != i // hdr["stride"]:
            raise FormatError("reference crosses a segment boundary at node %d" % i)
        copied: list[int] = []
        if g > 0:
            ref = lists[i - g]
            if depth[i - g] + 1 > R:
                raise FormatError("reference chain deeper than R at node %d" % i)
            depth[i] = depth[i - g] + 1
            nblocks = br.gamma()
            pos, keep = 0, True
            for b in range(nblocks):
                ln = br.gamma() if b == 0 else br.gamma() + 1
                if pos + ln > len(ref):
                    raise FormatError("copy blocks exceed the reference list at node %d" % i)
                if keep:
                    copied.extend(ref[pos:pos + ln])
                pos += ln
                keep = not keep
            if keep:                      # b even: the rest is copied
                copied.extend(ref[pos:])
            refs[i] = g
            stats[i, 0] = depth[i]
            stats[i, 1] = len(ref) - len(copied)
        ne = d - len(copied)
        if ne < 0:
            raise FormatError("more copied entries than the degree at node %d" % i)
        extras: list[int] = []
        if ne > 0:
            nint = br.gamma() if ne >= Lmin else 0
            prev_last = None
            for k in range(nint):
                if k == 0:
                    s = i + nu_inv(br.gamma())
                else:
                    s = prev_last + 2 + br.gamma()
                ln = br.gamma() + Lmin
                extras.extend(range(s, s + ln))
                prev_last = s + ln - 1
            nres = ne - len(extras)
            if nres < 0:
                raise FormatError("intervals exceed the degree at node %d" % i)
            stats[i, 2:5] = (nint, len(extras), nres)
            res = []
            prev = None
            for k in range(nres):
                if k == 0:
                    j = i + nu_inv(br.zeta(zk))
                else:
                    j = prev + 1 + br.zeta(zk)
                res.append(j)
                prev = j
            extras = sorted(extras + res)
        row = sorted(copied + extras)
        for a, b in zip(row, row[1:]):
            if a >= b:
                raise FormatError("duplicate id in row %d" % i)
        if row and (row[0] < 0 or row[-1] >= n):
            raise FormatError("id out of range in row %d" % i)
        lists.append(row)
    m = sum(len(r) for r in lists)
    if m != hdr["m"]:
        raise FormatError("edge count %d differs from header %d" % (m, hdr["m"]))
    rowptr = np.zeros(n + 1, dtype=np.uint64)
    rowptr[1:] = np.cumsum([len(r) for r in lists])
    col = np.fromiter((j for r in lists for j in r), dtype=np.uint32, count=m)
    if with_stats:
        return rowptr, col, refs, hdr, stats
    return rowptr, col, refs, hdr
