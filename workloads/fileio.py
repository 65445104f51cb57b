"""Binary edge-list file (``.cflg``) shared by every consumer.

Layout, all little-endian:

    8 bytes   magic  b"CFLG0001"
    u32       n  (vertices, ids 0..n-1)
    u64       m  (edges)
    u32       L  (label names)
    L times:  u32 byte length, UTF-8 name bytes
    u32 src[m], u32 dst[m], u32 label[m]   (label indexes the name table)
"""

from __future__ import annotations

import struct

import numpy as np

from .graphs import Graph

MAGIC = b"CFLG0001"


def write_cflg(path, g: Graph) -> None:
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<IQI", g.n, g.m, len(g.label_names)))
        for name in g.label_names:
            b = name.encode("utf-8")
            f.write(struct.pack("<I", len(b)))
            f.write(b)
        for a in (g.src, g.dst, g.label):
            f.write(np.ascontiguousarray(a, dtype="<u4").tobytes())


def read_cflg(path) -> Graph:
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not a CFLG0001 file")
        n, m, L = struct.unpack("<IQI", f.read(16))
        names = []
        for _ in range(L):
            (k,) = struct.unpack("<I", f.read(4))
            names.append(f.read(k).decode("utf-8"))
        arrs = [np.frombuffer(f.read(4 * m), dtype="<u4").astype(np.uint32)
                for _ in range(3)]
    return Graph(n, arrs[0], arrs[1], arrs[2], names)
