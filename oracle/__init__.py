"""CPU oracle for CFL-reachability -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from here.  The product library never does,
and nothing here imports the product package: the two share only the seeded
input generators of ``workloads``.

Contents:

* ``cflr_oracle.c``  the worklist solver (what every non-terminal derives,
  Section 1 and Algorithm 1's Result), compiled by :func:`build`;
* ``brute.py``       path enumeration plus CYK membership (pins the solver on
  tiny graphs);
* ``naive.py``       Algorithm 1 as printed (dense boolean matrices, one
  product per binary production, repeat while anything changes);
* ``certificate.py`` checks a derivation certificate and the closure of a
  result under every production.
"""

from __future__ import annotations

import os
import struct
import subprocess
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "cflr_oracle.c")
BINARY = os.path.join(HERE, "cflr_oracle")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (a plain -O2 build)."""
    if force or not os.path.exists(BINARY) or \
            os.path.getmtime(BINARY) < os.path.getmtime(SOURCE):
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra",
                        "-o", BINARY, SOURCE], check=True)
    return BINARY


def _ensure_built():
    if not os.path.exists(BINARY) or \
            os.path.getmtime(BINARY) < os.path.getmtime(SOURCE):
        build(force=True)


class OracleResult:
    """Per non-terminal: pair count, SHA-256 digest and (optionally) pairs."""

    def __init__(self):
        self.order = []
        self.count = {}
        self.digest = {}
        self.pairs = {}
        self.seconds = None
        self.facts = None
        self.cert_path = None

    def pair_set(self, nt):
        p = self.pairs[nt]
        return set(zip(p[:, 0].tolist(), p[:, 1].tolist()))


def _read_pairs(path, res):
    with open(path, "rb") as f:
        (k,) = struct.unpack("<I", f.read(4))
        for _ in range(k):
            (ln,) = struct.unpack("<I", f.read(4))
            name = f.read(ln).decode("utf-8")
            (cnt,) = struct.unpack("<Q", f.read(8))
            arr = np.frombuffer(f.read(8 * cnt), dtype="<u4").reshape(cnt, 2)
            res.pairs[name] = arr.astype(np.uint32)


def solve(grammar_text: str, graph, pairs: bool = True, digest: bool = True,
          cert: bool = False, workdir: str | None = None,
          timeout: float | None = None, cpu: int | None = None) -> OracleResult:
    """Run the C oracle on (grammar text, workloads.Graph).

    cpu pins the process to one host core (taskset) for timing runs.
    """
    from workloads.fileio import write_cflg
    _ensure_built()
    own = workdir is None
    tmp = tempfile.mkdtemp(prefix="cflr_oracle_") if own else workdir
    try:
        gpath = os.path.join(tmp, "grammar.txt")
        fpath = os.path.join(tmp, "graph.cflg")
        ppath = os.path.join(tmp, "pairs.bin")
        cpath = os.path.join(tmp, "cert.bin")
        with open(gpath, "w") as f:
            f.write(grammar_text)
        write_cflg(fpath, graph)
        cmd = [BINARY, gpath, fpath, "--stats"]
        if digest:
            cmd.append("--digest")
        if pairs:
            cmd += ["--pairs", ppath]
        if cert:
            cmd += ["--cert", cpath]
        if cpu is not None:
            cmd = ["taskset", "-c", str(cpu)] + cmd
        t0 = time.perf_counter()
        out = subprocess.run(cmd, check=True, capture_output=True, text=True,
                             timeout=timeout)
        wall = time.perf_counter() - t0
        res = OracleResult()
        for line in out.stdout.splitlines():
            tok = line.split()
            if tok[0] == "stats":
                res.facts = int(tok[2])
                res.seconds = float(tok[4])
            elif tok[0] == "nt":
                res.order.append(tok[1])
                res.count[tok[1]] = int(tok[2])
                res.digest[tok[1]] = tok[3]
        res.wall_seconds = wall
        if pairs:
            _read_pairs(ppath, res)
            if not digest:
                res.order = list(res.pairs)
                res.count = {k: int(v.shape[0]) for k, v in res.pairs.items()}
        if cert:
            keep = os.path.join(tmp, "cert.keep")
            os.replace(cpath, keep)
            res.cert_path = keep
        return res
    finally:
        if own and not cert:
            for fn in os.listdir(tmp):
                os.unlink(os.path.join(tmp, fn))
            os.rmdir(tmp)


def digest_pairs(src, dst) -> str:
    """SHA-256 of pairs in (i, j) order, each as two little-endian u32 --
    the digest the oracle prints.  Sorts its input first."""
    import hashlib
    src = np.asarray(src, dtype=np.uint64)
    dst = np.asarray(dst, dtype=np.uint64)
    order = np.lexsort((dst, src))
    buf = np.empty((src.shape[0], 2), dtype="<u4")
    buf[:, 0] = src[order]
    buf[:, 1] = dst[order]
    return hashlib.sha256(buf.tobytes()).hexdigest()
