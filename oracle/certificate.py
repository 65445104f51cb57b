"""Certificate and closure checks -- TEST INFRASTRUCTURE.

A set of facts equals the least fixpoint (the exact answer) when it is

* sound: every fact has a derivation -- here, every fact names the rule and
  midpoint that produced it, and the facts it rests on were inserted earlier
  (a well-founded order, so no fact justifies itself through a cycle);
* seeded: every edge whose label is a terminal of the grammar, and every
  (x, i, i) for x -> eps, is in the set;
* closed: for every binary rule x -> y z, R_y . R_z is contained in R_x, and
  for every unit rule x -> y, R_y is contained in R_x.

Sound means "contained in the least fixpoint"; seeded and closed mean
"contains it".  Both checks are written here independently of the solver.
"""

from __future__ import annotations

import struct

import numpy as np
import scipy.sparse as sp

from .textgrammar import TextGrammar

NONE = 0xFFFFFFFF
KIND = {0: "eps", 1: "unit", 2: "bin"}


def read_certificate(path):
    with open(path, "rb") as f:
        (nsym,) = struct.unpack("<I", f.read(4))
        names, is_nt = [], []
        for _ in range(nsym):
            (k,) = struct.unpack("<I", f.read(4))
            names.append(f.read(k).decode("utf-8"))
            (nt,) = struct.unpack("<I", f.read(4))
            is_nt.append(bool(nt))
        (nr,) = struct.unpack("<I", f.read(4))
        rules = [struct.unpack("<4I", f.read(16)) for _ in range(nr)]
        (nf,) = struct.unpack("<Q", f.read(8))
        facts = np.frombuffer(f.read(20 * nf), dtype="<u4").reshape(nf, 5)
    return names, is_nt, rules, facts


def check_certificate(grammar_text: str, graph, cert_path: str):
    """Verify soundness of the certificate; returns {nt: set of pairs} of
    the certified facts.  Raises AssertionError on any defect."""
    g = TextGrammar(grammar_text)
    if g.long:
        raise ValueError("certificates are checked for grammars with right sides of at most two symbols")
    names, is_nt, rules, facts = read_certificate(cert_path)
    # every rule the solver used must be a rule of the grammar text
    allowed = {("eps", x, None, None) for x in g.eps}
    allowed |= {("unit", x, y, None) for x, y in g.unit}
    allowed |= {("bin", x, y, z) for x, y, z in g.binary}
    named = []
    for kind, lhs, r1, r2 in rules:
        k = KIND[kind]
        key = (k, names[lhs],
               names[r1] if k in ("unit", "bin") else None,
               names[r2] if k == "bin" else None)
        assert key in allowed, f"rule not in grammar: {key}"
        named.append(key)
    edges = set(graph.edges())
    serial = {}
    for t, (s, i, j, r, mid) in enumerate(facts.tolist()):
        key = (s, i, j)
        assert key not in serial, f"duplicate fact {names[s]}({i},{j})"
        if r == NONE:
            assert not is_nt[s], "edge fact on a non-terminal"
            assert (i, names[s], j) in edges, f"no edge {i} -{names[s]}-> {j}"
        else:
            kind, lhs, y, z = named[r]
            assert lhs == names[s], "fact symbol differs from rule head"
            r1, r2 = rules[r][2], rules[r][3]
            if kind == "eps":
                assert i == j, "eps fact off the diagonal"
            elif kind == "unit":
                assert serial.get((r1, i, j), t) < t, \
                    f"unit fact {names[s]}({i},{j}) lacks an earlier premise"
            else:
                assert serial.get((r1, i, mid), t) < t and \
                    serial.get((r2, mid, j), t) < t, \
                    f"binary fact {names[s]}({i},{j}) via {mid} lacks premises"
        serial[key] = t
    out = {x: set() for x in g.nts}
    for (s, i, j) in serial:
        if is_nt[s]:
            out[names[s]].add((i, j))
    return out


def _csr(pairs, n):
    if not pairs:
        return sp.csr_matrix((n, n), dtype=np.int64)
    ij = np.array(sorted(pairs), dtype=np.int64)
    data = np.ones(ij.shape[0], dtype=np.int64)
    return sp.csr_matrix((data, (ij[:, 0], ij[:, 1])), shape=(n, n))


def check_closed(grammar_text: str, graph, result):
    """result: {nt: set of (i, j)}.  Asserts seeded and closed."""
    g = TextGrammar(grammar_text)
    n = graph.n
    term = {t: set() for t in g.terminals}
    for u, t, v in graph.edges():
        if t in term:
            term[t].add((u, v))

    def rel(s):
        return result[s] if s in result else term[s]

    for x in g.eps:
        assert all((i, i) in result[x] for i in range(n)), f"{x}: eps seed"
    for x, y in g.unit:
        missing = rel(y) - result[x]
        assert not missing, f"{x} -> {y}: {len(missing)} pairs missing"
    mats = {s: _csr(rel(s), n) for s in list(g.nts) + list(g.terminals)}
    for x, y, z in g.binary:
        prod = (mats[y] @ mats[z]).tocoo()
        need = set(zip(prod.row.tolist(), prod.col.tolist()))
        missing = need - result[x]
        assert not missing, f"{x} -> {y} {z}: {len(missing)} pairs missing"
