"""Turn the witnesses of a GPU solve (cflr_result_witness) into a derivation
certificate in the format oracle/certificate.py checks -- test
infrastructure.

A witness names, per pair (x, i, j), what derived it: an eps rule, an edge
(x -> t), or a binary rule with its midpoint, plus the round that derived
the pair.  The rule may be one of a non-terminal y that x reaches through
unit rules (the library copies y's productions into x); the pair is then
certified through the unit chain x -> y1 -> ... -> y, whose pairs the
result also holds.  Facts are ordered by round, and within a round by the
unit rules (a unit rule's premise first); a binary rule's premises come
from earlier rounds.  The checker then verifies each fact against the
grammar text and the facts before it, so a wrong witness cannot pass,
whatever this module does.
"""

from __future__ import annotations

import struct

import numpy as np

from oracle.textgrammar import TextGrammar

NONE = 0xFFFFFFFF


def _unit_order(tg):
    """rank[x] for non-terminals such that x -> y (unit) gives rank[y] <
    rank[x]; raises on a cycle of unit rules."""
    deps = {x: [y for a, y in tg.unit if a == x and tg.is_nt(y)] for x in tg.nts}
    rank, state = {}, {}

    def visit(x):
        if state.get(x) == 1:
            raise ValueError("unit rules form a cycle")
        if x in rank:
            return
        state[x] = 1
        for y in deps[x]:
            visit(y)
        state[x] = 2
        rank[x] = len(rank)

    for x in tg.nts:
        visit(x)
    return rank


def _unit_paths(tg):
    """first[x][y] = the first step of a shortest unit chain x -> ... -> y."""
    out = {}
    for x in tg.nts:
        first = {x: None}
        frontier = [(x, None)]
        while frontier:
            nxt = []
            for a, f in frontier:
                for u, y in tg.unit:
                    if u == a and tg.is_nt(y) and y not in first:
                        first[y] = y if f is None else f
                        nxt.append((y, first[y]))
            frontier = nxt
        out[x] = first
    return out


def write_certificate(path, text, graph, symbols, results):
    """results: {nt: (src, dst, left, right, mid, round)} numpy arrays for
    every non-terminal of the text; symbols: the library's symbol names
    (non-terminals, then terminals).  Writes the certificate to path."""
    tg = TextGrammar(text)
    if tg.long:
        raise ValueError("right sides of at most two symbols")
    names = list(tg.nts) + list(tg.terminals)
    sid = {s: k for k, s in enumerate(names)}
    rules, rid = [], {}

    def rule(kind, lhs, r1=None, r2=None):
        key = (kind, lhs, r1, r2)
        if key not in rid:
            rid[key] = len(rules)
            rules.append((kind, sid[lhs], sid[r1] if r1 is not None else NONE,
                          sid[r2] if r2 is not None else NONE))
        return rid[key]

    eps = set(tg.eps)
    units = set(tg.unit)
    binary = set(tg.binary)
    first = _unit_paths(tg)
    rank = _unit_order(tg)

    def owner(x, has):
        """x itself if has(x), else the first step of a unit chain from x to
        a non-terminal y with has(y)."""
        if has(x):
            return x, None
        for y, step in first[x].items():
            if y != x and has(y):
                return y, step
        raise AssertionError(f"no rule of {x} or of a unit-reachable non-terminal fits the witness")

    facts = []  # (order key, s, i, j, rule, mid)
    seen = set()
    for u, t, v in graph.edges():
        if t in sid and not tg.is_nt(t) and (t, u, v) not in seen:
            seen.add((t, u, v))
            facts.append(((-1, 0), sid[t], u, v, NONE, 0))
    for x, (src, dst, left, right, mid, rnd) in results.items():
        for i, j, l, r, k, rd in zip(src.tolist(), dst.tolist(), left.tolist(), right.tolist(),
                                     mid.tolist(), rnd.tolist()):
            assert rd != NONE, f"{x}({i},{j}) has no witness"
            if l == NONE:                     # eps
                y, step = owner(x, lambda y: y in eps)
                r_id, m = (rule(0, x), 0) if step is None else (rule(1, x, step), 0)
            elif r == NONE:                   # an edge: x -> t
                t = symbols[l]
                y, step = owner(x, lambda y: (y, t) in units)
                r_id, m = (rule(1, x, t), 0) if step is None else (rule(1, x, step), 0)
            else:                             # x -> a b through midpoint k
                a, b = symbols[l], symbols[r]
                y, step = owner(x, lambda y: (y, a, b) in binary)
                r_id, m = (rule(2, x, a, b), k) if step is None else (rule(1, x, step), 0)
            facts.append(((rd, rank[x]), sid[x], i, j, r_id, m))
    facts.sort(key=lambda f: f[0])
    with open(path, "wb") as f:
        f.write(struct.pack("<I", len(names)))
        for s in names:
            b = s.encode()
            f.write(struct.pack("<I", len(b)) + b + struct.pack("<I", 1 if tg.is_nt(s) else 0))
        f.write(struct.pack("<I", len(rules)))
        for rl in rules:
            f.write(struct.pack("<4I", *rl))
        f.write(struct.pack("<Q", len(facts)))
        arr = np.array([fa[1:] for fa in facts], dtype="<u4").reshape(-1, 5)
        f.write(arr.tobytes())
