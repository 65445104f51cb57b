"""Algorithm 1 as printed, on dense matrices -- TEST INFRASTRUCTURE.

M is kept as one dense boolean |V| x |V| matrix per non-terminal.  The edges
seed it (each edge (i, t, j) puts every x with x -> t into M_ij), a
non-terminal that derives the empty word holds every (i, i) (the empty path
of Algorithm 1's Result), and then M <- M U (M . M) is repeated while M
changes, where the product in the reachability semiring decomposes into one
boolean matrix product per binary production (Definition 2).  A terminal in
a binary position reads the adjacency matrix of its label; a unit rule
x -> y copies M_y into M_x.

Exact for any graph, but O(|P| n^3) per iteration: small n only.
"""

from __future__ import annotations

import numpy as np

from .textgrammar import TextGrammar


def naive_closure(grammar_text: str, graph, max_iter: int = 100000):
    g = TextGrammar(grammar_text)
    if g.long:
        raise ValueError("Algorithm 1 works on WCNF: right sides of at most two symbols")
    n = graph.n
    adj = {t: np.zeros((n, n), dtype=bool) for t in g.terminals}
    for u, t, v in graph.edges():
        if t in adj:
            adj[t][u, v] = True
    M = {x: np.zeros((n, n), dtype=bool) for x in g.nts}

    def mat(s):
        return M[s] if s in M else adj[s]

    for x, y in g.unit:
        if y in adj:
            M[x] |= adj[y]
    for x in g.eps:
        M[x] |= np.eye(n, dtype=bool)
    iterations = 0
    while True:
        iterations += 1
        if iterations > max_iter:
            raise RuntimeError("no fixpoint")
        new = {x: M[x].copy() for x in g.nts}
        for x, y, z in g.binary:
            prod = mat(y).astype(np.int64) @ mat(z).astype(np.int64)
            new[x] |= prod > 0
        for x, y in g.unit:
            new[x] |= mat(y)
        if all((new[x] == M[x]).all() for x in g.nts):
            break
        M = new
    out = {}
    for x in g.nts:
        i, j = np.nonzero(M[x])
        out[x] = set(zip(i.tolist(), j.tolist()))
    return out, iterations
