"""Brute force CFL-reachability for tiny graphs -- TEST INFRASTRUCTURE.

Straight from the problem statement (Section 1): (i, j) belongs to R_x when
some path from i to j spells a word of L(x).  Every path of length at most L
(the empty path included) is enumerated, and its label word is tested for
membership with the CYK table construction (textbook dynamic programming over
spans; empty spans hold the nullable symbols).

On an acyclic graph with L >= n - 1 every path is seen, so the result is
exact.  On a graph with cycles it is a subset of the exact answer that grows
with L.
"""

from __future__ import annotations

from .textgrammar import TextGrammar


class _Cyk:
    """Incremental CYK: the word grows by one terminal at a time; column e of
    the table holds, for each start s <= e, the symbols deriving word[s:e]."""

    def __init__(self, g: TextGrammar):
        self.g = g
        self.null = frozenset(g.nullable())
        self.unit = g.unit
        self.seqs = g.sequences()

    def _close(self, cell, span, s, e):
        # cell: symbols deriving w[s:e]; span(a, b) = T[a][b] for
        # s <= a <= b <= e (span(s, e) is the cell itself).  x -> y1 ... yk
        # holds when split points s = m0 <= m1 <= ... <= mk = e exist with
        # yq in T[m(q-1)][mq]: the set of reachable m is carried symbol by
        # symbol.
        changed = True
        while changed:
            changed = False
            for x, y in self.unit:
                if y in cell and x not in cell:
                    cell.add(x)
                    changed = True
            for x, ys in self.seqs:
                if x in cell:
                    continue
                reach = {s}
                for y in ys:
                    reach = {b for a in reach for b in range(a, e + 1) if y in span(a, b)}
                    if not reach:
                        break
                if e in reach:
                    cell.add(x)
                    changed = True
        return cell

    def extend(self, cols, terminal):
        """cols[e][s] = T[s][e] for e < len(cols); returns the new column."""
        e = len(cols)            # new end index (word length after extension)
        col = [None] * (e + 1)
        col[e] = set(self.null)  # empty span T[e][e]
        for s in range(e - 1, -1, -1):
            cell = {terminal} if s == e - 1 else set()

            # T[a][b]: earlier columns for b < e, this column (computed for
            # a > s already) for b = e, the cell for (s, e)
            def span(a, b, cell=cell, s=s):
                if b < e:
                    return cols[b][a]
                return cell if a == s else col[a]
            col[s] = self._close(cell, span, s, e)
        return col


def brute_force(grammar_text: str, graph, max_len: int):
    """{nt: set of (i, j)} from all paths of length <= max_len."""
    g = TextGrammar(grammar_text)
    cyk = _Cyk(g)
    adj = [[] for _ in range(graph.n)]
    for u, t, v in graph.edges():
        adj[u].append((t, v))
    out = {x: set() for x in g.nts}
    col0 = [set(cyk.null)]

    def dfs(root, v, cols, depth):
        for x in cols[-1][0]:
            if x in out:
                out[x].add((root, v))
        if depth == max_len:
            return
        for t, w in adj[v]:
            cols.append(cyk.extend(cols, t))
            dfs(root, w, cols, depth + 1)
            cols.pop()

    for i in range(graph.n):
        dfs(i, i, [col0], 0)
    return out


def word_in(grammar_text: str, nt: str, word) -> bool:
    """Membership of one word in L(nt) (CYK)."""
    g = TextGrammar(grammar_text)
    cyk = _Cyk(g)
    cols = [[set(cyk.null)]]
    for t in word:
        cols.append(cyk.extend(cols, t))
    return nt in cols[-1][0]
