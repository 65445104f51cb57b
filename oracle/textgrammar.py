"""Reader of the grammar text format for the Python-side checkers.

Test infrastructure.  Format: ``LHS -> ALT | ALT``, ALT is ``eps`` or one
or more symbols; left-hand sides are the non-terminals, all other symbols
are terminals (edge labels); ``#`` starts a comment.  Right-hand sides of
three or more symbols (the CFPQ Data grammars, Figs. 4a-7a) are kept as they
are in ``long``.
"""

from __future__ import annotations


class TextGrammar:
    def __init__(self, text: str):
        self.nts = []          # non-terminals, first left-side order
        self.eps = []          # x  for x -> eps
        self.unit = []         # (x, y) for x -> y   (y terminal or NT)
        self.binary = []       # (x, y, z) for x -> y z
        self.long = []         # (x, (y1, ..., yk)) for x -> y1 ... yk, k >= 3
        lines = []
        for raw in text.splitlines():
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            if "->" not in line:
                raise ValueError(f"line without '->': {raw!r}")
            lhs, body = line.split("->", 1)
            lhs = lhs.strip()
            if not lhs or len(lhs.split()) != 1:
                raise ValueError(f"bad left side: {raw!r}")
            if lhs not in self.nts:
                self.nts.append(lhs)
            lines.append((lhs, body))
        for lhs, body in lines:
            for alt in body.split("|"):
                sy = alt.split()
                if len(sy) == 1 and sy[0] == "eps":
                    self.eps.append(lhs)
                elif len(sy) == 1:
                    self.unit.append((lhs, sy[0]))
                elif len(sy) == 2 and "eps" not in sy:
                    self.binary.append((lhs, sy[0], sy[1]))
                elif len(sy) >= 3 and "eps" not in sy:
                    self.long.append((lhs, tuple(sy)))
                else:
                    raise ValueError(f"bad right side in: {lhs} -> {alt}")
        syms = set(self.nts)
        rhs = {y for _, y in self.unit} | {y for _, y, _ in self.binary} | \
            {z for _, _, z in self.binary} | {y for _, ys in self.long for y in ys}
        self.terminals = sorted(rhs - syms)

    def is_nt(self, s):
        return s in self.nts

    def nullable(self):
        """Non-terminals deriving the empty word (plain fixpoint)."""
        null = set(self.eps)
        changed = True
        while changed:
            changed = False
            for x, y in self.unit:
                if y in null and x not in null:
                    null.add(x)
                    changed = True
            for x, y, z in self.binary:
                if y in null and z in null and x not in null:
                    null.add(x)
                    changed = True
            for x, ys in self.long:
                if x not in null and all(y in null for y in ys):
                    null.add(x)
                    changed = True
        return null

    def sequences(self):
        """(x, right side) of every rule with two or more symbols."""
        return [(x, (y, z)) for x, y, z in self.binary] + list(self.long)
