"""Grammar texts for the workloads (data only: no solver arithmetic).

Text format, shared by every consumer (each parses it with its own code):

* one production per line, ``LHS -> RHS``; alternatives may be joined with
  ``|`` on one line;
* ``RHS`` is ``eps`` (the empty word) or one or more symbols separated by
  whitespace (right sides longer than two symbols are the CFPQ Data form of
  Figs. 4a-7a; each consumer normalises them with its own code);
* every symbol that appears as a left-hand side is a non-terminal, every other
  symbol is a terminal (an edge label);
* ``#`` starts a comment.

This is weak Chomsky normal form (Definition 1 of the paper) relaxed in the
two ways the paper's own appendix figures use: a terminal may stand in a
binary right-hand side (e.g. ``PT -> assign PT``, Fig. 4b) and a right-hand
side may be a single non-terminal (the unit rule ``V -> M``, Fig. 6b).

Indexed non-terminals (``LP_i``, ``AR_i``; Section 3, optimisation 4) are
templates here: they are expanded to one explicit non-terminal per index.
A bar over a label (reversed edge) is spelled with a ``_bar`` suffix; the
reversed edges themselves are part of the graph, never implied.
"""

from __future__ import annotations


def _join(lines):
    return "\n".join(lines) + "\n"


# Dyck-1 in WCNF (the tiny configuration's grammar).
DYCK1 = _join([
    "# Dyck-1 over a/b in weak Chomsky normal form",
    "S -> eps",
    "S -> S S",
    "S -> A B",
    "S -> A X",
    "X -> S B",
    "A -> a",
    "B -> b",
])

# Field-insensitive C/C++ memory alias, Fig. 5a of the paper, made binary.
# Fig. 5a:  M -> d_bar V d;  V -> eps | V1 V2 V3;  V1 -> eps | V2 a_bar V1;
#           V2 -> eps | M;  V3 -> eps | a V2 V3.
# Each right-hand side of length three gets one helper non-terminal (Y1..Y4);
# the unit rule V2 -> M is kept (the solver lowers it).
ALIAS_FIG5A_WCNF = _join([
    "# memory alias (Fig. 5a) binarised: helpers Y1..Y4",
    "M -> d_bar Y1",
    "Y1 -> V d",
    "V -> eps | V1 Y2",
    "Y2 -> V2 V3",
    "V1 -> eps | V2 Y3",
    "Y3 -> a_bar V1",
    "V2 -> eps | M",
    "V3 -> eps | a Y4",
    "Y4 -> V2 V3",
])

# Field-insensitive C/C++ memory alias, Fig. 5a as given (CFPQ Data form,
# right sides of three symbols).
ALIAS_FIG5A = _join([
    "# memory alias (Fig. 5a)",
    "M -> d_bar V d",
    "V -> eps | V1 V2 V3",
    "V1 -> eps | V2 a_bar V1",
    "V2 -> eps | M",
    "V3 -> eps | a V2 V3",
])

# Field-insensitive C/C++ memory alias, hand-made WCNF of Fig. 5b.
ALIAS_FIG5B = _join([
    "# memory alias, hand WCNF (Fig. 5b)",
    "M -> N1 N3 | N2 N3",
    "N1 -> d_bar | N1 a_bar | N2 a_bar",
    "N2 -> N1 M",
    "N3 -> d | a N3 | AM N3",
    "AM -> a M",
])

# Context-sensitive value flow, Fig. 7a made binary (helper C_i per index).
def cscvf_fig7a(fields: int) -> str:
    lines = ["# value flow (Fig. 7a) binarised", "A -> A A | a | eps"]
    for i in range(fields):
        lines.append(f"A -> call_{i} C_{i}")
        lines.append(f"C_{i} -> A ret_{i}")
    return _join(lines)


# Context-sensitive value flow, Fig. 7a as given (call_i A ret_i).
def cscvf_fig7a_cfg(fields: int) -> str:
    lines = ["# value flow (Fig. 7a)", "A -> A A | a | eps"]
    for i in range(fields):
        lines.append(f"A -> call_{i} A ret_{i}")
    return _join(lines)


# Context-sensitive value flow, WCNF of Fig. 7b.
def cscvf_fig7b(fields: int) -> str:
    lines = ["# value flow (Fig. 7b)", "A -> A a | A AH | eps"]
    for i in range(fields):
        lines.append(f"AH -> call_{i} AR_{i}")
        lines.append(f"AR_{i} -> A ret_{i}")
    return _join(lines)


# Field-sensitive Java points-to, hand WCNF of Fig. 4b, indices expanded.
def pointsto_fig4b(fields: int) -> str:
    lines = [
        f"# field-sensitive points-to (Fig. 4b), {fields} fields",
        "PT -> alloc | assign PT",
        "FT -> alloc_bar | FT assign_bar",
    ]
    for i in range(fields):
        lines += [
            f"PT -> LPFS_{i} PT",
            f"FT -> FT SPFL_{i}",
            f"LPFS_{i} -> LP_{i} FS_{i}",
            f"LP_{i} -> load_{i} PT",
            f"FS_{i} -> FT store_{i}",
            f"SPFL_{i} -> SP_{i} FL_{i}",
            f"SP_{i} -> store_bar_{i} PT",
            f"FL_{i} -> FT load_bar_{i}",
        ]
    return _join(lines)


# Field-sensitive Java points-to, Fig. 4a (the CFPQ Data grammar) made binary.
# Fig. 4a: PT -> PTH alloc; PTH -> eps | assign PTH | load_i Al store_i PTH;
#          FT -> alloc_bar FTH; FTH -> eps | assign_bar FTH
#                | store_bar_i Al load_bar_i FTH;  Al -> PT FT.
def pointsto_fig4a(fields: int) -> str:
    lines = [
        f"# field-sensitive points-to (Fig. 4a) binarised, {fields} fields",
        "PT -> PTH alloc",
        "PTH -> eps | assign PTH",
        "FT -> alloc_bar FTH",
        "FTH -> eps | assign_bar FTH",
        "Al -> PT FT",
    ]
    for i in range(fields):
        lines += [
            f"PTH -> load_{i} Z1_{i}",
            f"Z1_{i} -> Al Z2_{i}",
            f"Z2_{i} -> store_{i} PTH",
            f"FTH -> store_bar_{i} W1_{i}",
            f"W1_{i} -> Al W2_{i}",
            f"W2_{i} -> load_bar_{i} FTH",
        ]
    return _join(lines)


# Field-sensitive Java points-to, Fig. 4a as given (right sides of up to
# four symbols).
def pointsto_fig4a_cfg(fields: int) -> str:
    lines = [
        f"# field-sensitive points-to (Fig. 4a), {fields} fields",
        "PT -> PTH alloc",
        "PTH -> eps | assign PTH",
        "FT -> alloc_bar FTH",
        "FTH -> eps | assign_bar FTH",
        "Al -> PT FT",
    ]
    for i in range(fields):
        lines += [
            f"PTH -> load_{i} Al store_{i} PTH",
            f"FTH -> store_bar_{i} Al load_bar_{i} FTH",
        ]
    return _join(lines)


# Field-sensitive C/C++ alias, Fig. 6b (includes the unit rule V -> M).
def fsca_fig6b(fields: int) -> str:
    lines = [
        "# field-sensitive alias (Fig. 6b)",
        "M -> DV d",
        "DV -> d_bar V",
        "V -> Abar V | V A | M | eps",
        "A -> a M | a | eps",
        "Abar -> M a_bar | a_bar | eps",
    ]
    for i in range(fields):
        lines.append(f"V -> FV_{i} f_{i}")
        lines.append(f"FV_{i} -> f_bar_{i} V")
    return _join(lines)


# Field-sensitive C/C++ alias, Fig. 6a made binary; the optional "M?" of the
# figure is expanded into its two alternatives.
def fsca_fig6a(fields: int) -> str:
    lines = [
        "# field-sensitive alias (Fig. 6a) binarised",
        "M -> d_bar Y",
        "Y -> V d",
        "V -> Abar Z | M | eps",
        "Z -> V A",
        "A -> a | a M | eps",
        "Abar -> a_bar | M a_bar | eps",
    ]
    for i in range(fields):
        lines.append(f"V -> f_bar_{i} Q_{i}")
        lines.append(f"Q_{i} -> V f_{i}")
    return _join(lines)


# Field-sensitive C/C++ alias, Fig. 6a as given, the optional "M?" expanded
# into its two alternatives.
def fsca_fig6a_cfg(fields: int) -> str:
    lines = [
        "# field-sensitive alias (Fig. 6a)",
        "M -> d_bar V d",
        "V -> Abar V A | M | eps",
        "A -> a M | a | eps",
        "Abar -> M a_bar | a_bar | eps",
    ]
    for i in range(fields):
        lines.append(f"V -> f_bar_{i} V f_{i}")
    return _join(lines)


# Textbook special cases used as pins.
TRANSITIVE = _join(["S -> S S | a"])
REFLEXIVE_TRANSITIVE = _join(["S -> S S | a | eps"])


def symbols_of(text: str):
    """Return (nonterminals in first-LHS order, terminals sorted) of a text.

    A plain reader of the format above, for generators that need to know
    which labels a grammar uses.  It validates nothing beyond that.
    """
    nts, rhs = [], []
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        lhs, body = line.split("->", 1)
        lhs = lhs.strip()
        if lhs not in nts:
            nts.append(lhs)
        for alt in body.split("|"):
            rhs += [s for s in alt.split() if s != "eps"]
    terms = sorted(set(s for s in rhs if s not in nts))
    return nts, terms
