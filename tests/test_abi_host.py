"""Host-only checks of libcflr (no GPU): every symbol of include/cflr.h is
exported, the grammar parser rejects malformed text, and the lowering to
strict weak Chomsky normal form has the expected shape."""

import ctypes as C
import os
import re

import pytest

from workloads import grammars as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "cflr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cflr_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function(cflr_lib):
    names = header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(cflr_lib, name), name


def test_binding_declares_every_function():
    from paper_2401_11029_amd._lib import SIGNATURES
    assert sorted(SIGNATURES) == header_functions()


def test_version_and_defaults(cflr_lib):
    import paper_2401_11029_amd as cflr
    assert b"gfx950" in cflr_lib.cflr_version()
    o = cflr.opts()
    assert o.semi_naive == 1 and o.max_rounds == 0
    # automatic sizes unless set: new-pair buffer, grid, replay depth, item size
    assert o.delta_capacity == 0 and o.grid_waves == 0 and o.rounds_per_sync == 0 and o.chunk_pairs == 0
    assert o.mirror == 0 and o.sparse_heavy == 0 and o.witness == 0
    assert cflr.opts(chunk_pairs=1000).chunk_pairs == 1000


def info(text):
    import paper_2401_11029_amd as cflr
    g = cflr.Grammar(text)
    return g.nonterminals, g.info()


def test_lowering_dyck1(cflr_lib):
    nts, i = info(G.DYCK1)
    assert nts == ["S", "X", "A", "B"]
    assert i == dict(user_nonterminals=4, wrappers=0, matrices=4, binary=4,
                     terminal_rules=2, eps_rules=1, terminals=2, helpers=0, mirror_skipped=0)


def test_mirror_of_grammars(cflr_lib):
    # Fig. 4b is closed under reversal (PT <-> FT, LP_i <-> FL_i, FS_i <->
    # SP_i, LPFS_i <-> SPFL_i; t <-> t_bar): one production of each of the
    # 257 mirror pairs keeps its product.  Fig. 4a, the alias grammars and
    # Dyck-1 have no syntactic mirror.
    assert info(G.pointsto_fig4b(64))[1]["mirror_skipped"] == 257
    assert info(G.pointsto_fig4b(8))[1]["mirror_skipped"] == 33
    for text in (G.pointsto_fig4a(8), G.ALIAS_FIG5A, G.ALIAS_FIG5B, G.DYCK1, G.fsca_fig6b(4), G.cscvf_fig7b(4)):
        assert info(text)[1]["mirror_skipped"] == 0
    # a mirror pair found through the structure: FT's production mirrors PT's
    base = "PT -> alloc | assign PT\nFT -> alloc_bar | FT assign_bar\n"
    assert info(base)[1]["mirror_skipped"] == 1
    # a rule whose mirror is missing breaks it
    assert info(base + "PT -> PT load\n")[1]["mirror_skipped"] == 0
    assert info("PT -> alloc | assign PT\nFT -> alloc_bar | assign_bar FT\n")[1]["mirror_skipped"] == 0
    # a self-mirrored non-terminal: S -> A T | T2 B with T -> S B, T2 -> A S
    # (S and the eps rule are their own mirror; T <-> T2, A <-> B)
    assert info("S -> eps | A T | T2 B\nT -> S B\nT2 -> A S\nA -> a\nB -> a_bar\n")[1]["mirror_skipped"] == 2
    # a label without a partner is its own reverse: X <-> Y through c
    assert info("R -> c | X R | R Y\nX -> c\nY -> c\n")[1]["mirror_skipped"] == 1
    # the same language without the mirrored productions has no mirror
    assert info("S -> eps | A S2\nS2 -> S B\nA -> a\nB -> a_bar\n")[1]["mirror_skipped"] == 0


def test_lowering_long_right_sides(cflr_lib):
    # Fig. 5a as given: M -> d_bar V d, V -> V1 V2 V3, V1 -> V2 a_bar V1 and
    # V3 -> a V2 V3 need helpers for the suffixes "V d", "V2 V3" (shared by two
    # rules) and "a_bar V1"; four wrappers; V2 -> M is removed by copying
    nts, i = info(G.ALIAS_FIG5A)
    assert nts == ["M", "V", "V1", "V2", "V3"]
    assert i == dict(user_nonterminals=5, wrappers=4, matrices=12, binary=8,
                     terminal_rules=4, eps_rules=4, terminals=4, helpers=3, mirror_skipped=0)
    # a right side of four symbols: two helpers per distinct suffix chain
    nts, i = info("S -> a S b S | eps")
    assert nts == ["S"] and i["helpers"] == 2 and i["binary"] == 3 and i["wrappers"] == 2


def test_lowering_alias_fig5a(cflr_lib):
    # V2 -> M is removed by giving V2 the rule M -> d_bar Y1; four wrappers
    nts, i = info(G.ALIAS_FIG5A_WCNF)
    assert nts == ["M", "Y1", "V", "Y2", "V1", "Y3", "V2", "V3", "Y4"]
    assert i["wrappers"] == 4 and i["matrices"] == 13
    assert i["binary"] == 8 + 1 and i["eps_rules"] == 4 and i["terminal_rules"] == 4


def test_lowering_alias_fig5b(cflr_lib):
    nts, i = info(G.ALIAS_FIG5B)
    assert nts == ["M", "N1", "N2", "N3", "AM"]
    assert i["wrappers"] == 2 and i["binary"] == 8


def test_lowering_pointsto_64_fields(cflr_lib):
    nts, i = info(G.pointsto_fig4b(64))
    assert len(nts) == 2 + 6 * 64
    assert i["wrappers"] == 2 + 4 * 64
    assert i["binary"] == 2 + 8 * 64
    assert i["matrices"] == 386 + 258


def test_lowering_unit_cycle_and_chain(cflr_lib):
    nts, i = info("A -> B\nB -> A | C\nC -> c | A A\n")
    # A, B, C all reach each other: each gets C's two productions
    assert i["terminal_rules"] == 3 and i["binary"] == 3


@pytest.mark.parametrize("bad", [
    "", "S", "S -> a b eps c", "S -> -> a", "S T -> a", "S -> a eps",
    "S -> |", "eps -> a",
])
def test_parse_errors(cflr_lib, bad):
    import paper_2401_11029_amd as cflr
    with pytest.raises(cflr.CflrError) as e:
        cflr.Grammar(bad)
    assert e.value.status == 2  # CFLR_EPARSE


def test_null_arguments_are_rejected(cflr_lib):
    out = C.c_void_p()
    assert cflr_lib.cflr_grammar_parse(None, 5, C.byref(out)) == 1
    assert cflr_lib.cflr_grammar_info_get(None, None) == 1
    assert cflr_lib.cflr_result_count(None, 0, None) == 1
    assert cflr_lib.cflr_grammar_nonterminal_name(None, 0) is None


def test_failing_server_calls_set_the_error_message(cflr_lib):
    # every cflr_server_* failure returns a status and leaves a message in
    # cflr_last_error (argument errors are caught before any device call)
    L = cflr_lib
    out = C.c_void_p()
    t = C.c_uint64()
    assert L.cflr_server_create(None, 1 << 20, 4, None, C.byref(out)) == 1  # CFLR_EINVAL
    assert L.cflr_last_error() not in (None, b"")
    L.cflr_opts_default  # keep the binding loaded
    assert L.cflr_server_submit(None, None, None, C.byref(t)) == 1
    assert b"null" in L.cflr_last_error()
    assert L.cflr_server_poll(None, 1, C.byref(out)) == 1
    assert L.cflr_last_error() != b""
    assert L.cflr_server_wait(None, 1, 0, C.byref(out)) == 1
    assert L.cflr_last_error() != b""
    assert L.cflr_server_times(None, 1, None, None, None) == 1
    assert L.cflr_last_error() != b""


def _struct_fields(name):
    """Field names of `typedef struct name { ... } name;` in include/cflr.h."""
    import re
    with open(os.path.join(ROOT, "include", "cflr.h")) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, re.S).group(1)
    return re.findall(r"\b(?:uint32_t|uint64_t|double|int)\s+(\w+);", body)


def test_binding_structs_mirror_the_header():
    import paper_2401_11029_amd as cflr
    from paper_2401_11029_amd._lib import Opts, Stats
    assert [f[0] for f in Opts._fields_] == _struct_fields("cflr_opts")
    assert [f[0] for f in Stats._fields_] == _struct_fields("cflr_stats")
    assert cflr.opts().storage == 0 and cflr.opts(storage=2).storage == 2
    assert cflr.opts().witness == 0 and cflr.opts(witness=1).witness == 1


def test_grammar_symbols_for_witnesses():
    import ctypes as C
    import paper_2401_11029_amd as cflr
    g = cflr.Grammar("S -> eps | a S b | S S\nT -> c\n")
    assert g.nonterminals == ["S", "T"]
    assert sorted(g.terminals) == ["a", "b", "c"]
    assert g.symbols == g.nonterminals + g.terminals
    L = cflr.lib()
    assert L.cflr_grammar_terminal_name(g._h, 3) is None
    w = C.c_uint64()
    assert L.cflr_result_witness(None, 0, None, None, None, None, 0, 0, C.byref(w)) == 1
    assert L.cflr_last_error() != b""


def test_mirror_of_random_closed_grammars(cflr_lib):
    # grammars closed under reversal by construction (every production
    # added with its mirror: X_k <-> Y_k, t <-> t_bar) have a mirror, and
    # the plan keeps one production of each mirror pair; dropping one
    # production of a pair breaks the mirror
    import random
    for seed in range(20):
        rnd = random.Random(seed)
        k = rnd.randint(2, 6)
        nts = [(f"X{i}", f"Y{i}") for i in range(k)]
        mir = {}
        for x, y in nts:
            mir[x], mir[y] = y, x
        terms = [(f"t{i}", f"t{i}_bar") for i in range(rnd.randint(1, 3))]
        lines, prods = [], set()
        for x, y in nts:  # every non-terminal derives a terminal
            t, tb = rnd.choice(terms)
            lines += [f"{x} -> {t}", f"{y} -> {tb}"]
        for _ in range(rnd.randint(2, 8)):
            c, a, b = (rnd.choice(nts)[rnd.randint(0, 1)] for _ in range(3))
            p, q = (c, a, b), (mir[c], mir[b], mir[a])
            if p in prods or q in prods:
                continue
            prods |= {p, q}
            lines += [f"{c} -> {a} {b}", f"{mir[c]} -> {mir[b]} {mir[a]}"]
        text = "\n".join(lines) + "\n"
        pairs = len({frozenset([p, (mir[p[0]], mir[p[2]], mir[p[1]])]) for p in prods})
        self_mirrored = sum(1 for p in prods if p == (mir[p[0]], mir[p[2]], mir[p[1]]))
        assert info(text)[1]["mirror_skipped"] == pairs - self_mirrored, (seed, text)
        # remove the second production of one non-self pair
        non_self = [p for p in prods if p != (mir[p[0]], mir[p[2]], mir[p[1]])]
        if non_self:
            c, a, b = non_self[0]
            broken = text.replace(f"{c} -> {a} {b}\n", "", 1)
            assert info(broken)[1]["mirror_skipped"] < pairs - self_mirrored or pairs == 0, (seed, broken)
