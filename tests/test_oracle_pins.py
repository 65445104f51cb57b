"""Pins of the CPU oracle against what the definitions fix (no GPU).

Each pin is independent of the oracle's code: brute force over paths with
CYK membership (exact on acyclic graphs), Algorithm 1 run as printed on dense
matrices, closed forms (Dyck-1 on a path, transitive closure by BFS, a
right-linear language by BFS on a product automaton), the paper's pairs of
equivalent grammars (Figs. 4a/4b, 5a/5b, 6a/6b, 7a/7b), the CFPQ Data forms
with long right sides against their hand-binarised forms, and a derivation
certificate plus closure check that pins the exact least fixpoint at any
size.
"""

import hashlib
import os
import shutil
import subprocess
import tempfile
from collections import deque

import numpy as np
import pytest

import oracle
from oracle.brute import brute_force, word_in
from oracle.certificate import check_certificate, check_closed
from oracle.naive import naive_closure
from workloads import grammars as G
from workloads import graphs


def grammar_cases(fields=2):
    return {
        "dyck1": (G.DYCK1, ["a", "b"]),
        "alias5a": (G.ALIAS_FIG5A_WCNF, ["a", "d", "a_bar", "d_bar"]),
        "alias5b": (G.ALIAS_FIG5B, ["a", "d", "a_bar", "d_bar"]),
        "pointsto4b": (G.pointsto_fig4b(fields),
                       G.symbols_of(G.pointsto_fig4b(fields))[1]),
        "pointsto4a": (G.pointsto_fig4a(fields),
                       G.symbols_of(G.pointsto_fig4a(fields))[1]),
        "valueflow7a": (G.cscvf_fig7a(fields), G.symbols_of(G.cscvf_fig7a(fields))[1]),
        "valueflow7b": (G.cscvf_fig7b(fields), G.symbols_of(G.cscvf_fig7b(fields))[1]),
        "fsca6a": (G.fsca_fig6a(fields), G.symbols_of(G.fsca_fig6a(fields))[1]),
        "fsca6b": (G.fsca_fig6b(fields), G.symbols_of(G.fsca_fig6b(fields))[1]),
        "transitive": (G.TRANSITIVE, ["a"]),
        "refl_trans": (G.REFLEXIVE_TRANSITIVE, ["a"]),
    }


def long_cases(fields=2):
    """Grammars with right sides of three or more symbols (the paper's CFPQ
    Data forms, plus two textbook ones)."""
    return {
        "alias5a_long": (G.ALIAS_FIG5A, ["a", "d", "a_bar", "d_bar"]),
        "pointsto4a_long": (G.pointsto_fig4a_cfg(fields),
                            G.symbols_of(G.pointsto_fig4a_cfg(fields))[1]),
        "valueflow7a_long": (G.cscvf_fig7a_cfg(fields), G.symbols_of(G.cscvf_fig7a_cfg(fields))[1]),
        "fsca6a_long": (G.fsca_fig6a_cfg(fields), G.symbols_of(G.fsca_fig6a_cfg(fields))[1]),
        "dyck_long": ("S -> a S b S | eps\n", ["a", "b"]),
        "five_symbols": ("S -> a T b T c | d\nT -> S | eps\n", ["a", "b", "c", "d"]),
    }


def assert_same(oracle_res, expected, nts=None):
    for x in nts or oracle_res.order:
        got = oracle_res.pair_set(x)
        assert got == expected[x], (x, sorted(got ^ expected[x])[:10])


@pytest.mark.parametrize("name", list(grammar_cases()))
def test_oracle_equals_brute_force_on_dags(name, oracle_bin):
    text, labels = grammar_cases()[name]
    for seed in range(6):
        g = graphs.random_graph(6, 10, labels, seed=100 + seed, dag=True)
        exact = brute_force(text, g, max_len=g.n)   # every path of a DAG
        assert_same(oracle.solve(text, g), exact)


@pytest.mark.parametrize("name", list(long_cases()))
def test_oracle_equals_brute_force_on_dags_long_rules(name, oracle_bin):
    text, labels = long_cases()[name]
    for seed in range(6):
        g = graphs.random_graph(7, 12, labels, seed=150 + seed, dag=True)
        exact = brute_force(text, g, max_len=g.n)
        assert_same(oracle.solve(text, g), exact)


def balanced(word):
    depth = 0
    for t in word:
        depth += 1 if t == "a" else -1
        if depth < 0:
            return False
    return depth == 0


def test_cyk_long_rules_closed_form():
    # S -> a S b S | eps is the Dyck language: every word over {a, b} up to
    # length 8 is in it exactly when it is balanced
    import itertools
    text = "S -> a S b S | eps\n"
    for n in range(9):
        for word in itertools.product("ab", repeat=n):
            assert word_in(text, "S", list(word)) == balanced(word), word


LONG_EQUIVALENT = [
    ("alias 5a", G.ALIAS_FIG5A, G.ALIAS_FIG5A_WCNF, ["M", "V", "V1", "V2", "V3"],
     lambda s: graphs.alias_graph(300, seed=s)),
    ("points-to 4a", G.pointsto_fig4a_cfg(6), G.pointsto_fig4a(6), ["PT", "FT", "PTH", "FTH", "Al"],
     lambda s: graphs.pointsto_graph(400, fields=6, seed=s)),
    ("value-flow 7a", G.cscvf_fig7a_cfg(5), G.cscvf_fig7a(5), ["A"],
     lambda s: graphs.valueflow_graph(300, calls=5, p_call=0.3, seed=s)),
    ("fsca 6a", G.fsca_fig6a_cfg(3), G.fsca_fig6a(3), ["M", "V", "A", "Abar"],
     lambda s: graphs.random_graph(40, 90, G.symbols_of(G.fsca_fig6b(3))[1], seed=s,
                                   self_loops=True)),
]


@pytest.mark.parametrize("case", LONG_EQUIVALENT, ids=[c[0] for c in LONG_EQUIVALENT])
def test_long_rules_equal_their_binarised_forms(case, oracle_bin):
    # the same grammar with each long right side written out by hand as a
    # chain of helpers (bracketed to the right) on cyclic graphs
    _, long_text, bin_text, shared, make = case
    for seed in range(3):
        g = make(800 + seed)
        r1, r2 = oracle.solve(long_text, g), oracle.solve(bin_text, g)
        for x in shared:
            assert r1.pair_set(x) == r2.pair_set(x), x
        assert any(r1.count[x] for x in shared)


@pytest.mark.parametrize("name", ["dyck1", "alias5a", "valueflow7b", "transitive"])
def test_brute_force_is_a_lower_bound_on_cycles(name, oracle_bin):
    text, labels = grammar_cases()[name]
    for seed in range(4):
        g = graphs.random_graph(5, 9, labels, seed=200 + seed, self_loops=True)
        o = oracle.solve(text, g)
        short = brute_force(text, g, max_len=4)
        longer = brute_force(text, g, max_len=7)
        for x in o.order:
            assert short[x] <= longer[x] <= o.pair_set(x), x


@pytest.mark.parametrize("name", list(grammar_cases()))
def test_oracle_equals_algorithm1_dense(name, oracle_bin):
    text, labels = grammar_cases()[name]
    for seed in range(4):
        g = graphs.random_graph(24, 60, labels, seed=300 + seed, self_loops=True)
        exact, _ = naive_closure(text, g)
        assert_same(oracle.solve(text, g), exact)


@pytest.mark.parametrize("case", ["dyck_er", "alias", "pointsto", "valueflow"])
def test_certificate_pins_the_least_fixpoint(case, oracle_bin):
    if case == "dyck_er":
        text, g = G.DYCK1, graphs.erdos_renyi(256, 1024, seed=0)
    elif case == "alias":
        text, g = G.ALIAS_FIG5A_WCNF, graphs.alias_graph(400, seed=11)
    elif case == "pointsto":
        text, g = G.pointsto_fig4b(8), graphs.pointsto_graph(600, fields=8, seed=12)
    else:
        text, g = G.cscvf_fig7b(4), graphs.valueflow_graph(500, calls=4, seed=13)
    r = oracle.solve(text, g, cert=True)
    try:
        certified = check_certificate(text, g, r.cert_path)   # sound
        for x in r.order:
            assert certified[x] == r.pair_set(x)
        check_closed(text, g, certified)                      # closed + seeded
    finally:
        shutil.rmtree(os.path.dirname(r.cert_path))


def dyck_chain_expected(word):
    """Closed form of Dyck-1 (a = open, b = close) on a labelled path: with
    h the running height (#a - #b), S(i, j) iff h(j) = h(i) and h stays >=
    h(i) on [i, j]; A, B are the a- and b-edges; X = S B."""
    h = np.concatenate([[0], np.cumsum([1 if t == "a" else -1 for t in word])])
    n = len(word) + 1
    S, X = set(), set()
    for i in range(n):
        lo = h[i]
        for j in range(i, n):
            if h[j] < h[i]:
                break
            if h[j] == h[i]:
                S.add((i, j))
    for (i, k) in S:
        if k < len(word) and word[k] == "b":
            X.add((i, k + 1))
    A = {(i, i + 1) for i, t in enumerate(word) if t == "a"}
    B = {(i, i + 1) for i, t in enumerate(word) if t == "b"}
    return {"S": S, "X": X, "A": A, "B": B}


@pytest.mark.parametrize("seed", range(4))
def test_dyck1_on_a_path_closed_form(seed, oracle_bin):
    rng = np.random.default_rng(seed)
    word = ["a" if x else "b" for x in rng.random(600 + 300 * seed) < 0.5]
    g = graphs.chain(word, labels=["a", "b"])
    assert_same(oracle.solve(G.DYCK1, g), dyck_chain_expected(word))


def test_dyck1_without_closing_edges_is_identity(oracle_bin):
    g = graphs.random_graph(50, 200, ["a"], seed=5)
    r = oracle.solve(G.DYCK1, g)
    assert r.pair_set("S") == {(i, i) for i in range(50)}
    assert r.pair_set("X") == set() and r.pair_set("B") == set()


def bfs_closure(n, edges, reflexive):
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
    out = set()
    for s in range(n):
        seen = set()
        dq = deque(adj[s])
        while dq:
            v = dq.popleft()
            if v in seen:
                continue
            seen.add(v)
            dq.extend(adj[v])
        if reflexive:
            seen.add(s)
        out |= {(s, v) for v in seen}
    return out


@pytest.mark.parametrize("reflexive", [False, True])
def test_transitive_closure_by_bfs(reflexive, oracle_bin):
    text = G.REFLEXIVE_TRANSITIVE if reflexive else G.TRANSITIVE
    for seed in range(3):
        g = graphs.random_graph(300, 450, ["a", "z"], seed=400 + seed,
                                self_loops=True)
        a_edges = [(u, v) for u, t, v in g.edges() if t == "a"]
        r = oracle.solve(text, g)
        assert r.pair_set("S") == bfs_closure(g.n, a_edges, reflexive)


def test_right_linear_language_by_product_bfs(oracle_bin):
    # S -> a S | b : words a* b; reachability on graph x {before b, after b}
    text = "S -> a S | b\n"
    for seed in range(3):
        g = graphs.random_graph(200, 500, ["a", "b"], seed=500 + seed,
                                self_loops=True)
        a_adj = [[] for _ in range(g.n)]
        b_adj = [[] for _ in range(g.n)]
        for u, t, v in g.edges():
            (a_adj if t == "a" else b_adj)[u].append(v)
        exp = set()
        for s in range(g.n):
            seen = {s}
            dq = deque([s])
            while dq:
                u = dq.popleft()
                for v in a_adj[u]:
                    if v not in seen:
                        seen.add(v)
                        dq.append(v)
            exp |= {(s, w) for u in seen for w in b_adj[u]}
        assert oracle.solve(text, g).pair_set("S") == exp


EQUIVALENT = [
    ("alias 5a/5b", G.ALIAS_FIG5A_WCNF, G.ALIAS_FIG5B, ["M"],
     lambda s: graphs.alias_graph(300, seed=s)),
    ("points-to 4a/4b", G.pointsto_fig4a(6), G.pointsto_fig4b(6), ["PT", "FT"],
     lambda s: graphs.pointsto_graph(400, fields=6, seed=s)),
    ("value-flow 7a/7b", G.cscvf_fig7a(5), G.cscvf_fig7b(5), ["A"],
     lambda s: graphs.valueflow_graph(300, calls=5, p_call=0.3, seed=s)),
]


@pytest.mark.parametrize("case", EQUIVALENT, ids=[c[0] for c in EQUIVALENT])
def test_paper_equivalent_grammars_agree(case, oracle_bin):
    _, text1, text2, shared, make = case
    for seed in range(3):
        g = make(600 + seed)
        r1, r2 = oracle.solve(text1, g), oracle.solve(text2, g)
        for x in shared:
            assert r1.pair_set(x) == r2.pair_set(x), x
        assert any(r1.count[x] for x in shared)


def test_fsca_6a_6b_agree(oracle_bin):
    labels = G.symbols_of(G.fsca_fig6b(3))[1]
    for seed in range(3):
        g = graphs.random_graph(40, 90, labels, seed=700 + seed, self_loops=True)
        r1, r2 = oracle.solve(G.fsca_fig6a(3), g), oracle.solve(G.fsca_fig6b(3), g)
        for x in ["M", "V", "A", "Abar"]:
            assert r1.pair_set(x) == r2.pair_set(x), x


def test_cyk_membership_textbook_words():
    assert word_in(G.DYCK1, "S", [])
    assert word_in(G.DYCK1, "S", list("aabbab"))
    assert not word_in(G.DYCK1, "S", list("aab"))
    assert not word_in(G.DYCK1, "S", list("ba"))
    assert word_in(G.ALIAS_FIG5B, "M", ["d_bar", "d"])
    assert word_in(G.ALIAS_FIG5B, "M", ["d_bar", "a_bar", "a", "d"])
    assert not word_in(G.ALIAS_FIG5B, "M", ["d_bar", "a"])


def test_digest_is_sha256_of_sorted_pairs(oracle_bin):
    g = graphs.erdos_renyi(128, 400, seed=9)
    r = oracle.solve(G.DYCK1, g)
    for x in r.order:
        p = r.pairs[x]
        buf = np.ascontiguousarray(p, dtype="<u4").tobytes()
        assert hashlib.sha256(buf).hexdigest() == r.digest[x]
        assert r.count[x] == p.shape[0]
        assert np.all(np.diff(p[:, 0].astype(np.int64) * 10**6 + p[:, 1]) > 0)


def test_golden_files_reproduce(oracle_bin):
    import json
    from tests.golden.make_goldens import GOLDENS
    for name in ["dyck_er_256", "pointsto_4k"]:
        with open(os.path.join(os.path.dirname(__file__), "golden", f"{name}.json")) as f:
            gold = json.load(f)
        text, g = GOLDENS[name]()
        r = oracle.solve(text, g, pairs=False)
        assert r.count == gold["count"] and r.digest == gold["sha256"]


# A mistake planted in the oracle (compiled on the CPU from the same source
# with one change) must be caught by the pins above.
MUTANTS = {
    "drop_right_products": ("for (uint32_t t = 0; t < n_right[y]; t++) {",
                            "for (uint32_t t = 0; t < 0 * n_right[y]; t++) {"),
    "transposed_operand": ("const vset_t *zr = row_set[z][j];",
                           "const vset_t *zr = col_set[z][j];"),
    "eps_only_first_vertex": ("for (uint32_t i = 0; i < n_vert; i++) add_fact(rules[r].lhs, i, i, r, UINT32_MAX);",
                              "for (uint32_t i = 0; i < 1 && i < n_vert; i++) add_fact(rules[r].lhs, i, i, r, UINT32_MAX);"),
    "unit_rules_ignored": ("add_fact(rules[r].lhs, i, j, r, UINT32_MAX);\n        }",
                           "(void)r;\n        }"),
    "long_rule_reversed": ("add_rule(R_BIN, p, left, sym_lookup(tok[q], 1));",
                           "add_rule(R_BIN, p, sym_lookup(tok[q], 1), left);"),
    "long_rule_last_dropped": ("add_rule(R_BIN, x, left, sym_lookup(tok[nt - 1], 1));",
                               "add_rule(R_UNIT, x, left, 0);"),
}


@pytest.mark.parametrize("mutant", list(MUTANTS))
def test_planted_oracle_mistakes_are_caught(mutant, oracle_bin, monkeypatch):
    src = open(oracle.SOURCE).read()
    old, new = MUTANTS[mutant]
    assert old in src
    tmp = tempfile.mkdtemp(prefix="cflr_mutant_")
    path = os.path.join(tmp, "mutant.c")
    exe = os.path.join(tmp, "mutant")
    with open(path, "w") as f:
        f.write(src.replace(old, new, 1))
    subprocess.run(["gcc", "-O1", "-std=c11", "-o", exe, path], check=True,
                   capture_output=True)
    monkeypatch.setattr(oracle, "BINARY", exe)
    monkeypatch.setattr(oracle, "_ensure_built", lambda: None)
    caught = False
    try:
        cases = {**grammar_cases(), **long_cases()}
        for name in ["dyck1", "alias5a", "alias5b", "fsca6b", "refl_trans", "dyck_long",
                     "five_symbols"]:
            text, labels = cases[name]
            for seed in range(3):
                g = graphs.random_graph(6, 10, labels, seed=100 + seed, dag=True)
                exact = brute_force(text, g, max_len=g.n)
                r = oracle.solve(text, g)
                if any(r.pair_set(x) != exact[x] for x in r.order):
                    caught = True
                    break
            if caught:
                break
    finally:
        for fn in os.listdir(tmp):
            os.unlink(os.path.join(tmp, fn))
        os.rmdir(tmp)
    assert caught, f"pins did not catch mutant {mutant}"


# The certificate checker must reject certificates with a planted defect, and
# the closure check results with one pair or seed missing; a checker that
# accepted anything would pass the test above.

def _read_raw_cert(path):
    import struct
    with open(path, "rb") as f:
        data = f.read()
    off = 0
    (nsym,) = struct.unpack_from("<I", data, off)
    off += 4
    syms = []
    for _ in range(nsym):
        (k,) = struct.unpack_from("<I", data, off)
        name = data[off + 4: off + 4 + k]
        (nt,) = struct.unpack_from("<I", data, off + 4 + k)
        syms.append((name, nt))
        off += 8 + k
    (nr,) = struct.unpack_from("<I", data, off)
    off += 4
    rules = np.frombuffer(data, dtype="<u4", count=4 * nr, offset=off).reshape(nr, 4).copy()
    off += 16 * nr
    (nf,) = struct.unpack_from("<Q", data, off)
    off += 8
    facts = np.frombuffer(data, dtype="<u4", count=5 * nf, offset=off).reshape(nf, 5).copy()
    return syms, rules, facts


def _write_raw_cert(path, syms, rules, facts):
    import struct
    with open(path, "wb") as f:
        f.write(struct.pack("<I", len(syms)))
        for name, nt in syms:
            f.write(struct.pack("<I", len(name)) + name + struct.pack("<I", nt))
        f.write(struct.pack("<I", rules.shape[0]) + rules.astype("<u4").tobytes())
        f.write(struct.pack("<Q", facts.shape[0]) + facts.astype("<u4").tobytes())


def test_certificate_checker_rejects_planted_defects(oracle_bin):
    text, g = G.ALIAS_FIG5A_WCNF, graphs.alias_graph(300, seed=11)
    r = oracle.solve(text, g, cert=True)
    tmp = os.path.dirname(r.cert_path)
    try:
        syms, rules, facts = _read_raw_cert(r.cert_path)
        good = os.path.join(tmp, "good.bin")
        _write_raw_cert(good, syms, rules, facts)
        certified = check_certificate(text, g, good)  # the rewrite itself is faithful
        check_closed(text, g, certified)
        NONE = 0xFFFFFFFF
        binary = [t for t in range(facts.shape[0]) if facts[t, 3] != NONE and rules[facts[t, 3], 0] == 2]
        assert binary
        t = binary[len(binary) // 2]
        s, i, j, rule, mid = facts[t].tolist()
        left = rules[rule, 2]
        premise = next(u for u in range(t) if facts[u, 0] == left and facts[u, 1] == i and facts[u, 2] == mid)
        bad = os.path.join(tmp, "bad.bin")
        defects = {
            # a premise of a derived fact dropped from the certificate
            "dropped premise": np.delete(facts, premise, axis=0),
            # the derived fact placed before its premise
            "premise after use": np.concatenate([facts[:premise], facts[t:t + 1], facts[premise:t], facts[t + 1:]]),
        }
        wrong_mid = facts.copy()
        wrong_mid[t, 4] = (mid + 1) % g.n if not any(
            facts[u, 0] == left and facts[u, 1] == i and facts[u, 2] == (mid + 1) % g.n for u in range(t)) else g.n
        defects["wrong midpoint"] = wrong_mid
        wrong_head = facts.copy()
        other = next(x for x in range(len(syms)) if syms[x][1] == 1 and x != s)
        wrong_head[t, 0] = other
        defects["head of another symbol"] = wrong_head
        fake_edge = facts.copy()
        first_edge = next(u for u in range(facts.shape[0]) if facts[u, 3] == NONE)
        fake_edge[first_edge, 2] = (facts[first_edge, 2] + 1) % g.n
        defects["edge not in the graph"] = fake_edge
        duplicated = np.concatenate([facts, facts[t:t + 1]])
        defects["fact listed twice"] = duplicated
        for name, f in defects.items():
            _write_raw_cert(bad, syms, rules, f)
            with pytest.raises(AssertionError):
                check_certificate(text, g, bad)
            print("rejected:", name)
        # closure: one derived pair missing, one eps seed missing
        x = next(x for x in r.order if len(certified[x]) > 1 and x != "V")
        short = {k: set(v) for k, v in certified.items()}
        short[x].discard(next(iter(sorted(certified[x]))))
        with pytest.raises(AssertionError):
            check_closed(text, g, short)
        no_eps = {k: set(v) for k, v in certified.items()}
        no_eps["V"].discard((0, 0))
        with pytest.raises(AssertionError):
            check_closed(text, g, no_eps)
    finally:
        shutil.rmtree(tmp)
