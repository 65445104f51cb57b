"""Full-size parity: the 50,000-vertex memory-alias configuration, the
200,000-vertex field-sensitive points-to configuration (Fig. 4b, 64 fields,
386 non-terminals), value flow at the size of Table 3's povray graph and
the 256-graph memory-alias batch, each solved with the launch configuration
bench.py times (default options), against the oracle's stored
per-non-terminal counts and SHA-256 digests (tests/golden/alias_50k.json,
pointsto_200k.json, valueflow_346k.json, alias_batch_le8k.json, written by
tests/golden/make_goldens.py)."""

import hashlib
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "alias_50k.json")
GOLDEN_PT = os.path.join(os.path.dirname(__file__), "golden", "pointsto_200k.json")
GOLDEN_BATCH = os.path.join(os.path.dirname(__file__), "golden", "alias_batch_le8k.json")
GOLDEN_VF = os.path.join(os.path.dirname(__file__), "golden", "valueflow_346k.json")


def sha_of_pairs(s, d, chunk=1 << 26):
    h = hashlib.sha256()
    buf = np.empty((min(chunk, s.shape[0]), 2), dtype="<u4")
    for a in range(0, s.shape[0], chunk):
        b = min(a + chunk, s.shape[0])
        v = buf[: b - a]
        v[:, 0] = s[a:b]
        v[:, 1] = d[a:b]
        h.update(v.tobytes())
    return h.hexdigest()


def test_alias_50k_matches_oracle_digests(ctx):
    import paper_2401_11029_amd as cflr
    with open(GOLDEN) as f:
        gold = json.load(f)
    text, g = workloads.config("alias_50k")
    r = cflr.solve(ctx, cflr.Grammar(text), cflr.Graph.from_workload(ctx, g))
    assert r.grammar.nonterminals == gold["order"]
    st = r.stats()
    assert st["total_pairs"] == gold["total"]
    print(f"alias_50k: {st['total_pairs']} pairs, {st['rounds']} rounds, "
          f"{st['fixpoint_ms']:.0f} ms", flush=True)
    for x in gold["order"]:
        assert r.count(x) == gold["count"][x], x
        s, d = r.pairs(x)
        assert sha_of_pairs(s, d) == gold["sha256"][x], x
        del s, d


def test_pointsto_200k_matches_oracle_digests(ctx):
    import paper_2401_11029_amd as cflr
    with open(GOLDEN_PT) as f:
        gold = json.load(f)
    text, g = workloads.config("pointsto_200k")
    r = cflr.solve(ctx, cflr.Grammar(text), cflr.Graph.from_workload(ctx, g))
    st = r.stats()
    print(f"pointsto_200k: {st['total_pairs']} pairs, {st['rounds']} rounds, "
          f"{st['fixpoint_ms']:.0f} ms, storage {st['storage']}", flush=True)
    assert st["storage"] == 2  # the dense matrices would not fit: sparse storage
    assert st["mirror"] == 1   # Fig. 4b on a graph with every reverse edge: the mirror plan
    assert r.grammar.nonterminals == gold["order"]
    assert st["total_pairs"] == gold["total"]
    for x in gold["order"]:
        assert r.count(x) == gold["count"][x], x
        s, d = r.pairs(x)
        assert sha_of_pairs(s, d) == gold["sha256"][x], x
        del s, d
    r.close()
    # every production with its own product: the same counts
    r = cflr.solve(ctx, cflr.Grammar(text), cflr.Graph.from_workload(ctx, g), mirror=1)
    st = r.stats()
    print(f"pointsto_200k without the mirror plan: {st['fixpoint_ms']:.0f} ms", flush=True)
    assert st["mirror"] == 0 and st["total_pairs"] == gold["total"]
    assert r.counts() == gold["count"]
    r.close()


def test_valueflow_346k_matches_oracle_digests(ctx):
    """Value flow (Fig. 7b, 64 call sites) at the vertex and edge counts of
    Table 3's povray graph: 1.54e9 pairs on sparse storage (chosen by the
    default), every non-terminal's count and digest against the oracle's."""
    import paper_2401_11029_amd as cflr
    with open(GOLDEN_VF) as f:
        gold = json.load(f)
    text, g = workloads.config("valueflow_346k")
    r = cflr.solve(ctx, cflr.Grammar(text), cflr.Graph.from_workload(ctx, g))
    st = r.stats()
    print(f"valueflow_346k: {st['total_pairs']} pairs, {st['rounds']} rounds, "
          f"{st['fixpoint_ms']:.0f} ms, storage {st['storage']}", flush=True)
    assert st["storage"] == 2
    assert r.grammar.nonterminals == gold["order"]
    assert st["total_pairs"] == gold["total"]
    for x in gold["order"]:
        assert r.count(x) == gold["count"][x], x
        s, d = r.pairs(x)
        assert sha_of_pairs(s, d) == gold["sha256"][x], x
        del s, d
    r.close()


def test_alias_batch_matches_oracle_digests(ctx):
    """One batched call over the whole 256-graph memory-alias batch (n
    log-uniform in [1000, 40000]), as the batched bench mode makes it; each
    of its 141 graphs of at most 8,000 vertices against the oracle's counts
    and digests for every non-terminal (the oracle solved each alone)."""
    import paper_2401_11029_amd as cflr
    from workloads import grammars, graphs
    with open(GOLDEN_BATCH) as f:
        gold = json.load(f)
    gs = graphs.alias_batch(256)
    gr = cflr.Grammar(grammars.ALIAS_FIG5A_WCNF)
    objs = [cflr.Graph.from_workload(ctx, g) for g in gs]
    print("alias batch: one solve_batch call over 256 graphs", flush=True)
    res = cflr.solve_batch(ctx, gr, objs)
    try:
        assert len(gold["graphs"]) == sum(1 for g in gs if g.n <= 8000)
        for key, want in gold["graphs"].items():
            q = int(key)
            assert (gs[q].n, gs[q].m) == (want["n"], want["m"]), q
            r = res[q]
            assert r.grammar.nonterminals == want["order"]
            assert r.counts() == want["count"], q
            for x in want["order"]:
                s, d = r.pairs(x)
                assert sha_of_pairs(s, d) == want["sha256"][x], (q, x)
    finally:
        for r in res:
            r.close()


def test_pointsto_200k_witnesses_on_a_sample(ctx):
    """Witnesses at full size: the solve with witnesses gives the oracle's
    counts; for 2,000 sampled pairs of each of eight non-terminals (both
    sides of field 0 and PT, FT), the witness's premises are pairs of the
    result (or edges of the graph) derived in earlier rounds -- the
    soundness condition of a derivation, checked one pair at a time."""
    import paper_2401_11029_amd as cflr
    with open(GOLDEN_PT) as f:
        gold = json.load(f)
    text, g = workloads.config("pointsto_200k")
    gr = cflr.Grammar(text)
    r = cflr.solve(ctx, gr, cflr.Graph.from_workload(ctx, g), witness=1)
    st = r.stats()
    print(f"pointsto_200k with witnesses: {st['rounds']} rounds, {st['fixpoint_ms']:.0f} ms", flush=True)
    assert st["total_pairs"] == gold["total"]
    assert st["mirror"] == 1  # the mirrored pairs carry the mirror production
    syms = gr.symbols
    U = len(gr.nonterminals)
    n = g.n
    edges = {}
    for name in set(g.label_names):
        k = g.label_names.index(name)
        sel = g.label == k
        edges[name] = np.unique(g.src[sel].astype(np.uint64) * n + g.dst[sel].astype(np.uint64))
    cache = {}

    def keys_and_rounds(x):
        # sorted pair keys of non-terminal x and the round of each
        if x not in cache:
            s, d = r.pairs(x)
            _, _, _, rd = r.witness(x)
            cache[x] = (s.astype(np.uint64) * n + d.astype(np.uint64), rd)
        return cache[x]

    def premise_round(sym, i, j):
        key = np.uint64(i) * np.uint64(n) + np.uint64(j)
        if sym >= U:                                   # a terminal: an edge, present before round 1
            e = edges.get(syms[sym])
            ok = e is not None and np.searchsorted(e, key) < e.size and e[np.searchsorted(e, key)] == key
            return 0 if ok else None
        keys, rd = keys_and_rounds(syms[sym])
        p = np.searchsorted(keys, key)
        return int(rd[p]) if p < keys.size and keys[p] == key else None

    rng = np.random.Generator(np.random.PCG64(7))
    for x in ("PT", "FT", "LP_0", "FS_0", "LPFS_0", "SP_0", "FL_0", "SPFL_0"):
        keys, rd = keys_and_rounds(x)
        left, right, mid, _ = r.witness(x)
        assert keys.size == gold["count"][x], x
        for p in rng.choice(keys.size, size=min(2000, keys.size), replace=False).tolist():
            i, j = int(keys[p] // n), int(keys[p] % n)
            if right[p] == 0xFFFFFFFF:                 # an edge x -> t
                assert left[p] != 0xFFFFFFFF and premise_round(int(left[p]), i, j) == 0, (x, i, j)
                continue
            k = int(mid[p])
            ra = premise_round(int(left[p]), i, k)
            rb = premise_round(int(right[p]), k, j)
            assert ra is not None and rb is not None, (x, i, j, k)
            assert ra < rd[p] and rb < rd[p], (x, i, j, k, ra, rb, int(rd[p]))
    r.close()
