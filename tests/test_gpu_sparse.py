"""The sparse storage engine (adjacency lists + hash set; cflr_opts.storage =
CFLR_STORAGE_SPARSE) against the CPU oracle, pair for pair (tolerance 0).
Every call goes through libcflr's C interface."""

import json
import os

import numpy as np
import pytest

import oracle
import workloads
from workloads import grammars as G
from workloads import graphs

from tests.test_gpu_parity import SWEEP, assert_matches_oracle, digest, GOLDEN

pytestmark = pytest.mark.gpu

SPARSE = 2

# The product's paths: buckets of new pairs sorted by key, heavy ones through
# an LDS bit set (the default threshold), every bucket heavy, every bucket
# heavy with small uses sent straight to the hash set, every bucket heavy
# without clearing the head's own pairs from the bit set, every bucket
# light, and the unsorted product.
MODES = {
    "grouped": {},
    "all_heavy": {"CFLR_SPARSE_HEAVY": "1", "CFLR_SPARSE_DIRECT": "0", "CFLR_SPARSE_ROWF": str(2**32 - 1)},
    "heavy_direct": {"CFLR_SPARSE_HEAVY": "1", "CFLR_SPARSE_DIRECT": "200"},
    "heavy_no_row_clear": {"CFLR_SPARSE_HEAVY": "1", "CFLR_SPARSE_DIRECT": "0", "CFLR_SPARSE_ROWF": "0"},
    "all_light": {"CFLR_SPARSE_HEAVY": str(1 << 62)},
    "ungrouped": {"CFLR_SPARSE_UNGROUPED": "1"},
}

KNOBS = ("CFLR_SPARSE_HEAVY", "CFLR_SPARSE_UNGROUPED", "CFLR_SPARSE_DIRECT", "CFLR_SPARSE_ROWF")


@pytest.fixture(params=list(MODES))
def mode(request, monkeypatch):
    for k in KNOBS:
        monkeypatch.delenv(k, raising=False)
    for k, v in MODES[request.param].items():
        monkeypatch.setenv(k, v)
    return request.param


def cflr():
    import paper_2401_11029_amd as m
    return m


def sparse_solve(ctx, text, g, **kw):
    m = cflr()
    r = m.solve(ctx, m.Grammar(text), m.Graph.from_workload(ctx, g), storage=SPARSE, **kw)
    assert r.stats()["storage"] == SPARSE
    return r


@pytest.mark.parametrize("case", SWEEP, ids=[c[0] for c in SWEEP])
def test_sparse_random_sweep(ctx, case, mode):
    name, text, labels = case
    for k, (n, m) in enumerate([(1, 3), (5, 12), (33, 90), (64, 200), (65, 260), (200, 600)]):
        g = graphs.random_graph(n, m, labels, seed=1000 + 17 * k, self_loops=True)
        print(f"sparse sweep {name} n={n} m={m} mode={mode}", flush=True)
        assert_matches_oracle(sparse_solve(ctx, text, g), text, g, f"{name} n={n}")


@pytest.mark.parametrize("name", ["pointsto_4k", "pointsto_12k", "alias_8k"])
def test_sparse_golden_digests(ctx, name, mode):
    from tests.golden.make_goldens import GOLDENS
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        gold = json.load(f)
    text, g = GOLDENS[name]()
    print(f"sparse golden {name} mode={mode}", flush=True)
    r = sparse_solve(ctx, text, g)
    assert r.grammar.nonterminals == gold["order"]
    for x in gold["order"]:
        s, d = r.pairs(x)
        assert s.shape[0] == gold["count"][x], x
        assert digest(s, d) == gold["sha256"][x], x


def test_sparse_long_lists_read_out_in_order(ctx, mode):
    # rows of far more than 2,048 pairs take the bit-set readout path: the
    # transitive closure of a dense random relation
    g = graphs.random_graph(3000, 30000, ["a"], seed=5150, self_loops=True)
    r = sparse_solve(ctx, G.TRANSITIVE, g)
    assert r.count("S") > 3000 * 2048
    assert_matches_oracle(r, G.TRANSITIVE, g, "long rows")


def test_sparse_edge_cases(ctx):
    g = graphs.make_graph(0, [], label_names=["a", "b"])
    r = sparse_solve(ctx, G.DYCK1, g)
    assert all(v == 0 for v in r.counts().values())
    g = graphs.make_graph(70, [], label_names=["a"])
    r = sparse_solve(ctx, G.DYCK1, g)
    assert r.pair_set("S") == {(i, i) for i in range(70)}
    assert r.count("X") == 0
    g = graphs.make_graph(4, [(0, "a", 1), (0, "a", 1), (1, "zz", 2), (1, "b", 3), (2, "b", 2)],
                          label_names=["a", "b", "zz"])
    assert_matches_oracle(sparse_solve(ctx, G.DYCK1, g), G.DYCK1, g)
    text = "A -> a\nB -> b | a\n"
    g = graphs.random_graph(50, 120, ["a", "b"], seed=3)
    assert_matches_oracle(sparse_solve(ctx, text, g), text, g)
    r = sparse_solve(ctx, "E -> eps\n", graphs.random_graph(9, 5, ["a"], seed=1))
    assert r.pair_set("E") == {(i, i) for i in range(9)}


def test_sparse_overflows_rerun_exactly(ctx, mode):
    # a 64-pair new-pair buffer and the smallest pool and hash table: every
    # round overflows at least once and is re-run; the result is unchanged
    g = graphs.alias_graph(2500, seed=77)
    r = sparse_solve(ctx, G.ALIAS_FIG5A_WCNF, g, delta_capacity=64)
    assert r.stats()["reruns"] > 0
    assert_matches_oracle(r, G.ALIAS_FIG5A_WCNF, g, "overflow")
    text, g = workloads.config("pointsto_200k", n=3000)
    r = sparse_solve(ctx, text, g, delta_capacity=100)
    assert r.stats()["reruns"] > 0
    assert_matches_oracle(r, text, g, "overflow points-to")


def test_sparse_round_limit(ctx):
    import ctypes as C
    m = cflr()
    L = m.lib()
    text, g = G.ALIAS_FIG5A_WCNF, graphs.alias_graph(2000, seed=11)
    gr = m.Grammar(text)
    graph = m.Graph.from_workload(ctx, g)
    o = m.opts(max_rounds=2, storage=SPARSE)
    h = C.c_void_p()
    assert L.cflr_solve(ctx._h, gr._h, graph._h, C.byref(o), C.byref(h)) == 6  # CFLR_ETIMEOUT
    res = m.Result(h, gr)
    orc = oracle.solve(text, g)
    for x in orc.order:
        assert res.pair_set(x) <= orc.pair_set(x), x
    assert sum(res.counts().values()) < sum(orc.count.values())
    res.close()


def test_sparse_and_dense_agree_and_repeat(ctx):
    m = cflr()
    text, g = workloads.config("pointsto_200k", n=6000)
    gr = m.Grammar(text)
    graph = m.Graph.from_workload(ctx, g)
    dense = m.solve(ctx, gr, graph, storage=1)
    assert dense.stats()["storage"] == 1
    want = {x: digest(*dense.pairs(x)) for x in gr.nonterminals}
    for _ in range(2):
        r = m.solve(ctx, gr, graph, storage=SPARSE)
        assert {x: digest(*r.pairs(x)) for x in gr.nonterminals} == want


def test_sparse_device_pointer_readout(ctx):
    import torch
    g = graphs.erdos_renyi(300, 900, seed=8)
    r = sparse_solve(ctx, G.DYCK1, g)
    dev = torch.device("cuda", 0)
    s, d = r.pairs("S", device=dev)
    hs, hd = r.pairs("S")
    assert np.array_equal(s.cpu().numpy().astype(np.uint32), hs)
    assert np.array_equal(d.cpu().numpy().astype(np.uint32), hd)


def test_sparse_rejects_the_naive_variant(ctx):
    m = cflr()
    with pytest.raises(m.CflrError) as e:
        sparse_solve(ctx, G.DYCK1, graphs.erdos_renyi(30, 60, seed=1), semi_naive=0)
    assert e.value.status == 7


def test_sparse_largest_vertex_ids(ctx):
    # the most vertices sparse storage takes (2^24 - 1): pairs whose vertex
    # ids fill the 24-bit fields of the keys and sorted entries
    n = (1 << 24) - 1
    rng = np.random.Generator(np.random.PCG64(31))
    ids = np.concatenate([[0, 1], np.arange(n - 400, n)]).astype(np.int64)
    triples = [(int(rng.choice(ids)), "a" if rng.random() < 0.5 else "b", int(rng.choice(ids)))
               for _ in range(1200)]
    g = graphs.make_graph(n, triples, label_names=["a", "b"])
    text = "S -> A B | A X | S S\nX -> S B\nA -> a\nB -> b\n"
    print(f"sparse largest ids n={n}", flush=True)
    assert_matches_oracle(sparse_solve(ctx, text, g), text, g, "n = 2^24 - 1")
    m = cflr()
    with pytest.raises(m.CflrError) as e:
        sparse_solve(ctx, text, graphs.make_graph(1 << 24, triples, label_names=["a", "b"]))
    assert e.value.status == 7
