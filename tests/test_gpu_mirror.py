"""Mirror plans of the sparse engine (cflr_opts.mirror): on a grammar closed
under reversal and a graph that holds every edge with its reverse, one
production of each mirror pair keeps its product and the other's new pairs
are the transposes.  The result must be the oracle's pair for pair, with the
plan and without it; a graph whose seeds are not their own mirror image must
make the library solve without the plan.  Every call goes through libcflr's
C interface."""

import numpy as np
import pytest

import oracle
import workloads
from workloads import grammars as G
from workloads import graphs
from workloads.graphs import Graph

from tests.test_gpu_parity import assert_matches_oracle
from tests.test_gpu_sparse import mode  # noqa: F401  (the product paths as a fixture)

pytestmark = pytest.mark.gpu

SPARSE = 2
MIRROR_AUTO, MIRROR_OFF = 0, 1


def cflr():
    import paper_2401_11029_amd as m
    return m


def solve(ctx, text, g, **kw):
    m = cflr()
    r = m.solve(ctx, m.Grammar(text), m.Graph.from_workload(ctx, g), storage=SPARSE, **kw)
    assert r.stats()["storage"] == SPARSE
    return r


def mirror_pairs_hold(r, pairs):
    """x's pairs are the transposes of y's for every (x, y) of `pairs`."""
    for x, y in pairs:
        sx, dx = r.pairs(x)
        sy, dy = r.pairs(y)
        a = set(zip(sx.tolist(), dx.tolist()))
        b = set(zip(dy.tolist(), sy.tolist()))
        assert a == b, (x, y)


@pytest.mark.parametrize("fields,n", [(64, 3000), (8, 2500)])
def test_mirror_plan_equals_oracle(ctx, fields, n, mode):  # noqa: F811
    text = G.pointsto_fig4b(fields)
    g = graphs.pointsto_graph(n, fields=fields, seed=31 + fields)
    print(f"mirror pointsto fields={fields} n={n} mode={mode}", flush=True)
    r = solve(ctx, text, g)
    assert r.stats()["mirror"] == 1
    assert_matches_oracle(r, text, g, f"mirror fields={fields}")
    mirror_pairs_hold(r, [("PT", "FT")] + [(f"LP_{i}", f"FL_{i}") for i in range(fields)]
                      + [(f"LPFS_{i}", f"SPFL_{i}") for i in range(fields)])
    st = r.stats()
    off = solve(ctx, text, g, mirror=MIRROR_OFF)
    assert off.stats()["mirror"] == 0
    assert off.stats()["total_pairs"] == st["total_pairs"] and off.stats()["rounds"] == st["rounds"]
    assert off.counts() == r.counts()
    off.close()
    r.close()


def test_mirror_plan_with_overflow_reruns(ctx):
    text = G.pointsto_fig4b(8)
    g = graphs.pointsto_graph(2000, fields=8, seed=40)
    print("mirror with a 64-pair buffer", flush=True)
    r = solve(ctx, text, g, delta_capacity=64)
    st = r.stats()
    assert st["mirror"] == 1 and st["reruns"] > 0
    assert_matches_oracle(r, text, g, "mirror reruns")
    r.close()


def drop_edge(g, keep):
    return Graph(g.n, g.src[keep].copy(), g.dst[keep].copy(), g.label[keep].copy(), list(g.label_names),
                 dict(g.meta, edited=True))


def test_mirror_rejected_without_every_reverse_edge(ctx):
    text = G.pointsto_fig4b(8)
    g = graphs.pointsto_graph(1500, fields=8, seed=41)
    # one load edge loses its reverse (load_bar) edge: seeds of FL's wrapper
    # are no longer the transposes of LP's
    names = g.label_names
    bar = np.isin(g.label, [names.index(f"load_bar_{i}") for i in range(8)])
    victim = int(np.flatnonzero(bar)[0])
    keep = np.ones(g.m, dtype=bool)
    keep[victim] = False
    h = drop_edge(g, keep)
    print("mirror rejected: one reverse edge missing", flush=True)
    r = solve(ctx, text, h)
    assert r.stats()["mirror"] == 0
    assert_matches_oracle(r, text, h, "asymmetric")
    r.close()
    # a label without a t_bar partner is its own reverse: the plan needs
    # its edges both ways.  R -> X R mirrors R -> R Y (X <-> Y, c <-> c).
    text2 = "R -> c | X R | R Y\nX -> c\nY -> c\n"
    assert cflr().Grammar(text2).info()["mirror_skipped"] == 1
    rng = np.random.Generator(np.random.PCG64(43))
    u = rng.integers(0, 400, 900).astype(np.uint32)
    v = rng.integers(0, 400, 900).astype(np.uint32)
    for both, want in ((True, 1), (False, 0)):
        src = np.concatenate([u, v]) if both else u
        dst = np.concatenate([v, u]) if both else v
        h2 = Graph(400, src, dst, np.zeros(src.shape[0], np.uint32), ["c"], {"kind": "test"})
        print(f"own-reverse label, both directions={both}", flush=True)
        r2 = solve(ctx, text2, h2)
        assert r2.stats()["mirror"] == want
        assert_matches_oracle(r2, text2, h2, f"own reverse {both}")
        r2.close()


def test_self_mirrored_grammar(ctx):
    # S and the eps rule are their own mirror, T <-> T2, A <-> B; on a graph
    # with each a edge reversed as a_bar the plan applies
    text = "S -> eps | A T | T2 B\nT -> S B\nT2 -> A S\nA -> a\nB -> a_bar\n"
    rng = np.random.Generator(np.random.PCG64(42))
    n, m = 300, 700
    u = rng.integers(0, n, m).astype(np.uint32)
    v = rng.integers(0, n, m).astype(np.uint32)
    g = Graph(n, np.concatenate([u, v]), np.concatenate([v, u]),
              np.concatenate([np.zeros(m, np.uint32), np.ones(m, np.uint32)]), ["a", "a_bar"], {"kind": "test"})
    print("self-mirrored grammar", flush=True)
    r = solve(ctx, text, g)
    assert r.stats()["mirror"] == 1
    assert_matches_oracle(r, text, g, "self mirror")
    mirror_pairs_hold(r, [("S", "S"), ("T", "T2"), ("A", "B")])
    r.close()


def test_mirror_plan_on_the_points_to_workload_shape(ctx):
    text, g = workloads.config("pointsto_200k", n=6000)
    print("mirror pointsto_200k generator at n=6000", flush=True)
    r = solve(ctx, text, g)
    assert r.stats()["mirror"] == 1
    o = oracle.solve(text, g, pairs=False, digest=True)
    from tests.test_gpu_parity import digest
    for x in o.order:
        s, d = r.pairs(x)
        assert s.shape[0] == o.count[x] and digest(s, d) == o.digest[x], x
    r.close()
