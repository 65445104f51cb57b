"""Single-path semantics (the footnote to Section 5: the fixpoint over a
semiring that carries one derivation per pair): witnesses recorded by the
sparse engine (cflr_opts.witness = 1) are turned into a derivation
certificate and checked by oracle/certificate.py (every pair derived from
earlier pairs by a rule of the grammar text: sound) and by its closure
check (seeded and closed), and the pairs equal the oracle's.  Every call
goes through libcflr's C interface."""

import os

import numpy as np
import pytest

import oracle
import workloads
from oracle.certificate import check_certificate, check_closed
from workloads import grammars as G
from workloads import graphs

from tests.witness_cert import NONE, write_certificate

pytestmark = pytest.mark.gpu

CASES = [
    # Dyck-1 (eps, terminal and binary rules)
    ("dyck", G.DYCK1, lambda: graphs.erdos_renyi(300, 900, seed=21)),
    # memory alias, Fig. 5a binarised by hand: the unit rule V2 -> M makes
    # the library copy M's production into V2
    ("alias", G.ALIAS_FIG5A_WCNF, lambda: graphs.alias_graph(1500, seed=22)),
    # Fig. 5b, hand WCNF
    ("alias5b", G.ALIAS_FIG5B, lambda: graphs.alias_graph(1200, seed=23)),
    # points-to, Fig. 4b at 64 fields (386 non-terminals)
    ("pointsto", None, lambda: workloads.config("pointsto_200k", n=3000)),
]


def cflr():
    import paper_2401_11029_amd as m
    return m


def solve_with_witnesses(ctx, text, g):
    m = cflr()
    gr = m.Grammar(text)
    r = m.solve(ctx, gr, m.Graph.from_workload(ctx, g), witness=1)
    assert r.stats()["storage"] == 2
    out = {}
    for x in gr.nonterminals:
        s, d = r.pairs(x)
        out[x] = (s, d) + r.witness(x)
    return gr, r, out


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_witnesses_certify_the_fixpoint(ctx, tmp_path, case):
    name, text, make = case
    g = make()
    if text is None:
        text, g = g
    print(f"witness {name} n={g.n} m={g.m}", flush=True)
    gr, r, res = solve_with_witnesses(ctx, text, g)
    if name == "pointsto":  # Fig. 4b: half of the pairs come from the mirror plan's transposes
        assert r.stats()["mirror"] == 1
    orc = oracle.solve(text, g)
    for x in gr.nonterminals:
        s, d = res[x][:2]
        assert set(zip(s.tolist(), d.tolist())) == orc.pair_set(x), x
    rounds = r.stats()["rounds"]
    for x, (s, d, left, right, mid, rnd) in res.items():
        assert (rnd <= rounds).all(), x
        eps = left == NONE
        assert (s[eps] == d[eps]).all(), x                   # eps pairs sit on the diagonal
        binary = right != NONE
        assert (mid[binary] < g.n).all() and (mid[~binary] == NONE).all(), x
    cert = os.path.join(tmp_path, "gpu.cert")
    write_certificate(cert, text, g, gr.symbols, res)
    certified = check_certificate(text, g, cert)             # sound
    for x in gr.nonterminals:
        s, d = res[x][:2]
        assert certified[x] == set(zip(s.tolist(), d.tolist())), x
    check_closed(text, g, certified)                          # seeded and closed
    r.close()


def test_witness_device_readout_and_repeat(ctx):
    import torch
    text, g = G.DYCK1, graphs.erdos_renyi(200, 600, seed=24)
    gr, r, res = solve_with_witnesses(ctx, text, g)
    dev = torch.device("cuda", 0)
    for x in gr.nonterminals:
        wd = r.witness(x, device=dev)
        for a, b in zip(wd, res[x][2:]):
            assert np.array_equal(a.cpu().numpy().astype(np.uint32), b), x
    # the same pairs as a solve without witnesses
    m = cflr()
    plain = m.solve(ctx, gr, m.Graph.from_workload(ctx, g))
    for x in gr.nonterminals:
        assert plain.pair_set(x) == set(zip(res[x][0].tolist(), res[x][1].tolist())), x
    plain.close()
    r.close()


def test_witness_rejected_where_not_recorded(ctx):
    m = cflr()
    g = graphs.erdos_renyi(50, 120, seed=25)
    gr = m.Grammar(G.DYCK1)
    graph = m.Graph.from_workload(ctx, g)
    with pytest.raises(m.CflrError) as e:               # dense storage
        m.solve(ctx, gr, graph, witness=1, storage=1)
    assert e.value.status == 7
    with pytest.raises(m.CflrError) as e:               # right sides of three symbols
        m.solve(ctx, m.Grammar(G.ALIAS_FIG5A), m.Graph.from_workload(ctx, graphs.alias_graph(100, seed=2)),
                witness=1)
    assert e.value.status == 7
    with pytest.raises(m.CflrError) as e:               # batches
        m.solve_batch(ctx, gr, [graph], witness=1)
    assert e.value.status == 7
    r = m.solve(ctx, gr, graph, storage=2)               # a solve without witnesses
    with pytest.raises(m.CflrError) as e:
        r.witness("S")
    assert e.value.status == 1
    r.close()
