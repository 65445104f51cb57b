"""Seeded synthetic workloads: grammar texts, graph generators, file format.

This package holds inputs only.  It is shared by the CPU oracle's tests and by
the GPU path, and contains none of the reachability arithmetic itself.

Named configurations (the shapes the paper's Table 3 suggests, at sizes that
fit one GPU):

* ``dyck_er``      Dyck-1 on a directed G(256, 1024), labels a/b, seed 0;
* ``alias_50k``    memory-alias grammar (Fig. 5a, binarised) on a 50,000
  vertex power-law graph (alpha 2.1, 50,000 forward a/d edges plus their
  reversed a_bar/d_bar edges), seed 1;
* ``pointsto_200k`` field-sensitive points-to (Fig. 4b, 64 fields) on a
  200,000 vertex power-law graph (300,000 forward edges plus reversed),
  seed 2;
* ``alias_batch``  256 alias graphs with n log-uniform in [1k, 40k].
"""

from . import grammars, graphs
from .graphs import Graph, make_graph

CONFIGS = {
    "dyck_er": dict(grammar=grammars.DYCK1,
                    make=lambda: graphs.erdos_renyi(256, 1024, seed=0)),
    "alias_50k": dict(grammar=grammars.ALIAS_FIG5A_WCNF,
                      make=lambda: graphs.alias_graph(50_000, seed=1)),
    "pointsto_200k": dict(grammar=grammars.pointsto_fig4b(64),
                          make=lambda: graphs.pointsto_graph(200_000,
                                                             seed=2)),
    # context-sensitive value flow (Fig. 7b) on a graph with the vertex and
    # edge counts of Table 3's povray value-flow graph (346,034 vertices,
    # 581,210 edges), with 64 call sites (the table's graph has thousands)
    "valueflow_346k": dict(grammar=grammars.cscvf_fig7b(64),
                           make=lambda: graphs.valueflow_graph(346_034, m_fwd=581_210, calls=64)),
}


def config(name, n=None):
    """(grammar text, Graph) of a named configuration; n rescales the graph
    (same generator and seed, n vertices) for parity at oracle-friendly
    sizes."""
    c = CONFIGS[name]
    if n is None:
        return c["grammar"], c["make"]()
    if name == "dyck_er":
        return c["grammar"], graphs.erdos_renyi(n, 4 * n, seed=0)
    if name == "alias_50k":
        return c["grammar"], graphs.alias_graph(n, seed=1)
    if name == "pointsto_200k":
        return c["grammar"], graphs.pointsto_graph(n, seed=2)
    if name == "valueflow_346k":
        return c["grammar"], graphs.valueflow_graph(n, m_fwd=n * 581_210 // 346_034, calls=64)
    raise KeyError(name)


__all__ = ["grammars", "graphs", "Graph", "make_graph", "CONFIGS", "config"]
