"""Write the stored expected values under tests/golden/ -- calls only the
CPU oracle (``oracle/``) on the seeded inputs of ``workloads``.

    python tests/golden/make_goldens.py NAME [NAME ...]

NAME is one of the keys of GOLDENS or of BATCH_GOLDENS.  A GOLDENS entry
writes ``NAME.json`` holding, per non-terminal, the pair count and the
SHA-256 of its pairs in (i, j) order (two little-endian u32 each), plus the
oracle's own fixpoint time.  A BATCH_GOLDENS entry writes the same record for
each graph of a batch that its filter selects, keyed by the graph's index.
"""

from __future__ import annotations

import json
import os
import platform
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from workloads import grammars, graphs  # noqa: E402

GOLDENS = {
    # the tiny Dyck-1 configuration at its full size
    "dyck_er_256": lambda: workloads.config("dyck_er"),
    # the memory-alias configuration at its full size (50,000 vertices)
    "alias_50k": lambda: workloads.config("alias_50k"),
    # the memory-alias shape at 8,000 vertices (a mid-size parity case)
    "alias_8k": lambda: workloads.config("alias_50k", n=8000),
    # the points-to shape (64 fields) at 4,000 and 12,000 vertices
    "pointsto_4k": lambda: workloads.config("pointsto_200k", n=4000),
    "pointsto_12k": lambda: workloads.config("pointsto_200k", n=12000),
    # Fig. 5b's hand WCNF on the 8,000 vertex alias graph
    "alias5b_8k": lambda: (grammars.ALIAS_FIG5B,
                           graphs.alias_graph(8000, seed=1)),
    # the points-to configuration at its full size (200,000 vertices)
    "pointsto_200k": lambda: workloads.config("pointsto_200k"),
    # value flow (Fig. 7b, 64 call sites) at the vertex and edge counts of
    # Table 3's povray graph
    "valueflow_346k": lambda: workloads.config("valueflow_346k"),
}

# The 256-graph alias batch (the batched configuration): every graph with at
# most 8,000 vertices, solved one by one.
BATCH_GOLDENS = {
    "alias_batch_le8k": (lambda: graphs.alias_batch(256),
                         grammars.ALIAS_FIG5A_WCNF, lambda g: g.n <= 8000),
}


def make(name):
    text, g = GOLDENS[name]()
    r = oracle.solve(text, g, pairs=False, digest=True)
    out = {
        "name": name,
        "n": g.n,
        "m": g.m,
        "meta": g.meta,
        "order": r.order,
        "count": r.count,
        "sha256": r.digest,
        "total": sum(r.count.values()),
        "oracle_seconds": r.seconds,
        "oracle_host": platform.processor() or platform.machine(),
    }
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(f"{name}: {out['total']} pairs, oracle {r.seconds:.1f} s -> {path}",
          flush=True)


def make_batch(name):
    make_graphs, text, keep = BATCH_GOLDENS[name]
    out = {"name": name, "graphs": {}, "oracle_host": platform.processor() or platform.machine()}
    secs = 0.0
    for k, g in enumerate(make_graphs()):
        if not keep(g):
            continue
        r = oracle.solve(text, g, pairs=False, digest=True)
        secs += r.seconds
        out["graphs"][str(k)] = {"n": g.n, "m": g.m, "meta": g.meta, "order": r.order,
                                 "count": r.count, "sha256": r.digest,
                                 "total": sum(r.count.values()), "oracle_seconds": r.seconds}
    out["oracle_seconds"] = secs
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(f"{name}: {len(out['graphs'])} graphs, oracle {secs:.1f} s -> {path}", flush=True)


if __name__ == "__main__":
    oracle.build(force=False)
    for nm in sys.argv[1:]:
        if nm in BATCH_GOLDENS:
            make_batch(nm)
        else:
            make(nm)
