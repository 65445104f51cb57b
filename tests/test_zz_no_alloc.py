"""cflr_solve_noalloc -- the solve without device allocation, its structures
in the library's fixed scratch region -- against cflr_solve of the same
input, pair for pair (tolerance 0), through the C-ABI: two calls in a row,
the second on a smaller input; then inputs the region cannot hold or that
are invalid, which must fail with a clear error."""

import ctypes as C

import numpy as np
import pytest

import workloads
from workloads import grammars as G
from workloads import graphs

pytestmark = pytest.mark.gpu


def cflr():
    import paper_2401_11029_amd as m
    return m


def call_noalloc(ctx, gr, g, capacity, src=None):
    """Raw C-ABI call; returns (status, counts, out_src, out_dst, stats)."""
    import torch
    m = cflr()
    from paper_2401_11029_amd._lib import Stats
    dev = torch.device("cuda", 0)
    s = torch.from_numpy(g.src.astype(np.int32)).to(dev) if src is None else src
    d = torch.from_numpy(g.dst.astype(np.int32)).to(dev)
    lab = torch.from_numpy(g.label.astype(np.int32)).to(dev)
    names = [x.encode() for x in g.label_names]
    arr = (C.c_char_p * max(1, len(names)))(*names)
    nts = gr.nonterminals
    counts = (C.c_uint64 * max(1, len(nts)))()
    out_s = torch.full((max(1, capacity),), -1, dtype=torch.int32, device=dev)
    out_d = torch.full((max(1, capacity),), -1, dtype=torch.int32, device=dev)
    st = Stats()
    torch.cuda.synchronize()
    rc = m.lib().cflr_solve_noalloc(ctx._h, gr._h, g.n, g.m, C.c_void_p(s.data_ptr()), C.c_void_p(d.data_ptr()),
                                    C.c_void_p(lab.data_ptr()), len(names), arr, None,
                                    C.c_void_p(out_s.data_ptr()), C.c_void_p(out_d.data_ptr()), capacity, counts,
                                    C.byref(st))
    torch.cuda.synchronize()
    return rc, [counts[k] for k in range(len(nts))], out_s.cpu().numpy(), out_d.cpu().numpy(), st


def test_noalloc_equals_cflr_solve_on_two_calls_the_second_smaller(ctx):
    m = cflr()
    cases = [workloads.config("pointsto_200k", n=4000),       # 644 matrices, 119k pairs
             (G.ALIAS_FIG5A_WCNF, graphs.alias_graph(700, seed=9))]  # smaller: 13 matrices
    for k, (text, g) in enumerate(cases):
        print(f"no-alloc call {k}: n={g.n} m={g.m}", flush=True)
        gr = m.Grammar(text)
        ref = m.solve(ctx, gr, m.Graph.from_workload(ctx, g), storage=2)
        want = {x: ref.pairs(x) for x in gr.nonterminals}
        total = sum(w[0].shape[0] for w in want.values())
        rc, counts, out_s, out_d, st = call_noalloc(ctx, gr, g, total + 5)
        assert rc == 0, m.lib().cflr_last_error()
        assert st.storage == 2 and st.total_pairs == total
        at = 0
        for x, c in zip(gr.nonterminals, counts):
            ws, wd = want[x]
            assert c == ws.shape[0], x
            assert np.array_equal(out_s[at:at + c].astype(np.uint32), ws), x
            assert np.array_equal(out_d[at:at + c].astype(np.uint32), wd), x
            at += c
        assert np.all(out_s[at:] == -1)  # nothing written past the total


def test_noalloc_rejects_what_it_cannot_hold(ctx):
    import torch
    m = cflr()
    # capacity below the total: EINVAL, counts written, no pairs
    text, g = G.DYCK1, graphs.erdos_renyi(256, 1024, seed=0)
    gr = m.Grammar(text)
    rc, counts, out_s, _, _ = call_noalloc(ctx, gr, g, 10)
    assert rc == 1 and sum(counts) > 10 and np.all(out_s == -1)
    assert b"capacity" in m.lib().cflr_last_error()
    # an edge naming a vertex >= n: EINVAL before any solve
    bad = torch.from_numpy(g.src.astype(np.int32)).to("cuda")
    bad[5] = 256
    rc, _, _, _, _ = call_noalloc(ctx, gr, g, 1 << 20, src=bad)
    assert rc == 1 and b"vertex" in m.lib().cflr_last_error()
    # 644 matrices on 12,000 vertices: the list directory alone exceeds the region
    text, g = workloads.config("pointsto_200k", n=12000)
    rc, _, _, _, _ = call_noalloc(ctx, m.Grammar(text), g, 1 << 20)
    assert rc == 3 and b"no-alloc scratch" in m.lib().cflr_last_error()
    # a dense closure: more pairs than the region's hash set
    g = graphs.random_graph(3000, 30000, ["a"], seed=5150, self_loops=True)
    rc, _, _, _, _ = call_noalloc(ctx, m.Grammar(G.TRANSITIVE), g, 1 << 20)
    assert rc == 3 and b"no-alloc scratch" in m.lib().cflr_last_error()
    # and the region still serves a solve afterwards
    text, g = G.DYCK1, graphs.erdos_renyi(300, 900, seed=4)
    gr = m.Grammar(text)
    rc, counts, out_s, out_d, _ = call_noalloc(ctx, gr, g, 1 << 20)
    assert rc == 0
    ref = m.solve(ctx, gr, m.Graph.from_workload(ctx, g), storage=2)
    assert counts == [ref.count(x) for x in gr.nonterminals]
