"""GPU path vs the CPU oracle, pair for pair (tolerance 0: the result is a set
of integer pairs).  Every call goes through libcflr's C interface."""

import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from workloads import grammars as G
from workloads import graphs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cflr():
    import paper_2401_11029_amd as m
    return m


def gpu_solve(ctx, text, g, **kw):
    m = cflr()
    gr = m.Grammar(text)
    graph = m.Graph.from_workload(ctx, g)
    return m.solve(ctx, gr, graph, **kw)


def assert_matches_oracle(res, text, g, tag=""):
    o = oracle.solve(text, g)
    assert res.grammar.nonterminals == o.order
    for x in o.order:
        s, d = res.pairs(x)
        want = o.pairs[x]
        assert s.shape[0] == want.shape[0], (tag, x, s.shape[0], want.shape[0])
        assert np.array_equal(s, want[:, 0]) and np.array_equal(d, want[:, 1]), (tag, x)


def digest(s, d):
    buf = np.empty((s.shape[0], 2), dtype="<u4")
    buf[:, 0] = s
    buf[:, 1] = d
    return hashlib.sha256(buf.tobytes()).hexdigest()


def test_dyck1_erdos_renyi_256(ctx):
    text, g = workloads.config("dyck_er")
    r = gpu_solve(ctx, text, g)
    assert_matches_oracle(r, text, g)
    st = r.stats()
    assert st["rounds"] >= 2 and st["total_pairs"] == sum(r.counts().values())


SWEEP = [
    ("dyck1", G.DYCK1, ["a", "b"]),
    ("alias5a", G.ALIAS_FIG5A_WCNF, ["a", "d", "a_bar", "d_bar"]),
    ("alias5b", G.ALIAS_FIG5B, ["a", "d", "a_bar", "d_bar"]),
    ("pointsto4b", G.pointsto_fig4b(3), G.symbols_of(G.pointsto_fig4b(3))[1]),
    ("pointsto4a", G.pointsto_fig4a(3), G.symbols_of(G.pointsto_fig4a(3))[1]),
    ("valueflow7a", G.cscvf_fig7a(3), G.symbols_of(G.cscvf_fig7a(3))[1]),
    ("fsca6b", G.fsca_fig6b(2), G.symbols_of(G.fsca_fig6b(2))[1]),
    ("refl_trans", G.REFLEXIVE_TRANSITIVE, ["a"]),
    # right sides of three or more symbols (CFPQ Data forms), normalised by the library
    ("alias5a_long", G.ALIAS_FIG5A, ["a", "d", "a_bar", "d_bar"]),
    ("pointsto4a_long", G.pointsto_fig4a_cfg(3), G.symbols_of(G.pointsto_fig4a_cfg(3))[1]),
    ("valueflow7a_long", G.cscvf_fig7a_cfg(3), G.symbols_of(G.cscvf_fig7a_cfg(3))[1]),
    ("fsca6a_long", G.fsca_fig6a_cfg(2), G.symbols_of(G.fsca_fig6a_cfg(2))[1]),
]


@pytest.mark.parametrize("case", SWEEP, ids=[c[0] for c in SWEEP])
def test_random_sweep(ctx, case):
    name, text, labels = case
    for k, (n, m) in enumerate([(1, 3), (5, 12), (33, 90), (64, 200), (65, 260),
                                (200, 600)]):
        g = graphs.random_graph(n, m, labels, seed=1000 + 17 * k, self_loops=True)
        assert_matches_oracle(gpu_solve(ctx, text, g), text, g, f"{name} n={n}")


@pytest.mark.parametrize("n", [4095, 4096, 4097, 8193])
def test_row_segment_boundaries(ctx, n):
    # the alias grammar at n around multiples of 4096 columns (one segment)
    g = graphs.alias_graph(n, m_fwd=n // 2, seed=n)
    assert_matches_oracle(gpu_solve(ctx, G.ALIAS_FIG5A_WCNF, g), G.ALIAS_FIG5A_WCNF, g)


@pytest.mark.parametrize("n", [255, 256, 257, 511, 513, 769])
def test_key_tile_boundaries(ctx, n):
    # the product works on tiles of 256 keys: n just below, at and above a
    # multiple of 256 (a last tile with one key, a full last tile)
    for text, labels in [(G.ALIAS_FIG5A_WCNF, ["a", "d", "a_bar", "d_bar"]), (G.DYCK1, ["a", "b"])]:
        g = graphs.random_graph(n, 3 * n, labels, seed=4000 + n, self_loops=True)
        assert_matches_oracle(gpu_solve(ctx, text, g), text, g, f"n={n}")


@pytest.mark.parametrize("chunk", [0, 32768, 1000])
def test_tiles_split_into_pair_chunks(ctx, chunk):
    # a dense relation: in round 2 one key tile holds ~145k new pairs of one
    # operand; with a small chunk_pairs the tile is split into several work
    # items, each flushing its own partial accumulators (1000 also ends a
    # chunk inside a window of 64 pairs)
    g = graphs.random_graph(600, 20000, ["a"], seed=4242, self_loops=True)
    r = gpu_solve(ctx, G.TRANSITIVE, g, chunk_pairs=chunk)
    assert r.stats()["max_delta"] > 2 * 32768
    assert_matches_oracle(r, G.TRANSITIVE, g)


@pytest.mark.parametrize("name", ["alias_8k", "alias5b_8k", "pointsto_4k", "pointsto_12k"])
def test_golden_digests(ctx, name):
    from tests.golden.make_goldens import GOLDENS
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        gold = json.load(f)
    text, g = GOLDENS[name]()
    r = gpu_solve(ctx, text, g)
    assert r.grammar.nonterminals == gold["order"]
    for x in gold["order"]:
        s, d = r.pairs(x)
        assert s.shape[0] == gold["count"][x], x
        assert digest(s, d) == gold["sha256"][x], x


@pytest.mark.parametrize("case", ["fsca6b", "fsca6a_long", "cscvf7b", "cscvf7a_long"])
def test_analyses_on_their_graph_shapes(ctx, case):
    # field-sensitive alias (Fig. 6) and value flow (Fig. 7) on graphs of
    # their Table 3 shapes at 3,000 vertices (the bench times them at 40,000)
    if case.startswith("fsca"):
        g = graphs.fsca_graph(3000, fields=8)
        text = G.fsca_fig6b(8) if case == "fsca6b" else G.fsca_fig6a_cfg(8)
    else:
        g = graphs.valueflow_graph(3000, m_fwd=5100, calls=8)
        text = G.cscvf_fig7b(8) if case == "cscvf7b" else G.cscvf_fig7a_cfg(8)
    assert_matches_oracle(gpu_solve(ctx, text, g), text, g, case)


def test_long_right_sides_match_binarised_golden(ctx):
    # Fig. 5a as given (right sides of three symbols, normalised by the
    # library) on the 8,000-vertex alias graph: its five non-terminals equal
    # those of the hand-binarised text, whose oracle digests are stored
    from tests.golden.make_goldens import GOLDENS
    with open(os.path.join(GOLDEN, "alias_8k.json")) as f:
        gold = json.load(f)
    _, g = GOLDENS["alias_8k"]()
    r = gpu_solve(ctx, G.ALIAS_FIG5A, g)
    assert r.grammar.nonterminals == ["M", "V", "V1", "V2", "V3"]
    for x in r.grammar.nonterminals:
        s, d = r.pairs(x)
        assert s.shape[0] == gold["count"][x], x
        assert digest(s, d) == gold["sha256"][x], x


def test_edge_cases(ctx):
    m = cflr()
    # no vertices
    g = graphs.make_graph(0, [], label_names=["a", "b"])
    r = gpu_solve(ctx, G.DYCK1, g)
    assert all(v == 0 for v in r.counts().values())
    # vertices but no edges: only eps pairs
    g = graphs.make_graph(70, [], label_names=["a"])
    r = gpu_solve(ctx, G.DYCK1, g)
    assert r.pair_set("S") == {(i, i) for i in range(70)}
    assert r.count("X") == 0
    # labels the grammar does not use are ignored; duplicates collapse
    g = graphs.make_graph(4, [(0, "a", 1), (0, "a", 1), (1, "zz", 2), (1, "b", 3),
                              (2, "b", 2)], label_names=["a", "b", "zz"])
    assert_matches_oracle(gpu_solve(ctx, G.DYCK1, g), G.DYCK1, g)
    # a grammar with only terminal rules (no binary productions)
    text = "A -> a\nB -> b | a\n"
    g = graphs.random_graph(50, 120, ["a", "b"], seed=3)
    assert_matches_oracle(gpu_solve(ctx, text, g), text, g)
    # eps only
    r = gpu_solve(ctx, "E -> eps\n", graphs.random_graph(9, 5, ["a"], seed=1))
    assert r.pair_set("E") == {(i, i) for i in range(9)}
    # invalid graphs are rejected
    with pytest.raises(m.CflrError) as e:
        m.Graph(ctx, 3, [0], [3], [0], ["a"])
    assert e.value.status == 1
    with pytest.raises(m.CflrError) as e:
        m.Graph(ctx, 3, [0], [1], [1], ["a"])
    assert e.value.status == 1


def test_round_limit_and_argument_errors(ctx):
    import ctypes as C
    m = cflr()
    L = m.lib()
    text, g = G.ALIAS_FIG5A_WCNF, graphs.alias_graph(2000, seed=11)
    gr = m.Grammar(text)
    graph = m.Graph.from_workload(ctx, g)
    # round limit: ETIMEOUT with a partial result, every pair of which lies
    # in the least fixpoint
    o = m.opts(max_rounds=2)
    h = C.c_void_p()
    assert L.cflr_solve(ctx._h, gr._h, graph._h, C.byref(o), C.byref(h)) == 6  # CFLR_ETIMEOUT
    assert h.value
    res = m.Result(h, gr)
    orc = oracle.solve(text, g)
    for x in orc.order:
        assert res.pair_set(x) <= orc.pair_set(x), x
    assert sum(res.counts().values()) < sum(orc.count.values())
    # copy into too small a buffer, non-terminal out of range
    cnt = res.count("M")
    assert cnt > 0
    buf = np.empty(cnt, dtype=np.uint32)
    w = C.c_uint64()
    p = C.c_void_p(buf.ctypes.data)
    assert L.cflr_result_copy(res._h, 0, p, p, cnt - 1, 0, C.byref(w)) == 1  # CFLR_EINVAL
    c = C.c_uint64()
    assert L.cflr_result_count(res._h, 99, C.byref(c)) == 1
    # a graph of another context
    ctx2 = m.Context(0)
    g2 = m.Graph.from_workload(ctx2, g)
    with pytest.raises(m.CflrError) as e:
        m.solve(ctx, gr, g2)
    assert e.value.status == 1
    res.close()


def test_autotune_then_batch_matches_oracle():
    m = cflr()
    own = m.Context(0)  # the tuned launch shape stays in this context
    gs = [graphs.alias_graph(1500 + 400 * k, seed=20 + k) for k in range(3)]
    gr = m.Grammar(G.ALIAS_FIG5A_WCNF)
    gg = [m.Graph.from_workload(own, g) for g in gs]
    t = m.autotune(own, gr, gg)
    assert t["grid_waves"] > 0 and t["rounds_per_sync"] in (2, 4, 8) and t["best_ms"] > 0
    assert t["chunk_pairs"] in (1 << 18, 1 << 20, 1 << 22) and t["sparse_heavy"] == 0  # dense storage
    res = m.solve_batch(own, gr, gg)
    for r, g in zip(res, gs):
        assert_matches_oracle(r, G.ALIAS_FIG5A_WCNF, g, "tuned batch")


def test_autotune_sparse_then_solve_matches_oracle():
    # the points-to generator at 24,000 vertices: its 644 dense matrices
    # would take more than a quarter of the device, so the solves are
    # sparse; the tuner picks the grid, then the heavy-bucket threshold,
    # and a later solve on the context uses them
    m = cflr()
    own = m.Context(0)
    text, g = workloads.config("pointsto_200k", n=24000)
    gr = m.Grammar(text)
    go = m.Graph.from_workload(own, g)
    t = m.autotune(own, gr, [go])
    assert t["sparse_heavy"] in (64, 128, 256) and t["chunk_pairs"] == 0 and t["rounds_per_sync"] == 1
    r = m.solve(own, gr, go)
    assert r.stats()["storage"] == 2
    o = oracle.solve(text, g, pairs=False, digest=True)
    for x in o.order:
        s_, d_ = r.pairs(x)
        assert s_.shape[0] == o.count[x] and digest(s_, d_) == o.digest[x], x


def test_naive_variant_matches(ctx):
    for seed in range(3):
        g = graphs.random_graph(120, 300, ["a", "d", "a_bar", "d_bar"], seed=40 + seed)
        r = gpu_solve(ctx, G.ALIAS_FIG5B, g, semi_naive=0)
        assert_matches_oracle(r, G.ALIAS_FIG5B, g, "naive")


def test_overflowing_new_pair_buffer_reruns_round(ctx):
    g = graphs.alias_graph(2000, seed=77)
    r = gpu_solve(ctx, G.ALIAS_FIG5A_WCNF, g, delta_capacity=256)
    assert r.stats()["reruns"] > 0
    assert_matches_oracle(r, G.ALIAS_FIG5A_WCNF, g, "overflow")


def test_repeat_solves_are_identical(ctx):
    text, g = workloads.config("alias_50k", n=3000)
    first = None
    for _ in range(3):
        r = gpu_solve(ctx, text, g)
        d = {x: digest(*r.pairs(x)) for x in r.grammar.nonterminals}
        if first is None:
            first = d
        assert d == first


def test_device_pointer_io(ctx):
    import torch
    m = cflr()
    g = graphs.erdos_renyi(300, 900, seed=8)
    dev = torch.device("cuda", 0)
    graph = m.Graph(ctx, g.n, torch.from_numpy(g.src.astype(np.int32)).to(dev),
                    torch.from_numpy(g.dst.astype(np.int32)).to(dev),
                    torch.from_numpy(g.label.astype(np.int32)).to(dev), g.label_names)
    r = m.solve(ctx, m.Grammar(G.DYCK1), graph)
    s, d = r.pairs("S", device=dev)
    assert s.is_cuda
    hs, hd = r.pairs("S")
    assert np.array_equal(s.cpu().numpy().astype(np.uint32), hs)
    assert np.array_equal(d.cpu().numpy().astype(np.uint32), hd)


def test_batch_matches_single_solves(ctx):
    m = cflr()
    cases = [(G.DYCK1, graphs.erdos_renyi(n, 3 * n, seed=s)) for s, n in
             [(1, 100), (2, 700), (3, 64)]]
    cases += [(G.ALIAS_FIG5A_WCNF, graphs.alias_graph(n, seed=s)) for s, n in
              [(4, 1500), (5, 300), (6, 5000)]]
    cases += [(G.pointsto_fig4b(4), graphs.pointsto_graph(n, fields=4, seed=s))
              for s, n in [(7, 900), (8, 2500)]]
    cases.append((G.DYCK1, graphs.make_graph(0, [], label_names=["a"])))
    grams = {t: m.Grammar(t) for t, _ in cases}
    graph_objs = [m.Graph.from_workload(ctx, g) for _, g in cases]
    res = m.solve_batch(ctx, [grams[t] for t, _ in cases], graph_objs)
    for (text, g), r in zip(cases, res):
        assert r.stats()["storage"] == 1
        assert_matches_oracle(r, text, g, "batch")


@pytest.mark.parametrize("rounds_per_sync", [1, 3, 7])
def test_batch_graph_replay_matches_oracle(ctx, rounds_per_sync):
    # rounds captured into a hipGraph and replayed rounds_per_sync at a time,
    # with host reads between replays; instances converge mid-replay
    m = cflr()
    cases = [(G.ALIAS_FIG5A_WCNF, graphs.alias_graph(n, seed=s)) for s, n in
             [(31, 2500), (32, 400), (33, 6000)]]
    cases.append((G.DYCK1, graphs.erdos_renyi(500, 1500, seed=34)))
    grams = {t: m.Grammar(t) for t, _ in cases}
    objs = [m.Graph.from_workload(ctx, g) for _, g in cases]
    for rep in range(2):
        res = m.solve_batch(ctx, [grams[t] for t, _ in cases], objs,
                            rounds_per_sync=rounds_per_sync)
        for (text, g), r in zip(cases, res):
            assert_matches_oracle(r, text, g, f"graph R={rounds_per_sync} rep={rep}")


@pytest.mark.parametrize("rounds_per_sync", [2, 5])
def test_overflow_inside_graph_replay_reruns_round(ctx, rounds_per_sync):
    # a tiny new-pair buffer overflows inside replayed rounds: every kernel
    # after the overflow must leave the round's state intact for the re-run
    m = cflr()
    cases = [(G.ALIAS_FIG5A_WCNF, graphs.alias_graph(n, seed=s)) for s, n in [(41, 3000), (42, 900)]]
    cases.append((G.DYCK1, graphs.erdos_renyi(700, 2100, seed=43)))
    grams = {t: m.Grammar(t) for t, _ in cases}
    objs = [m.Graph.from_workload(ctx, g) for _, g in cases]
    res = m.solve_batch(ctx, [grams[t] for t, _ in cases], objs,
                        rounds_per_sync=rounds_per_sync, delta_capacity=512)
    assert res[0].stats()["reruns"] > 0
    for (text, g), r in zip(cases, res):
        assert_matches_oracle(r, text, g, f"overflow in replay R={rounds_per_sync}")


def test_server_results_equal_alone_and_in_the_mix(ctx):
    m = cflr()
    cases = [(G.DYCK1, graphs.erdos_renyi(400, 1200, seed=21)),
             (G.ALIAS_FIG5A_WCNF, graphs.alias_graph(3000, seed=22)),
             (G.pointsto_fig4b(4), graphs.pointsto_graph(2000, fields=4, seed=23)),
             (G.ALIAS_FIG5B, graphs.alias_graph(1000, seed=24))] * 2
    grams = {t: m.Grammar(t) for t, _ in cases}
    objs = [m.Graph.from_workload(ctx, g) for _, g in cases]
    # a 512 MiB budget: requests of at most 8 MiB (Dyck-1, alias 5b) run in
    # the small-request run, the others in the large one
    srv = m.Server(ctx, hbm_budget_bytes=512 << 20, max_slots=5)
    tickets = [srv.submit(grams[t], o) for (t, _), o in zip(cases, objs)]
    mixed = [srv.wait(t, timeout_s=300) for t in tickets]
    times = [srv.times(t) for t in tickets]
    srv.close()
    for (text, g), r in zip(cases, mixed):
        alone = m.solve(ctx, grams[text], m.Graph.from_workload(ctx, g))
        for x in r.grammar.nonterminals:
            sa, da = alone.pairs(x)
            sm, dm = r.pairs(x)
            assert np.array_equal(sa, sm) and np.array_equal(da, dm), x
        assert_matches_oracle(r, text, g, "served")
    # requests overlapped on the device: some admitted before others finished
    admits = sorted(t[1] for t in times)
    finishes = sorted(t[2] for t in times)
    assert admits[1] < finishes[0]


def test_server_sends_large_requests_to_the_sparse_lane(ctx):
    # a 16 MiB budget: requests whose dense matrices would not fit it are
    # solved on the sparse engine by the server's second lane, beside the
    # dense runs
    m = cflr()
    cases = [(G.ALIAS_FIG5A_WCNF, graphs.alias_graph(4000, seed=3)),
             (G.pointsto_fig4b(64), graphs.pointsto_graph(3000, seed=4)),
             (G.DYCK1, graphs.erdos_renyi(300, 900, seed=5)),
             (G.pointsto_fig4b(8), graphs.pointsto_graph(1500, fields=8, seed=6))]
    grams = {t: m.Grammar(t) for t, _ in cases}
    objs = [m.Graph.from_workload(ctx, g) for _, g in cases]
    srv = m.Server(ctx, hbm_budget_bytes=16 << 20, max_slots=2)
    tickets = [srv.submit(grams[t], o) for (t, _), o in zip(cases, objs)]
    res = [srv.wait(t, timeout_s=300) for t in tickets]
    srv.close()
    assert [r.stats()["storage"] for r in res] == [2, 2, 1, 2]
    assert res[1].stats()["mirror"] == 1  # Fig. 4b on its graph: the mirror plan
    for (text, g), r in zip(cases, res):
        assert_matches_oracle(r, text, g, "sparse lane")
        r.close()


def test_server_restarts_requests_at_the_pair_limit(ctx, monkeypatch, capfd):
    # more new pairs in one round than the dense buffer may hold (the limit
    # lowered through CFLR_DENSE_PAIR_LIMIT): the running requests start
    # again with half as many at once, and every result is the oracle's
    m = cflr()
    cases = [graphs.erdos_renyi(600, 1500, seed=80 + k) for k in range(8)]
    gr = m.Grammar(G.DYCK1)
    objs = [m.Graph.from_workload(ctx, g) for g in cases]
    need = 0
    for o in objs:
        r = m.solve(ctx, gr, o, storage=1)
        need = max(need, r.stats()["max_delta"] + 2 * 600 * 3)
        r.close()
    monkeypatch.setenv("CFLR_DENSE_PAIR_LIMIT", str(4 * need))
    monkeypatch.setenv("CFLR_PROGRESS", "1")
    srv = m.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=8, rounds_per_sync=1)
    tickets = [srv.submit(gr, o) for o in objs]
    res = [srv.wait(t, timeout_s=300) for t in tickets]
    srv.close()
    err = capfd.readouterr().err
    assert "start again" in err, err[-2000:]
    for g, r in zip(cases, res):
        assert_matches_oracle(r, G.DYCK1, g, "served at the limit")
        r.close()


def test_library_loaded_before_torch_still_leaves_torch_a_device():
    # torch carries its own HIP runtime: the binding starts it before loading
    # libcflr.so, so a process that loads the library first still solves and
    # still gives torch the device (a child process, so the order is real)
    import subprocess
    import sys
    code = (
        "from paper_2401_11029_amd import _lib\n"
        "_lib.load()\n"
        "import paper_2401_11029_amd as m\n"
        "import numpy as np\n"
        "ctx = m.Context(0)\n"
        "g = m.Grammar('S -> S S | a')\n"
        "src = np.arange(5, dtype=np.uint32); dst = src + 1\n"
        "gr = m.Graph(ctx, 6, src, dst, np.zeros(5, dtype=np.uint32), ['a'])\n"
        "r = m.solve(ctx, g, gr)\n"
        "assert r.count('S') == 15, r.count('S')\n"
        "import torch\n"
        "assert torch.cuda.is_available()\n"
        "print('ok')\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stderr[-2000:]


def test_trim_and_tuned_options_of_a_fresh_context():
    # a fresh context has nothing tuned; trimming its pool frees the cached
    # blocks and later solves allocate again
    m = cflr()
    own = m.Context(0)
    import ctypes as C
    t = m.Opts()
    assert m.lib().cflr_ctx_tuned(own._h, C.byref(t)) == 0
    assert t.grid_waves == 0 and t.rounds_per_sync == 0 and t.chunk_pairs == 0 and t.sparse_heavy == 0
    assert t.semi_naive == 1
    text, g = G.ALIAS_FIG5A_WCNF, graphs.alias_graph(3000, seed=91)
    gr = m.Grammar(text)
    go = m.Graph.from_workload(own, g)
    m.solve(own, gr, go).close()          # its buffers go back to the pool's cache
    free_before, _ = own.mem_info()
    own.trim()
    free_after, _ = own.mem_info()
    assert free_after >= free_before
    assert_matches_oracle(m.solve(own, gr, go), text, g, "after trim")
