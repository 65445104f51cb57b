"""Batched solves at the new-pair buffer's limit (the dense engine's 32-bit
sort positions cap one round's new pairs): when the running graphs of a
batch derive more pairs in one round than the buffer may hold, the batch
starts them again with at most half as many running at once, and every
result is still the oracle's.  The limit is lowered for the test through
CFLR_DENSE_PAIR_LIMIT.  Every call goes through libcflr's C interface."""

import pytest

from workloads import grammars as G
from workloads import graphs

from tests.test_gpu_parity import assert_matches_oracle

pytestmark = pytest.mark.gpu


def test_batch_restarts_graphs_at_the_pair_limit(ctx, monkeypatch, capfd):
    import paper_2401_11029_amd as m
    text = G.DYCK1
    cases = [graphs.erdos_renyi(600, 1500, seed=70 + k) for k in range(8)]
    gr = m.Grammar(text)
    objs = [m.Graph.from_workload(ctx, g) for g in cases]
    # what one graph needs at most in one round, alone
    need = 0
    for o in objs:
        r = m.solve(ctx, gr, o, storage=1)
        need = max(need, r.stats()["max_delta"] + 2 * 600 * 3)
        r.close()
    limit = 4 * need
    print(f"pair limit {limit} (one graph's round needs at most {need})", flush=True)
    monkeypatch.setenv("CFLR_DENSE_PAIR_LIMIT", str(limit))
    monkeypatch.setenv("CFLR_PROGRESS", "1")
    res = m.solve_batch(ctx, [gr] * len(objs), objs, rounds_per_sync=1)
    err = capfd.readouterr().err
    assert "start again" in err, err[-2000:]
    for g, r in zip(cases, res):
        assert_matches_oracle(r, text, g, "batch at the limit")
        r.close()
