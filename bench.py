"""Benchmark: CFL-reachability fixpoint on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode single|batch|serve|...]

A step is one whole solve of the largest single-solve workload: the
field-sensitive points-to grammar (Fig. 4b of the paper at 64 fields, 386
non-terminals, 644 matrices after lowering) on a 200,000-vertex power-law
graph (alpha 2.1, 300,000 forward edges alloc/assign/load_f/store_f plus
their reversed edges, fields Zipf(1.1), seed 2).  Its dense bit matrices
would need terabytes, so the library solves it on sparse storage.  The
graph is resident in device memory before timing starts; a step runs
seeding, every round and the convergence test.  value = derived pairs per
second over the K timed steps: pairs of the grammar's non-terminals minus
the pairs seeding puts there.  The grammar is closed under reversal and the
graph holds every edge with its reverse, so the library solves it with a
mirror plan (one production of each mirror pair keeps its product; the
transposes of its new pairs are the other's); other_configs gives the same
solve with every production's product (cflr_opts.mirror = OFF).  Under the
plan the pairs of FT and SP_i are held as the transposes of PT's and FS_i's
row lists (the readout writes them out transposed, outside the timed
region, as it writes every pair out); every pair is derived in the timed
steps and the counts include them all.

The JSON line also carries:
  roofline      the dominant kernel of the sparse engine's product (the
                light-bucket or the heavy-bucket kernel, whichever takes
                longer) against HBM: its algorithmic bytes per launch
                (counted on the device in an untimed accounting solve: 8 per
                sorted new pair, 4 per entry of each distinct partner list
                and output row read in a round, 16 per pair derived) over
                its average launch time (HIP events on the library's stream
                in the timed steps); traffic from the committed rocprofv3
                FETCH_SIZE / WRITE_SIZE summary of the same kernel; beside
                the 8 TB/s peak, the bandwidth of a plain device copy
                measured on the same GPU (stream_copy_gbs) as a second
                denominator;
  cpu_baseline  the CPU oracle, pinned to one host core, on a bounded sample
                of the same workload (the same generator at 24,000
                vertices), with the oracle's full-size time beside it;
  other_configs the memory-alias configuration (Fig. 5a, 50,000 vertices,
                dense storage), timed the same way, its pairs counted over
                Fig. 5a's own non-terminals (M, V, V1, V2, V3).

--mode batch reports the batched form (256 alias graphs in one call vs one
plain solve after another; --batch-grammar dyck: Dyck-1 on G(n, m) graphs of
the same sizes; beside it the oracle over the small graphs on every host
core); --mode serve reports the served form (Poisson
arrivals of mixed queries, solves/s and p50/p99 latency against a
one-at-a-time plain path); --mode grammars times the paper's hand-normalised
grammars against the automatically normalised ones on the same graphs
(Fig. 5b vs 5a on the alias graph, Fig. 4b vs 4a on a points-to graph);
--mode analyses times the field-sensitive alias and value-flow analyses
(Figs. 6, 7) on graphs of their shapes.  None of them is the default line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HEADLINE = "pointsto_200k"
PROFILE_PMC = os.path.join(ROOT, "profiles", "sparse_product_pointsto200k_pmc.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2401_11029_amd", "csrc", "sparse_kernels.hip")
GOLDEN_FULL = os.path.join(ROOT, "tests", "golden", "pointsto_200k.json")
CPU_SAMPLE_N = 40000
# Fig. 5a's own non-terminals in the binarised text (Y1..Y4 are its helpers)
ALIAS_FIG5A_NTS = ["M", "V", "V1", "V2", "V3"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary, or None when the kernel source changed since it was taken."""
    try:
        with open(PROFILE_PMC) as f:
            p = json.load(f)
    except (OSError, ValueError):
        return None
    if p.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return p.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def seeded_user_pairs(text, g, names=None):
    """Pairs that seeding puts into the grammar's non-terminals directly:
    (i, i) for x -> eps and the edges of t for x -> t (restricted to
    `names` when given)."""
    from oracle.textgrammar import TextGrammar
    tg = TextGrammar(text)
    keep = (lambda x: True) if names is None else (lambda x: x in names)
    count = len({x for x in tg.eps if keep(x)}) * g.n
    for x, y in tg.unit:
        if y in tg.terminals and keep(x):
            lab = g.label_names.index(y) if y in g.label_names else -1
            sel = g.label == lab
            count += len(set(zip(g.src[sel].tolist(), g.dst[sel].tolist())))
    return count


def cpu_baseline():
    """The oracle, as it is, pinned to one host core, on the same generator
    at CPU_SAMPLE_N vertices; the full-size oracle time from the stored
    golden beside it."""
    import oracle
    import workloads
    text, g = workloads.config(HEADLINE, n=CPU_SAMPLE_N)
    import shutil
    cpus = sorted(os.sched_getaffinity(0))
    cpu = cpus[0] if cpus and shutil.which("taskset") else None
    r = oracle.solve(text, g, pairs=False, digest=True, cpu=cpu)
    derived = sum(r.count.values()) - seeded_user_pairs(text, g)
    out = {"value": derived / r.seconds, "unit": "pairs/s", "cores": 1, "kind": "oracle",
           "sample": f"points-to generator at n={CPU_SAMPLE_N} (seed 2), one full solve: "
                     f"{derived} derived pairs in {r.seconds:.1f} s, "
                     + (f"pinned to host core {cpu} " if cpu is not None else "one thread, not pinned ")
                     + f"({host_cpu()}, {len(cpus)} cores available)"}
    try:
        with open(GOLDEN_FULL) as f:
            gold = json.load(f)
        _, gfull = workloads.config(HEADLINE)
        full_derived = gold["total"] - seeded_user_pairs(text, gfull)
        out["full_size"] = {"pairs_per_s": full_derived / gold["oracle_seconds"],
                            "seconds": gold["oracle_seconds"], "derived_pairs": full_derived,
                            "host": "the build container (one core of an x86_64 host), "
                                    "from tests/golden/pointsto_200k.json"}
    except (OSError, ValueError, KeyError):
        pass
    return out


def time_solves(cflr, ctx, gr, graph, warmup, steps, tag):
    import torch
    for w in range(warmup):
        r = cflr.solve(ctx, gr, graph)
        log(f"{tag} warmup {w}: {r.stats()['fixpoint_ms']:.1f} ms")
        r.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        r = cflr.solve(ctx, gr, graph, kernel_timing=1)
        stats.append(r.stats())
        counts = r.counts() if k == steps - 1 else None
        r.close()
        log(f"{tag} step {k}: {stats[-1]['fixpoint_ms']:.1f} ms, {stats[-1]['rounds']} rounds, "
            f"{stats[-1]['reruns']} re-runs")
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats, counts


def fix_summary(stats):
    fix = sorted(s["fixpoint_ms"] for s in stats)
    mean = sum(fix) / len(fix)
    std = (sum((x - mean) ** 2 for x in fix) / max(1, len(fix) - 1)) ** 0.5
    return {"fixpoint_ms_mean": mean, "fixpoint_ms_median": fix[len(fix) // 2], "fixpoint_ms_std": std}


def alias_context(cflr, args):
    """The memory-alias configuration, timed as the headline (fewer steps)."""
    import workloads
    text, g = workloads.config("alias_50k")
    ctx = cflr.Context(0)
    gr = cflr.Grammar(text)
    graph = cflr.Graph.from_workload(ctx, g)
    steps = max(1, min(3, args.steps))
    secs, stats, counts = time_solves(cflr, ctx, gr, graph, max(1, args.warmup), steps, "alias_50k")
    own = sum(counts[x] for x in ALIAS_FIG5A_NTS) - seeded_user_pairs(text, g, ALIAS_FIG5A_NTS)
    out = {"workload": "alias_50k: memory-alias grammar (Fig. 5a, binarised in the text with helpers "
                       "Y1..Y4) on a 50,000-vertex power-law graph (alpha 2.1, 100,000 stored edges, seed 1)",
           "storage": "dense" if stats[-1]["storage"] == 1 else "sparse",
           "rounds": stats[-1]["rounds"],
           "derived_pairs_fig5a_nts": own,
           "derived_pairs_per_s_fig5a_nts": own * steps / secs,
           "derived_pairs_all_nts_incl_helpers": stats[-1]["new_pairs"],
           "ms_per_step": secs * 1e3 / steps}
    out.update(fix_summary(stats))
    del graph, gr
    ctx.close()
    return out


def stream_copy_gbs(reps=5, words=1 << 29):
    """Bandwidth of a plain device copy (2 GiB read, 2 GiB written by one
    kernel), best of `reps`, timed with HIP events."""
    import torch
    a = torch.ones(words, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * words / (best / 1e3) / 1e9


def readout_all_ms(cflr, ctx, gr, graph, **kw):
    """One more solve, then every non-terminal's pairs written out sorted
    into device memory (cflr_result_copy to torch tensors): wall ms of the
    readout alone (under a mirror plan it includes writing out the
    non-terminals held as their mirror's transposed rows)."""
    import torch
    r = cflr.solve(ctx, gr, graph, **kw)
    dev = torch.device("cuda", 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x in gr.nonterminals:
        s, d = r.pairs(x, device=dev)
        del s, d
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    r.close()
    torch.cuda.empty_cache()
    return ms


def plain_plan(cflr, args, text, g):
    """The headline solve with every production's own product (no mirror
    plan), timed as the headline (fewer steps)."""
    ctx = cflr.Context(0)
    gr = cflr.Grammar(text)
    graph = cflr.Graph.from_workload(ctx, g)
    for w in range(max(1, args.warmup)):
        cflr.solve(ctx, gr, graph, mirror=1).close()
    stats = []
    for k in range(max(1, min(2, args.steps))):
        r = cflr.solve(ctx, gr, graph, mirror=1, kernel_timing=1)
        stats.append(r.stats())
        r.close()
        log(f"plain plan step {k}: {stats[-1]['fixpoint_ms']:.1f} ms")
    readout_ms = readout_all_ms(cflr, ctx, gr, graph, mirror=1)
    del graph, gr
    ctx.close()
    out = {"workload": "pointsto_200k without the mirror plan (cflr_opts.mirror = OFF): every one of "
                       "the 514 binary productions has its own product",
           "mirror_plan": bool(stats[-1]["mirror"]), "total_pairs": stats[-1]["total_pairs"],
           "heavy_ms_mean": sum(s["heavy_ms"] for s in stats) / len(stats),
           "readout_all_ms": readout_ms}
    out.update(fix_summary(stats))
    return out


def single(args):
    import torch
    import paper_2401_11029_amd as cflr
    import workloads
    copy_gbs = stream_copy_gbs()
    log(f"stream copy: {copy_gbs:.0f} GB/s")
    text, g = workloads.config(HEADLINE)
    log(f"workload {HEADLINE}: n={g.n} edges={g.m}")
    ctx = cflr.Context(0)
    gr = cflr.Grammar(text)
    graph = cflr.Graph.from_workload(ctx, g)
    torch.cuda.synchronize()
    for w in range(args.warmup):
        r = cflr.solve(ctx, gr, graph)
        log(f"warmup {w}: {r.stats()['fixpoint_ms']:.1f} ms, {r.stats()['reruns']} re-runs")
        r.close()
    # untimed accounting solve: algorithmic bytes of the product's kernels,
    # taken from a solve without overflow re-runs (a re-run launch is cut
    # short and would skew the per-launch figures)
    while True:
        r = cflr.solve(ctx, gr, graph, count_traffic=1)
        acct = r.stats()
        r.close()
        if not acct["reruns"]:
            break
        log(f"accounting solve had {acct['reruns']} re-runs; again with the grown buffers")
    nl = max(1, acct["heavy_launches"])
    log(f"accounting: heavy {acct['heavy_algo_bytes'] / 1e9:.1f} GB, light {acct['light_algo_bytes'] / 1e9:.1f} GB "
        f"over {nl} launches each")
    secs, stats, counts = time_solves(cflr, ctx, gr, graph, 0, args.steps, HEADLINE)
    readout_ms = readout_all_ms(cflr, ctx, gr, graph)
    log(f"readout of every non-terminal's pairs into device memory: {readout_ms:.0f} ms")
    derived = stats[-1]["total_pairs"] - seeded_user_pairs(text, g)
    value = derived * args.steps / secs
    launches = max(1, sum(s["heavy_launches"] for s in stats))
    kern = {}
    for name, key in (("heavy_kernel", "heavy"), ("light_kernel", "light")):
        ms = sum(s[f"{key}_ms"] for s in stats)
        per_launch_bytes = acct[f"{key}_algo_bytes"] / nl
        avg_s = ms / 1e3 / launches
        kern[name] = {"algo_bytes_per_launch": per_launch_bytes, "avg_launch_ms": avg_s * 1e3,
                      "achieved": per_launch_bytes / avg_s / 1e9 if avg_s > 0 else 0.0,
                      "share_of_fixpoint": ms / max(1e-9, sum(s["fixpoint_ms"] for s in stats))}
    dom = max(kern, key=lambda k: kern[k]["avg_launch_ms"])
    d = kern[dom]
    traffic = measured_traffic(dom)
    cfg = {"workload": "pointsto_200k: field-sensitive points-to grammar (Fig. 4b, 64 fields, "
                       "386 non-terminals) on a 200,000-vertex power-law graph (alpha 2.1, 600,000 "
                       "stored edges alloc/assign/load_f/store_f and reversed, fields Zipf(1.1), seed 2)",
           "vertices": g.n, "edges": g.m,
           "storage": "sparse" if stats[-1]["storage"] == 2 else "dense",
           "pairs": stats[-1]["total_pairs"], "derived_pairs": derived,
           "rounds": stats[-1]["rounds"],
           "mirror_plan": bool(stats[-1]["mirror"]),
           "readout_all_ms": readout_ms,
           "product_ms_mean": sum(s["product_ms"] for s in stats) / len(stats)}
    cfg.update(fix_summary(stats))
    out = {
        "metric": "CFL-r fixpoint derived pairs/s (single solve)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": "hbm", "achieved": d["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": d["achieved"] / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "amplification": (traffic / d["algo_bytes_per_launch"])
                     if traffic and d["algo_bytes_per_launch"] else None,
                     "stream_copy_gbs": copy_gbs,
                     "frac_of_stream_copy": d["achieved"] / copy_gbs,
                     "kernel": dom,
                     "algo_bytes_per_launch": d["algo_bytes_per_launch"],
                     "avg_launch_ms": d["avg_launch_ms"],
                     "kernels": kern},
    }
    if not args.no_other:
        del graph, gr
        ctx.close()
        out["other_configs"] = {"pointsto_200k_plain_plan": plain_plan(cflr, args, text, g),
                                "alias_50k": alias_context(cflr, args)}
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def oracle_pool(text, gs, threads):
    """The oracle, as it is, over independent graphs on `threads` host cores
    at once (one oracle process per graph): wall seconds."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda g: oracle.solve(text, g, pairs=False, digest=False), gs))
    return time.perf_counter() - t0


def batch(args):
    """256 graphs (n log-uniform in [1k, 40k], stored degree U[2, 3]) of the
    alias grammar (Fig. 5a; the default) or of Dyck-1 on G(n, m) graphs
    (--batch-grammar dyck) solved by one batched call vs one plain solve
    after another; beside it the oracle over the graphs of at most
    --batch-oracle-max-n vertices on every host core (one oracle process
    per graph) against the batched call on the same graphs."""
    import torch
    import paper_2401_11029_amd as cflr
    from workloads import graphs, grammars
    os.environ["CFLR_PROGRESS"] = "1"
    if args.batch_grammar == "dyck":
        gs = graphs.dyck_batch(args.batch_count, n_hi=args.batch_max_n)
        text = grammars.DYCK1
        wl = (f"dyck_batch: {len(gs)} Dyck-1 graphs (directed G(n, m), labels a/b), n log-uniform "
              f"[1000, {args.batch_max_n}], stored degree U[2,3], seeds 3000+g")
    else:
        gs = graphs.alias_batch(args.batch_count, n_hi=args.batch_max_n)
        text = grammars.ALIAS_FIG5A_WCNF
        wl = (f"alias_batch: {len(gs)} alias graphs, n log-uniform [1000, {args.batch_max_n}], "
              f"stored degree U[2,3], seeds 3000+g")
    log(f"batch: {len(gs)} graphs, n {min(g.n for g in gs)}..{max(g.n for g in gs)}, "
        f"{sum(g.m for g in gs)} edges")
    ctx = cflr.Context(0)
    gr = cflr.Grammar(text)
    objs = [cflr.Graph.from_workload(ctx, g) for g in gs]
    # warm-up: one full untimed batch, so that the timed one starts with the
    # new-pair buffer already grown to what the batch needs
    for r in cflr.solve_batch(ctx, gr, objs):
        r.close()
    log("warm-up done; autotuning on every 16th graph")
    # autotune the launch shape on a 16-graph sample (one line per candidate)
    os.environ["CFLR_TUNE_LOG"] = "1"
    tuned = cflr.autotune(ctx, gr, objs[::16])
    log(f"autotuned: {tuned}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = cflr.solve_batch(ctx, gr, objs)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    batch_pairs = [r.stats()["total_pairs"] for r in res]
    for r in res:
        r.close()
    log(f"batched: {tb:.2f} s")
    # the same call on the small graphs alone (the oracle's share below)
    small = [k for k, g in enumerate(gs) if g.n <= args.batch_oracle_max_n]
    tb_small = None
    if small:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in cflr.solve_batch(ctx, gr, [objs[k] for k in small]):
            r.close()
        torch.cuda.synchronize()
        tb_small = time.perf_counter() - t0
    # the plain solves get a context of their own: a context starts its
    # new-pair buffer at the largest size an earlier run on it needed, and
    # the batch's would oversize every single solve.  The batch's context
    # (and the memory its pool caches) goes first.
    del objs, res
    ctx.close()
    seq_ctx = cflr.Context(0)
    seq_objs = [cflr.Graph.from_workload(seq_ctx, g) for g in gs]
    # warm-up on the largest graph (its buffer size serves every smaller one)
    cflr.solve(seq_ctx, gr, seq_objs[max(range(len(gs)), key=lambda k: gs[k].n)]).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_pairs = []
    for q, o in enumerate(seq_objs):
        r = cflr.solve(seq_ctx, gr, o)
        seq_pairs.append(r.stats()["total_pairs"])
        r.close()
        if q % 32 == 31:
            log(f"sequential: {q + 1} solves, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    log(f"sequential: {ts:.2f} s")
    cpu = None
    if small and not args.no_cpu:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"oracle on {len(small)} graphs with n <= {args.batch_oracle_max_n}, {threads} at once ...")
        to = oracle_pool(text, [gs[k] for k in small], threads)
        cpu = {"value": len(small) / to, "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"the {len(small)} graphs of the batch with n <= {args.batch_oracle_max_n}, one "
                         f"oracle process per graph, {threads} at once on the host cores "
                         f"({host_cpu()}): {to:.1f} s",
               "gpu_batched_same_graphs_solves_per_s": len(small) / tb_small}
    print(json.dumps({
        "metric": "batched solves/s", "value": len(gs) / tb, "unit": "solves/s",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
        "sequential_solves_per_s": len(gs) / ts, "speedup_vs_sequential": ts / tb,
        "pairs": int(sum(batch_pairs)), "derived_pairs_per_s": sum(batch_pairs) / tb,
        "same_pair_counts_as_sequential": batch_pairs == seq_pairs,
        "autotuned": tuned,
        "cpu_baseline": cpu,
        "config": {"workload": wl}}),
        flush=True)


# Serving: per-grammar size caps keep every query's dense matrices small
# enough to run many at once (the points-to grammar has 644 matrices).
# The capped mix keeps every query on dense storage; the configured one
# draws n from [1000, 100000] for alias and points-to (the large points-to
# queries then go to the server's sparse lane) and from [1000, 60000] for
# Dyck-1: on G(n, 4n) its closure is dense (S holds about 0.6 n^2 pairs) and
# beyond about 80,000 vertices one round derives more than the 2^32 new
# pairs the dense engine's buffer holds.
SERVE_MIX = {"capped": [("dyck", 1000, 20000), ("alias", 1000, 30000), ("pointsto", 1000, 4096)],
             "configured": [("dyck", 1000, 60000), ("alias", 1000, 100000), ("pointsto", 1000, 100000)]}


def serve_pool(count_per_grammar, seed=4, mix="capped"):
    import numpy as np
    from workloads import graphs, grammars
    rng = np.random.Generator(np.random.PCG64(seed))
    pool = []
    for gi, (name, lo, hi) in enumerate(SERVE_MIX[mix]):
        for q in range(count_per_grammar):
            n = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
            s = 40000 + 1000 * gi + q
            if name == "dyck":
                pool.append((grammars.DYCK1, graphs.erdos_renyi(n, 4 * n, seed=s)))
            elif name == "alias":
                pool.append((grammars.ALIAS_FIG5A_WCNF, graphs.alias_graph(n, seed=s)))
            else:
                pool.append((grammars.pointsto_fig4b(64), graphs.pointsto_graph(n, seed=s)))
    order = rng.permutation(len(pool))
    return [pool[k] for k in order]


def fifo_latencies(arrivals, service):
    """Latencies of a one-at-a-time server taking requests in arrival order."""
    free, out = 0.0, []
    for a, s in zip(arrivals, service):
        start = max(a, free)
        free = start + s
        out.append(free - a)
    return out


def serve(args):
    import numpy as np
    import torch
    import paper_2401_11029_amd as cflr
    from workloads import graphs
    pool = serve_pool(args.serve_per_grammar, mix=args.serve_mix)
    ctx = cflr.Context(0)
    grams = {}
    objs = []
    for text, g in pool:
        if text not in grams:
            grams[text] = cflr.Grammar(text)
        objs.append((grams[text], cflr.Graph.from_workload(ctx, g)))
    log(f"serve: {len(pool)} queries")
    # plain path: one solve after another (also the service times of a FIFO)
    for gr, o in objs[:3]:
        cflr.solve(ctx, gr, o).close()
    service, plain_pairs = [], []
    for q, (gr, o) in enumerate(objs):
        log(f"plain {q}: {pool[q][0].splitlines()[0]} n={pool[q][1].n}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = cflr.solve(ctx, gr, o)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        plain_pairs.append(r.stats()["total_pairs"])
        r.close()
    plain_rate = len(objs) / sum(service)
    log(f"plain: {plain_rate:.1f} solves/s")
    ctx.trim()  # the plain solves' cached blocks: the budget is half of what is really free
    free, _ = ctx.mem_info()
    log(f"free device memory: {free / 2**30:.1f} GiB")
    rows = []
    for mult in args.serve_rates:
        lam = mult * plain_rate
        arrivals = graphs.poisson_trace(len(objs), lam, seed=4 + int(mult * 100))
        # the budget covers the dense runs' matrices; their new-pair buffers
        # (up to a quarter of the budget each) and the sparse lane's solves
        # take memory beside it, so the configured mix, whose lane requests
        # hold tens of GB, gets a quarter of the free memory
        frac = 0.25 if args.serve_mix == "configured" else 0.5
        srv = cflr.Server(ctx, hbm_budget_bytes=int(free * frac), max_slots=args.serve_slots)
        t0 = time.perf_counter()
        tickets = []
        for (gr, o), a in zip(objs, arrivals):
            now = time.perf_counter() - t0
            if a > now:
                time.sleep(a - now)
            tickets.append(srv.submit(gr, o))
        results, failed = [], []
        for q, t in enumerate(tickets):
            try:
                results.append(srv.wait(t, timeout_s=600))
            except cflr.CflrError as e:
                results.append(None)
                failed.append(f"query {q} (n={pool[q][1].n}): {e}")
                log(f"served query {q} failed: {e}")
            if q % 10 == 9:
                log(f"rate {mult}x: {q + 1} of {len(tickets)} served, {time.perf_counter() - t0:.1f} s")
        times = [srv.times(t) for t in tickets]
        srv.close()
        same = [r.stats()["total_pairs"] if r else None for r in results] == plain_pairs
        lane = sum(1 for r in results if r and r.stats()["storage"] == 2)
        for r in results:
            if r:
                r.close()
        lat = np.array([f - s for s, _, f in times])
        span = max(f for _, _, f in times) - min(s for s, _, _ in times)
        fifo = np.array(fifo_latencies(list(arrivals), service))
        row = {"rate_x_plain": mult, "offered_per_s": lam, "solves_per_s": len(objs) / span,
               "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
               "plain_fifo_p50_s": float(np.percentile(fifo, 50)),
               "plain_fifo_p99_s": float(np.percentile(fifo, 99)),
               "same_pair_counts_as_plain": same, "sparse_lane_requests": lane, "failed": failed}
        log(json.dumps(row))
        rows.append(row)
    best = max(r["solves_per_s"] for r in rows)
    cpu = None
    if not args.no_cpu:
        small = [k for k, (_, g) in enumerate(pool) if g.n <= args.batch_oracle_max_n]
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"oracle on the {len(small)} queries with n <= {args.batch_oracle_max_n}, {threads} at once ...")
        t0 = time.perf_counter()
        from concurrent.futures import ThreadPoolExecutor
        import oracle
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda k: oracle.solve(pool[k][0], pool[k][1], pairs=False, digest=False), small))
        to = time.perf_counter() - t0
        cpu = {"value": len(small) / to, "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"the {len(small)} queries of the pool with n <= {args.batch_oracle_max_n}, one oracle "
                         f"process per query, {threads} at once on the host cores ({host_cpu()}): {to:.1f} s",
               "gpu_plain_same_queries_solves_per_s": len(small) / sum(service[k] for k in small)}
    print(json.dumps({"metric": "served solves/s (continuous batching)", "value": best,
                      "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
                      "data": "synthetic", "plain_solves_per_s": plain_rate,
                      "sweep": rows, "max_slots_per_class": args.serve_slots, "cpu_baseline": cpu,
                      "config": {"workload": f"serve_mix ({args.serve_mix}): {len(objs)} queries, "
                                             + ", ".join(f"{nm} n in [{lo}, {hi}]" for nm, lo, hi in
                                                         SERVE_MIX[args.serve_mix])
                                             + " (points-to: Fig. 4b at 64 fields), n log-uniform, "
                                               "Poisson arrivals"}}),
          flush=True)


def compare_forms(cases, steps, metric):
    """Time each grammar form of each case on the case's graph (median of
    `steps` solves after one warm-up); check that the forms agree on the
    shared non-terminal (pair counts)."""
    import torch
    import paper_2401_11029_amd as cflr
    ctx = cflr.Context(0)
    rows = []
    for name, g, shared, variants in cases:
        graph = cflr.Graph.from_workload(ctx, g)
        counts = {}
        for label, text in variants:
            gr = cflr.Grammar(text)
            info = gr.info()
            r = cflr.solve(ctx, gr, graph)  # warm-up
            r.close()
            ms = []
            for k in range(max(1, steps)):
                r = cflr.solve(ctx, gr, graph)
                st = r.stats()
                ms.append(st["fixpoint_ms"])
                counts[label] = r.count(shared)
                r.close()
            torch.cuda.synchronize()
            ms.sort()
            med = ms[len(ms) // 2]
            log(f"{name} {label}: median {med:.1f} ms, {st['rounds']} rounds, "
                f"{info['matrices']} matrices, {counts[label]} {shared} pairs")
            rows.append({"graph": name, "vertices": g.n, "edges": g.m, "grammar": label,
                         "storage": "sparse" if st["storage"] == 2 else "dense",
                         "matrices": info["matrices"], "binary": info["binary"],
                         "fixpoint_ms_median": med, "rounds": st["rounds"],
                         "pairs": st["total_pairs"],
                         "derived_pairs_per_s": st["new_pairs"] / (med / 1e3) if med > 0 else None,
                         "shared_nt": shared, "shared_nt_pairs": counts[label]})
        for row in rows[-len(variants):]:
            row["same_shared_pairs"] = len(set(counts.values())) == 1
        del graph
    print(json.dumps({"metric": metric, "unit": "ms", "higher_is_better": False, "n_gpus": 1,
                      "data": "synthetic", "rows": rows}), flush=True)


def analyses_mode(args):
    """The two further analyses of the paper on graphs of their Table 3
    shapes: field-sensitive C/C++ alias (Fig. 6b by hand, Fig. 6a as given;
    64 fields, 2.7 stored edges per vertex) at 40,000 vertices, the size of
    its Table 3 graphs; context-sensitive value flow (Fig. 7b by hand, Fig.
    7a as given; 64 call sites, 1.7 edges per vertex) at 40,000 vertices and
    at the vertex and edge counts of Table 3's povray graph (346,034 and
    581,210; sparse storage, chosen by the default)."""
    import workloads
    from workloads import grammars as G, graphs
    cases = [("fsca", graphs.fsca_graph(40000, fields=64), "M",
              [("Fig. 6b (WCNF by hand)", G.fsca_fig6b(64)),
               ("Fig. 6a as given, normalised by the library", G.fsca_fig6a_cfg(64))]),
             ("cscvf", graphs.valueflow_graph(40000, m_fwd=68000, calls=64), "A",
              [("Fig. 7b (WCNF by hand)", G.cscvf_fig7b(64)),
               ("Fig. 7a as given, normalised by the library", G.cscvf_fig7a_cfg(64))]),
             ("cscvf_346k", workloads.config("valueflow_346k")[1], "A",
              [("Fig. 7b (WCNF by hand)", G.cscvf_fig7b(64)),
               ("Fig. 7a as given, normalised by the library", G.cscvf_fig7a_cfg(64))])]
    compare_forms(cases, args.steps, "fixpoint ms, field-sensitive alias and value-flow analyses")


def grammars_mode(args):
    """The paper's hand-normalised grammars (opt. 5) against the CFPQ Data
    grammars normalised automatically, on the same graph: Fig. 5a as given
    (the library binarises it), Fig. 5a binarised in the text, and Fig. 5b on
    the 50,000-vertex alias graph; the same three forms of Fig. 4a/4b at 64
    fields on a 12,000-vertex points-to graph.  All forms define the same
    relation on the shared non-terminal, checked here by pair counts."""
    import workloads
    from workloads import grammars as G, graphs
    cases = [("alias", workloads.config("alias_50k")[1], "M",
              [("Fig. 5a as given, normalised by the library", G.ALIAS_FIG5A),
               ("Fig. 5a binarised (helpers Y1..Y4)", G.ALIAS_FIG5A_WCNF),
               ("Fig. 5b (WCNF by hand)", G.ALIAS_FIG5B)]),
             ("pointsto", graphs.pointsto_graph(12000, seed=2), "PT",
              [("Fig. 4a as given, normalised by the library", G.pointsto_fig4a_cfg(64)),
               ("Fig. 4a binarised", G.pointsto_fig4a(64)),
               ("Fig. 4b (WCNF by hand)", G.pointsto_fig4b(64))])]
    compare_forms(cases, args.steps, "fixpoint ms, hand vs automatic WCNF")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="single",
                    choices=["single", "batch", "serve", "grammars", "analyses"])
    ap.add_argument("--serve-per-grammar", type=int, default=30)
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[0.5, 1.0, 2.0, 4.0, 8.0])
    ap.add_argument("--serve-slots", type=int, default=8, help="requests running at once per size class")
    ap.add_argument("--serve-mix", default="capped", choices=["capped", "configured"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="skip the memory-alias context line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB int32 read+write kernel "
                         "(reference for the HBM byte counters)")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-max-n", type=int, default=40000)
    ap.add_argument("--batch-grammar", default="alias", choices=["alias", "dyck"])
    ap.add_argument("--batch-oracle-max-n", type=int, default=8000,
                    help="graphs the oracle solves beside the batch (all host cores)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(each solve, batch or served request lives on one device)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "single":
        single(args)
    elif args.mode == "batch":
        batch(args)
    elif args.mode == "grammars":
        grammars_mode(args)
    elif args.mode == "analyses":
        analyses_mode(args)
    else:
        serve(args)
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)   # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one kernel")


if __name__ == "__main__":
    main()
