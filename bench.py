"""Benchmark: CFL-reachability fixpoint on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode single|batch|serve]

A step is one whole solve of the memory-alias workload: the binarised
alias grammar (Fig. 5a of the paper, 9 non-terminals, 13 matrices after
lowering) on a 50,000-vertex power-law graph (alpha 2.1, 50,000 forward a/d
edges plus their reversed a_bar/d_bar edges, seed 1).  The graph is resident
in device memory before timing starts; a step runs seeding, every round and
the convergence test.  value = derived pairs per second over the K timed
steps (pairs in the result minus pairs set by seeding).

The JSON line also carries:
  roofline      the product kernel (the dominant kernel) against HBM: the
                algorithmic bytes it must move per launch (counted on the
                device in an untimed accounting solve) over its average
                launch time (HIP events on the library's stream, timed
                steps);
  cpu_baseline  the CPU oracle on a bounded sample of the same workload (the
                same generator at 6,000 vertices), one host thread.

--mode batch / serve report the batched (256 graphs) and served forms
instead; they are not the default line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_PMC = os.path.join(ROOT, "profiles", "product_kernel_alias50k_pmc.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2401_11029_amd", "csrc", "kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per product launch from the committed rocprofv3 --pmc
    summary, or None when the kernel source changed since it was taken."""
    try:
        with open(PROFILE_PMC) as f:
            p = json.load(f)
    except (OSError, ValueError):
        return None
    if p.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return p.get("hbm_bytes_per_launch")


def cpu_baseline():
    """The oracle, as it is, on the same generator at 6,000 vertices."""
    import oracle
    import workloads
    n = 6000
    text, g = workloads.config("alias_50k", n=n)
    r = oracle.solve(text, g, pairs=False, digest=True)
    derived = sum(r.count.values()) - seeded_user_pairs(text, g)
    return {"value": derived / r.seconds, "unit": "pairs/s", "cores": 1,
            "kind": "oracle",
            "sample": f"alias generator at n={n} (seed 1), one full solve: "
                      f"{derived} derived pairs in {r.seconds:.1f} s on one host thread"}


def seeded_user_pairs(text, g):
    """Pairs that seeding puts into the grammar's non-terminals directly:
    (i, i) for x -> eps and the edges of t for x -> t."""
    from oracle.textgrammar import TextGrammar
    tg = TextGrammar(text)
    count = len(set(tg.eps)) * g.n
    names = g.label_names
    for x, y in tg.unit:
        if y in tg.terminals:
            lab = names.index(y) if y in names else -1
            sel = g.label == lab
            count += len(set(zip(g.src[sel].tolist(), g.dst[sel].tolist())))
    return count


def single(args):
    import torch
    import paper_2401_11029_amd as cflr
    import workloads
    text, g = workloads.config("alias_50k")
    log(f"workload alias_50k: n={g.n} edges={g.m}")
    ctx = cflr.Context(0)
    gr = cflr.Grammar(text)
    graph = cflr.Graph.from_workload(ctx, g)
    torch.cuda.synchronize()
    for w in range(args.warmup):
        r = cflr.solve(ctx, gr, graph)
        log(f"warmup {w}: {r.stats()['fixpoint_ms']:.1f} ms")
        r.close()
    # untimed accounting solve: algorithmic bytes of the product kernel
    r = cflr.solve(ctx, gr, graph, count_traffic=1)
    acct = r.stats()
    r.close()
    bytes_per_launch = acct["algo_bytes"] / max(1, acct["product_launches"])
    log(f"accounting: {acct['algo_bytes'] / 1e9:.1f} GB over {acct['product_launches']} launches")
    # timed steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        r = cflr.solve(ctx, gr, graph, kernel_timing=1)
        stats.append(r.stats())
        r.close()
        log(f"step {k}: {stats[-1]['fixpoint_ms']:.1f} ms, {stats[-1]['rounds']} rounds")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs = t1 - t0
    # every pair a round derives lies in a user non-terminal (helper wrappers
    # only ever hold seeded edges), so new_pairs is the derived-pair count
    derived = sum(s["new_pairs"] for s in stats)
    value = derived / secs
    launches = sum(s["product_launches"] for s in stats)
    prod_ms = sum(s["product_ms"] for s in stats)
    avg_launch_s = prod_ms / 1e3 / max(1, launches)
    achieved = bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    traffic = measured_traffic()
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
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "alias_50k: binarised memory-alias grammar (Fig. 5a) "
                               "on a 50,000-vertex power-law graph (alpha 2.1, "
                               "100,000 stored edges a/d/a_bar/d_bar, seed 1)",
                   "vertices": g.n, "edges": g.m,
                   "pairs": stats[-1]["total_pairs"],
                   "rounds": stats[-1]["rounds"],
                   "fixpoint_ms": stats[-1]["fixpoint_ms"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "product_kernel",
                     "algo_bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": avg_launch_s * 1e3},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def batch(args):
    import torch
    import paper_2401_11029_amd as cflr
    from workloads import graphs, grammars
    gs = graphs.alias_batch(args.batch_count, n_hi=args.batch_max_n)
    log(f"batch: {len(gs)} graphs, n {min(g.n for g in gs)}..{max(g.n for g in gs)}")
    ctx = cflr.Context(0)
    gr = cflr.Grammar(grammars.ALIAS_FIG5A_WCNF)
    objs = [cflr.Graph.from_workload(ctx, g) for g in gs]
    for r in cflr.solve_batch(ctx, gr, objs):
        r.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = cflr.solve_batch(ctx, gr, objs)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    pairs = sum(r.stats()["total_pairs"] for r in res)
    for r in res:
        r.close()
    t0 = time.perf_counter()
    for o in objs:
        cflr.solve(ctx, gr, o).close()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    print(json.dumps({"metric": "batched solves/s", "value": len(gs) / tb, "unit": "solves/s",
                      "sequential_solves_per_s": len(gs) / ts, "speedup": ts / tb,
                      "pairs": pairs, "graphs": len(gs)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="single", choices=["single", "batch"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB int32 read+write kernel "
                         "(reference for the HBM byte counters)")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-max-n", type=int, default=40000)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(each solve, batch or served request lives on one device)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "single":
        single(args)
    else:
        batch(args)
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)   # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one kernel")


if __name__ == "__main__":
    main()
