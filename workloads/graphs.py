"""Seeded synthetic edge-labelled graphs (data only: no solver arithmetic).

The paper's graphs (CFPQ Data, CPU17; Section 4) are not available, so these
generators produce stand-ins with the shapes of its Table 3: power-law
out-degree, a handful of labels for the alias analysis, thousands of field
labels for points-to, and explicit reversed ("bar") edges.

Every generator is a pure function of its arguments and seed (numpy PCG64),
returns a :class:`Graph`, deduplicates edges, and emits no self-loops unless
asked to.  Vertex ids are 0-based.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    n: int
    src: np.ndarray            # uint32 [m]
    dst: np.ndarray            # uint32 [m]
    label: np.ndarray          # uint32 [m], index into label_names
    label_names: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def edges(self):
        """Yield (u, label_name, v) triples (small graphs only)."""
        for u, v, l in zip(self.src.tolist(), self.dst.tolist(),
                           self.label.tolist()):
            yield u, self.label_names[l], v


def _u32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def make_graph(n, triples, label_names=None, meta=None) -> Graph:
    """Build a Graph from (u, label_name, v) triples (tests, small cases)."""
    triples = list(triples)
    if label_names is None:
        label_names = sorted({t[1] for t in triples})
    idx = {s: i for i, s in enumerate(label_names)}
    src = _u32([t[0] for t in triples])
    lab = _u32([idx[t[1]] for t in triples])
    dst = _u32([t[2] for t in triples])
    return Graph(n, src, dst, lab, list(label_names), dict(meta or {}))


def _distinct_pairs(rng, n, m, draw_src, allow_self=False):
    """Draw m distinct ordered pairs (u, v); u from draw_src, v uniform.

    Pairs are drawn in batches and kept in first-drawn order, so the result is
    a deterministic function of the generator state.
    """
    if n <= 1 and not allow_self:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    cap = n * n if allow_self else n * (n - 1)
    if m > cap:
        raise ValueError(f"cannot draw {m} distinct pairs on {n} vertices")
    keys = np.zeros(0, np.int64)
    while keys.shape[0] < m:
        want = max(1024, int((m - keys.shape[0]) * 1.3) + 16)
        u = draw_src(want).astype(np.int64)
        v = rng.integers(0, n, size=want, dtype=np.int64)
        if not allow_self:
            ok = u != v
            u, v = u[ok], v[ok]
        cand = np.concatenate([keys, u * n + v])
        _, first = np.unique(cand, return_index=True)
        keys = cand[np.sort(first)]
    keys = keys[:m]
    return keys // n, keys % n


def erdos_renyi(n, m, labels=("a", "b"), probs=None, seed=0) -> Graph:
    """Directed G(n, m): m distinct ordered pairs u != v drawn uniformly,
    each given a label drawn independently (uniform unless probs given)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u, v = _distinct_pairs(rng, n, m, lambda k: rng.integers(0, n, size=k))
    p = None if probs is None else np.asarray(probs, dtype=np.float64)
    lab = rng.choice(len(labels), size=u.shape[0], p=p)
    return Graph(n, _u32(u), _u32(v), _u32(lab), list(labels),
                 {"kind": "erdos_renyi", "n": n, "m": m, "seed": seed})


def _chung_lu_sources(rng, n, alpha):
    """Sampler of source vertices with power-law out-degree.

    Vertex weights w_u = (r_u + 1) ** (-1 / (alpha - 1)) over a seeded random
    rank permutation r; sources are drawn proportionally to w.
    """
    ranks = rng.permutation(n)
    w = (ranks + 1.0) ** (-1.0 / (alpha - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(k):
        return np.minimum(np.searchsorted(cdf, rng.random(k), side="right"),
                          n - 1)
    return draw


def alias_graph(n, m_fwd=None, alpha=2.1, p_d=0.5, seed=1) -> Graph:
    """Memory-alias shaped graph: forward edges labelled a (assignment) or d
    (dereference) with P(d) = p_d, sources power-law (Chung-Lu, alpha),
    targets uniform; every forward edge (u, t, v) also stored reversed as
    (v, t_bar, u).  Default m_fwd = n, i.e. a mean of 2 stored labelled edges
    per vertex, reversed ones included."""
    if m_fwd is None:
        m_fwd = n
    rng = np.random.Generator(np.random.PCG64(seed))
    u, v = _distinct_pairs(rng, n, m_fwd, _chung_lu_sources(rng, n, alpha))
    is_d = rng.random(u.shape[0]) < p_d
    names = ["a", "d", "a_bar", "d_bar"]
    lab_f = np.where(is_d, 1, 0)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    lab = np.concatenate([lab_f, lab_f + 2])
    return Graph(n, _u32(src), _u32(dst), _u32(lab), names,
                 {"kind": "alias", "n": n, "m_fwd": m_fwd, "alpha": alpha,
                  "p_d": p_d, "seed": seed})


def _zipf_fields(rng, k, fields, s):
    p = 1.0 / np.arange(1, fields + 1, dtype=np.float64) ** s
    p /= p.sum()
    return rng.choice(fields, size=k, p=p)


def pointsto_graph(n, m_fwd=None, fields=64, alpha=2.1, zipf_s=1.1,
                   class_p=(0.2, 0.4, 0.2, 0.2), seed=2) -> Graph:
    """Field-sensitive points-to shaped graph.

    Forward edge classes alloc / assign / load_f / store_f with probabilities
    class_p; the field f of loads and stores is Zipf(zipf_s) over [0, fields).
    Sources power-law (Chung-Lu, alpha), targets uniform.  Each forward edge
    (u, t, v) is also stored reversed as (v, t_bar, u).  Default m_fwd = 1.5 n,
    i.e. a mean of 3 stored labelled edges per vertex.
    """
    if m_fwd is None:
        m_fwd = (3 * n) // 2
    rng = np.random.Generator(np.random.PCG64(seed))
    u, v = _distinct_pairs(rng, n, m_fwd, _chung_lu_sources(rng, n, alpha))
    k = u.shape[0]
    cls = rng.choice(4, size=k, p=np.asarray(class_p, dtype=np.float64))
    fld = _zipf_fields(rng, k, fields, zipf_s)
    names = ["alloc", "assign", "alloc_bar", "assign_bar"]
    names += [f"load_{i}" for i in range(fields)]
    names += [f"store_{i}" for i in range(fields)]
    names += [f"load_bar_{i}" for i in range(fields)]
    names += [f"store_bar_{i}" for i in range(fields)]
    fwd = np.where(cls == 0, 0,
          np.where(cls == 1, 1,
          np.where(cls == 2, 4 + fld, 4 + fields + fld)))
    rev = np.where(cls == 0, 2,
          np.where(cls == 1, 3,
          np.where(cls == 2, 4 + 2 * fields + fld, 4 + 3 * fields + fld)))
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    lab = np.concatenate([fwd, rev])
    return Graph(n, _u32(src), _u32(dst), _u32(lab), names,
                 {"kind": "pointsto", "n": n, "m_fwd": m_fwd,
                  "fields": fields, "alpha": alpha, "zipf_s": zipf_s,
                  "class_p": list(class_p), "seed": seed})


def fsca_graph(n, m_fwd=None, fields=64, p_field=0.3, p_d=0.4, alpha=2.1,
               zipf_s=1.1, seed=6) -> Graph:
    """Field-sensitive C/C++ alias shaped graph (the labels of Fig. 6):
    forward edges are field edges f_i with probability p_field (i Zipf over
    [0, fields)), else dereference d with probability p_d or assignment a;
    sources power-law (Chung-Lu, alpha), targets uniform; every forward edge
    (u, t, v) is also stored reversed as (v, t_bar, u).  Default m_fwd =
    1.35 n, i.e. 2.7 stored labelled edges per vertex (Table 3's FSCA graphs:
    111,550 edges on 41,652 vertices, 110,874 on 38,091)."""
    if m_fwd is None:
        m_fwd = (27 * n) // 20
    rng = np.random.Generator(np.random.PCG64(seed))
    u, v = _distinct_pairs(rng, n, m_fwd, _chung_lu_sources(rng, n, alpha))
    k = u.shape[0]
    r = rng.random(k)
    is_f = r < p_field
    is_d = ~is_f & (rng.random(k) < p_d)
    fld = _zipf_fields(rng, k, fields, zipf_s)
    names = ["a", "d", "a_bar", "d_bar"]
    names += [f"f_{i}" for i in range(fields)]
    names += [f"f_bar_{i}" for i in range(fields)]
    fwd = np.where(is_f, 4 + fld, np.where(is_d, 1, 0))
    rev = np.where(is_f, 4 + fields + fld, np.where(is_d, 3, 2))
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    lab = np.concatenate([fwd, rev])
    return Graph(n, _u32(src), _u32(dst), _u32(lab), names,
                 {"kind": "fsca", "n": n, "m_fwd": m_fwd, "fields": fields,
                  "p_field": p_field, "p_d": p_d, "alpha": alpha, "seed": seed})


def valueflow_graph(n, m_fwd=None, calls=16, p_call=0.1, alpha=2.1,
                    seed=5) -> Graph:
    """Context-sensitive value-flow shaped graph: plain flow edges 'a' and
    matched call_i / ret_i edge pairs (i Zipf over [0, calls))."""
    if m_fwd is None:
        m_fwd = n
    rng = np.random.Generator(np.random.PCG64(seed))
    u, v = _distinct_pairs(rng, n, m_fwd, _chung_lu_sources(rng, n, alpha))
    k = u.shape[0]
    is_call = rng.random(k) < p_call
    site = _zipf_fields(rng, k, calls, 1.1)
    is_ret = is_call & (rng.random(k) < 0.5)
    names = ["a"] + [f"call_{i}" for i in range(calls)] + \
        [f"ret_{i}" for i in range(calls)]
    lab = np.where(~is_call, 0, np.where(is_ret, 1 + calls + site, 1 + site))
    return Graph(n, _u32(u), _u32(v), _u32(lab), names,
                 {"kind": "valueflow", "n": n, "m_fwd": m_fwd,
                  "calls": calls, "seed": seed})


def random_graph(n, m, labels, seed, dag=False, self_loops=False) -> Graph:
    """Small random multi-labelled graph for sweeps: m edges (u, t, v), with
    duplicates and (optionally) self-loops left in on purpose; dag=True
    orients every edge from the lower to the higher vertex id."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n == 0:
        m = 0
    u = rng.integers(0, max(n, 1), size=m)
    v = rng.integers(0, max(n, 1), size=m)
    if not self_loops and n > 1:
        same = u == v
        v = np.where(same, (v + 1) % n, v)
    if dag:
        lo, hi = np.minimum(u, v), np.maximum(u, v)
        keep = lo != hi
        u, v = lo[keep], hi[keep]
    lab = rng.integers(0, len(labels), size=u.shape[0])
    return Graph(n, _u32(u), _u32(v), _u32(lab), list(labels),
                 {"kind": "random", "n": n, "m": m, "seed": seed,
                  "dag": dag})


def chain(word, labels=None) -> Graph:
    """Path 0 -> 1 -> ... -> len(word) labelled by the given word."""
    n = len(word) + 1
    return make_graph(n, [(i, t, i + 1) for i, t in enumerate(word)],
                      label_names=labels)


def batch_specs(count=256, n_lo=1000, n_hi=40000, deg_lo=2.0, deg_hi=3.0,
                seed=3):
    """Sizes of a batch of independent graphs: n log-uniform in
    [n_lo, n_hi], stored mean degree uniform in [deg_lo, deg_hi] (reversed
    edges included, so forward edges = n * degree / 2); graph g is generated
    with seed 3000 + g."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count)))
    degs = rng.uniform(deg_lo, deg_hi, size=count)
    return [(int(n), float(d), 3000 + g) for g, (n, d) in
            enumerate(zip(ns, degs))]


def alias_batch(count=256, n_lo=1000, n_hi=40000, seed=3):
    out = []
    for n, deg, s in batch_specs(count, n_lo, n_hi, seed=seed):
        out.append(alias_graph(n, int(round(n * deg / 2)), seed=s))
    return out


def dyck_batch(count=256, n_lo=1000, n_hi=40000, seed=3):
    """The Dyck-1 reading of the batch: the same sizes as alias_batch, each
    graph a directed G(n, m) with labels a / b (p = 1/2) and m = n * degree
    stored edges (no reversed edges: Dyck-1 has no bar labels)."""
    return [erdos_renyi(n, int(round(n * deg)), seed=s) for n, deg, s in batch_specs(count, n_lo, n_hi, seed=seed)]


def poisson_trace(count, rate, seed=4):
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
