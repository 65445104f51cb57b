"""CFL-reachability on AMD MI355X: Python binding of libcflr.

Every step of the solve runs in the HIP kernels of ``libcflr.so``; this
module only marshals arguments (numpy arrays or torch tensors in, numpy or
torch tensors out).  It raises ImportError at first use if the library has
not been built, and has no other code path.

    import paper_2401_11029_amd as cflr
    ctx = cflr.Context()                       # device 0, own stream
    g = cflr.Grammar("S -> S S | a | eps")
    gr = cflr.Graph(ctx, n, src, dst, label, ["a"])
    r = cflr.solve(ctx, g, gr)
    src, dst = r.pairs("S")
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import Opts, Stats, GrammarInfo, STATUS_NAMES

__all__ = ["CflrError", "Context", "Grammar", "Graph", "Result", "Server",
           "solve", "solve_noalloc", "solve_batch", "autotune", "opts", "lib"]


class CflrError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def lib():
    return _lib.load()


def _check(status):
    if status != _lib.OK:
        msg = lib().cflr_last_error()
        raise CflrError(status, msg.decode() if msg else "")


def opts(**kw) -> Opts:
    o = Opts()
    lib().cflr_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, int(v))
    return o


class Context:
    """A HIP device and stream.  stream: a torch.cuda.Stream, a raw
    hipStream_t (int), or None for a stream the library creates."""

    def __init__(self, device: int = 0, stream=None):
        ptr = None
        if stream is not None:
            ptr = getattr(stream, "cuda_stream", stream)
        h = C.c_void_p()
        _check(lib().cflr_ctx_create(int(device), C.c_void_p(ptr), C.byref(h)))
        self._h = h
        self.device = device
        self._servers = 0  # servers alive on this context (no other solves meanwhile)

    def _no_server(self):
        if self._servers:
            raise RuntimeError("a Server is running on this Context: close it before other solves")

    def mem_info(self):
        f, t = C.c_uint64(), C.c_uint64()
        _check(lib().cflr_ctx_mem_info(self._h, C.byref(f), C.byref(t)))
        return f.value, t.value

    def trim(self):
        """Free the device blocks the context's pool keeps for reuse."""
        self._no_server()
        _check(lib().cflr_ctx_trim(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().cflr_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grammar:
    """Grammar text in (relaxed) weak Chomsky normal form; see cflr.h."""

    def __init__(self, text: str):
        b = text.encode("utf-8")
        h = C.c_void_p()
        _check(lib().cflr_grammar_parse(b, len(b), C.byref(h)))
        self._h = h

    @property
    def nonterminals(self):
        L = lib()
        k = L.cflr_grammar_num_nonterminals(self._h)
        return [L.cflr_grammar_nonterminal_name(self._h, i).decode()
                for i in range(k)]

    @property
    def terminals(self):
        L = lib()
        k = L.cflr_grammar_num_terminals(self._h)
        return [L.cflr_grammar_terminal_name(self._h, i).decode() for i in range(k)]

    @property
    def symbols(self):
        """Symbol numbering of witnesses: non-terminals, then terminals."""
        return self.nonterminals + self.terminals

    def info(self) -> dict:
        i = GrammarInfo()
        _check(lib().cflr_grammar_info_get(self._h, C.byref(i)))
        return i.as_dict()

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().cflr_grammar_free(self._h)
                self._h = None
        except Exception:
            pass


def _u32_buffer(a):
    """(pointer, on_device, keepalive) for a uint32 numpy array or a torch
    int32/uint32 tensor (host or device)."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            if a.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
                a = a.to(torch.int32)
            a = a.contiguous()
            return a.data_ptr(), int(a.is_cuda), a
    except ImportError:
        pass
    arr = np.ascontiguousarray(np.asarray(a), dtype=np.uint32)
    return arr.ctypes.data, 0, arr


class Graph:
    """Edge-labelled graph copied into device memory: edge e is
    (src[e], label_names[label[e]], dst[e])."""

    def __init__(self, ctx: Context, n: int, src, dst, label, label_names):
        ps, ds, ks = _u32_buffer(src)
        pd, dd, kd = _u32_buffer(dst)
        pl, dl, kl = _u32_buffer(label)
        if not (ds == dd == dl):
            raise ValueError("src, dst and label must all be host or all device")
        m = int(len(ks))
        names = [s.encode("utf-8") for s in label_names]
        arr = (C.c_char_p * max(1, len(names)))(*names)
        h = C.c_void_p()
        _check(lib().cflr_graph_create(ctx._h, int(n), m, C.c_void_p(ps), C.c_void_p(pd),
                                       C.c_void_p(pl), len(names), arr, ds, C.byref(h)))
        self._h = h
        self.ctx = ctx
        self.n = n
        self.m = m

    @classmethod
    def from_workload(cls, ctx, g):
        """From a workloads.Graph."""
        return cls(ctx, g.n, g.src, g.dst, g.label, g.label_names)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().cflr_graph_free(self._h)
                self._h = None
        except Exception:
            pass


class Result:
    def __init__(self, h, grammar: Grammar):
        self._h = h
        self.grammar = grammar
        self._names = grammar.nonterminals

    def _nt(self, nt):
        return self._names.index(nt) if isinstance(nt, str) else int(nt)

    def count(self, nt) -> int:
        c = C.c_uint64()
        _check(lib().cflr_result_count(self._h, self._nt(nt), C.byref(c)))
        return c.value

    def counts(self) -> dict:
        return {x: self.count(x) for x in self._names}

    def pairs(self, nt, device=None):
        """(src, dst) of nt sorted by (src, dst): numpy uint32 arrays, or
        torch int32 tensors on `device` when given."""
        k = self._nt(nt)
        cnt = self.count(k)
        w = C.c_uint64()
        if device is not None:
            import torch
            s = torch.empty(cnt, dtype=torch.int32, device=device)
            d = torch.empty(cnt, dtype=torch.int32, device=device)
            _check(lib().cflr_result_copy(self._h, k, C.c_void_p(s.data_ptr()),
                                          C.c_void_p(d.data_ptr()), cnt, 1, C.byref(w)))
            return s, d
        s = np.empty(cnt, dtype=np.uint32)
        d = np.empty(cnt, dtype=np.uint32)
        _check(lib().cflr_result_copy(self._h, k, C.c_void_p(s.ctypes.data),
                                      C.c_void_p(d.ctypes.data), cnt, 0, C.byref(w)))
        return s, d

    def witness(self, nt, device=None):
        """One derivation per pair of nt, in the order of pairs(nt), for a
        solve with witness=1: (left, right, mid, round) arrays -- see
        cflr_result_witness; symbols index Grammar.symbols and NONE
        (0xFFFFFFFF) marks an absent field.  numpy uint32 arrays, or torch
        int32 tensors on `device` when given."""
        k = self._nt(nt)
        cnt = self.count(k)
        w = C.c_uint64()
        if device is not None:
            import torch
            out = [torch.empty(cnt, dtype=torch.int32, device=device) for _ in range(4)]
            ptrs = [C.c_void_p(t.data_ptr()) for t in out]
            _check(lib().cflr_result_witness(self._h, k, *ptrs, cnt, 1, C.byref(w)))
            return tuple(out)
        out = [np.empty(cnt, dtype=np.uint32) for _ in range(4)]
        ptrs = [C.c_void_p(a.ctypes.data) for a in out]
        _check(lib().cflr_result_witness(self._h, k, *ptrs, cnt, 0, C.byref(w)))
        return tuple(out)

    def pair_set(self, nt):
        s, d = self.pairs(nt)
        return set(zip(s.tolist(), d.tolist()))

    def stats(self) -> dict:
        st = Stats()
        _check(lib().cflr_result_stats(self._h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().cflr_result_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(ctx: Context, grammar: Grammar, graph: Graph, options: Opts | None = None,
          **kw) -> Result:
    ctx._no_server()
    o = options if options is not None else opts(**kw)
    h = C.c_void_p()
    st = lib().cflr_solve(ctx._h, grammar._h, graph._h, C.byref(o), C.byref(h))
    if st != _lib.OK:
        if h.value:
            lib().cflr_result_free(h)
        _check(st)
    return Result(h, grammar)


def solve_noalloc(ctx: Context, grammar: Grammar, n: int, src, dst, label, label_names,
                  capacity: int, options: Opts | None = None, **kw):
    """The solve of ``solve`` without device allocation (cflr_solve_noalloc):
    src/dst/label are int32 or uint32 torch tensors on ctx's device, the
    pairs come back in two int32 tensors of ``capacity`` entries allocated
    here (by torch, before the call): returns (counts dict, src, dst, stats),
    each non-terminal's pairs sorted by (i, j), one after another in
    non-terminal order, in src[:total], dst[:total]."""
    import torch
    ctx._no_server()
    ps, ds, ks = _u32_buffer(src)
    pd, dd, kd = _u32_buffer(dst)
    pl, dl, kl = _u32_buffer(label)
    if not (ds and dd and dl):
        raise ValueError("src, dst and label must be device tensors")
    o = options if options is not None else opts(**kw)
    names = [s.encode("utf-8") for s in label_names]
    arr = (C.c_char_p * max(1, len(names)))(*names)
    dev = ks.device
    out_s = torch.empty(max(1, capacity), dtype=torch.int32, device=dev)
    out_d = torch.empty(max(1, capacity), dtype=torch.int32, device=dev)
    nts = grammar.nonterminals
    counts = (C.c_uint64 * max(1, len(nts)))()
    st = Stats()
    torch.cuda.synchronize(dev)
    _check(lib().cflr_solve_noalloc(ctx._h, grammar._h, int(n), int(len(ks)), C.c_void_p(ps), C.c_void_p(pd),
                                    C.c_void_p(pl), len(names), arr, C.byref(o), C.c_void_p(out_s.data_ptr()),
                                    C.c_void_p(out_d.data_ptr()), int(capacity), counts, C.byref(st)))
    return {x: counts[k] for k, x in enumerate(nts)}, out_s, out_d, st.as_dict()


def solve_batch(ctx: Context, grammars, graphs, options: Opts | None = None, **kw):
    """Solve many graphs together; grammars is one Grammar or one per graph."""
    ctx._no_server()
    graphs = list(graphs)
    if isinstance(grammars, Grammar):
        grammars = [grammars] * len(graphs)
    grammars = list(grammars)
    o = options if options is not None else opts(**kw)
    n = len(graphs)
    ga = (C.c_void_p * max(1, n))(*[g._h.value for g in grammars])
    gr = (C.c_void_p * max(1, n))(*[g._h.value for g in graphs])
    outs = (C.c_void_p * max(1, n))()
    st = lib().cflr_solve_batch(ctx._h, ga, gr, n, C.byref(o), outs)
    res = [Result(C.c_void_p(outs[k]), grammars[k]) if outs[k] else None
           for k in range(n)]
    _check(st)
    return res


def autotune(ctx: Context, grammars, graphs):
    """Pick the product grid (and, for several graphs, rounds per graph
    replay; on dense storage the work-item size, on sparse storage the
    heavy-bucket threshold) by timing each candidate; later solves on ctx
    use the choice."""
    ctx._no_server()
    graphs = list(graphs)
    if isinstance(grammars, Grammar):
        grammars = [grammars] * len(graphs)
    n = len(graphs)
    ga = (C.c_void_p * n)(*[g._h.value for g in grammars])
    gr = (C.c_void_p * n)(*[g._h.value for g in graphs])
    w, r, ms = C.c_uint32(), C.c_uint32(), C.c_double()
    _check(lib().cflr_autotune(ctx._h, ga, gr, n, C.byref(w), C.byref(r), C.byref(ms)))
    t = Opts()
    _check(lib().cflr_ctx_tuned(ctx._h, C.byref(t)))
    return {"grid_waves": w.value, "rounds_per_sync": r.value, "chunk_pairs": t.chunk_pairs,
            "sparse_heavy": t.sparse_heavy, "best_ms": ms.value}


class Server:
    """Continuous-batching request loop (see cflr.h)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int = 64,
                 options: Opts | None = None, **kw):
        o = options if options is not None else opts(**kw)
        h = C.c_void_p()
        _check(lib().cflr_server_create(ctx._h, int(hbm_budget_bytes), int(max_slots),
                                        C.byref(o), C.byref(h)))
        self._h = h
        self._ctx = ctx
        ctx._servers += 1
        self._keep = {}      # ticket -> grammar, until its result is taken
        self._inputs = []    # every grammar and graph submitted, alive until close()

    def submit(self, grammar: Grammar, graph: Graph) -> int:
        t = C.c_uint64()
        _check(lib().cflr_server_submit(self._h, grammar._h, graph._h, C.byref(t)))
        self._keep[t.value] = (grammar, graph)
        self._inputs.append((grammar, graph))
        return t.value

    def poll(self, ticket):
        h = C.c_void_p()
        st = lib().cflr_server_poll(self._h, ticket, C.byref(h))
        if st == _lib.PENDING:
            return None
        g, _ = self._keep.pop(ticket)
        _check(st)
        return Result(h, g)

    def wait(self, ticket, timeout_s: float = 600.0):
        h = C.c_void_p()
        st = lib().cflr_server_wait(self._h, ticket, int(timeout_s * 1e9), C.byref(h))
        if st == _lib.ETIMEOUT and not h.value:
            _check(st)
        g, _ = self._keep.pop(ticket)
        _check(st)
        return Result(h, g)

    def times(self, ticket):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(lib().cflr_server_times(self._h, ticket, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def close(self):
        if getattr(self, "_h", None):
            lib().cflr_server_free(self._h)
            self._h = None
            self._ctx._servers -= 1
            self._inputs = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
