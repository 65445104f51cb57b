"""ctypes declarations of libcflr (include/cflr.h).  Marshalling only."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcflr.so")

OK, EINVAL, EPARSE, ENOMEM, EDEVICE, PENDING, ETIMEOUT, EUNSUPPORTED = range(8)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "EPARSE", 3: "ENOMEM", 4: "EDEVICE",
                5: "PENDING", 6: "ETIMEOUT", 7: "EUNSUPPORTED"}


class Opts(C.Structure):
    _fields_ = [("max_rounds", C.c_uint32),
                ("semi_naive", C.c_uint32),
                ("kernel_timing", C.c_uint32),
                ("count_traffic", C.c_uint32),
                ("delta_capacity", C.c_uint64),
                ("grid_waves", C.c_uint32),
                ("rounds_per_sync", C.c_uint32),
                ("chunk_pairs", C.c_uint32),
                ("storage", C.c_uint32),
                ("witness", C.c_uint32),
                ("mirror", C.c_uint32),
                ("sparse_heavy", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [("rounds", C.c_uint32),
                ("reruns", C.c_uint32),
                ("seed_pairs", C.c_uint64),
                ("new_pairs", C.c_uint64),
                ("total_pairs", C.c_uint64),
                ("fixpoint_ms", C.c_double),
                ("product_ms", C.c_double),
                ("product_launches", C.c_uint64),
                ("algo_bytes", C.c_uint64),
                ("device_bytes", C.c_uint64),
                ("max_delta", C.c_uint64),
                ("storage", C.c_uint32),
                ("heavy_ms", C.c_double),
                ("heavy_launches", C.c_uint64),
                ("heavy_algo_bytes", C.c_uint64),
                ("light_ms", C.c_double),
                ("light_algo_bytes", C.c_uint64),
                ("mirror", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GrammarInfo(C.Structure):
    _fields_ = [("user_nonterminals", C.c_uint32),
                ("wrappers", C.c_uint32),
                ("matrices", C.c_uint32),
                ("binary", C.c_uint32),
                ("terminal_rules", C.c_uint32),
                ("eps_rules", C.c_uint32),
                ("terminals", C.c_uint32),
                ("helpers", C.c_uint32),
                ("mirror_skipped", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


P = C.c_void_p
U32P = C.POINTER(C.c_uint32)

# name -> (restype, argtypes); the full exported surface of cflr.h
SIGNATURES = {
    "cflr_opts_default": (None, [C.POINTER(Opts)]),
    "cflr_last_error": (C.c_char_p, []),
    "cflr_version": (C.c_char_p, []),
    "cflr_ctx_create": (C.c_int, [C.c_int, P, C.POINTER(P)]),
    "cflr_ctx_destroy": (None, [P]),
    "cflr_ctx_mem_info": (C.c_int, [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "cflr_ctx_tuned": (C.c_int, [P, C.POINTER(Opts)]),
    "cflr_ctx_trim": (C.c_int, [P]),
    "cflr_grammar_parse": (C.c_int, [C.c_char_p, C.c_size_t, C.POINTER(P)]),
    "cflr_grammar_free": (None, [P]),
    "cflr_grammar_num_nonterminals": (C.c_uint32, [P]),
    "cflr_grammar_nonterminal_name": (C.c_char_p, [P, C.c_uint32]),
    "cflr_grammar_info_get": (C.c_int, [P, C.POINTER(GrammarInfo)]),
    "cflr_grammar_num_terminals": (C.c_uint32, [P]),
    "cflr_grammar_terminal_name": (C.c_char_p, [P, C.c_uint32]),
    "cflr_graph_create": (C.c_int, [P, C.c_uint32, C.c_uint64, P, P, P, C.c_uint32,
                                    C.POINTER(C.c_char_p), C.c_int, C.POINTER(P)]),
    "cflr_graph_free": (None, [P]),
    "cflr_solve": (C.c_int, [P, P, P, C.POINTER(Opts), C.POINTER(P)]),
    "cflr_solve_noalloc": (C.c_int, [P, P, C.c_uint32, C.c_uint64, P, P, P, C.c_uint32,
                                     C.POINTER(C.c_char_p), C.POINTER(Opts), P, P, C.c_uint64,
                                     C.POINTER(C.c_uint64), C.POINTER(Stats)]),
    "cflr_solve_batch": (C.c_int, [P, C.POINTER(P), C.POINTER(P), C.c_uint32,
                                   C.POINTER(Opts), C.POINTER(P)]),
    "cflr_autotune": (C.c_int, [P, C.POINTER(P), C.POINTER(P), C.c_uint32,
                                C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                C.POINTER(C.c_double)]),
    "cflr_result_count": (C.c_int, [P, C.c_uint32, C.POINTER(C.c_uint64)]),
    "cflr_result_copy": (C.c_int, [P, C.c_uint32, P, P, C.c_uint64, C.c_int,
                                   C.POINTER(C.c_uint64)]),
    "cflr_result_witness": (C.c_int, [P, C.c_uint32, P, P, P, P, C.c_uint64, C.c_int,
                                      C.POINTER(C.c_uint64)]),
    "cflr_result_stats": (C.c_int, [P, C.POINTER(Stats)]),
    "cflr_result_free": (None, [P]),
    "cflr_server_create": (C.c_int, [P, C.c_uint64, C.c_uint32, C.POINTER(Opts),
                                     C.POINTER(P)]),
    "cflr_server_submit": (C.c_int, [P, P, P, C.POINTER(C.c_uint64)]),
    "cflr_server_poll": (C.c_int, [P, C.c_uint64, C.POINTER(P)]),
    "cflr_server_wait": (C.c_int, [P, C.c_uint64, C.c_uint64, C.POINTER(P)]),
    "cflr_server_times": (C.c_int, [P, C.c_uint64, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cflr_server_free": (None, [P]),
}

_lib = None


def _torch_first():
    """torch carries its own HIP runtime.  Loaded and started after the
    library's, it leaves one of the two without a device; so, when torch is
    installed, it is imported and its runtime started before the library is
    loaded."""
    try:
        import torch
    except ImportError:
        return
    torch.cuda.is_available()


def load(path: str = LIB_PATH):
    """Load libcflr.so; raises if it has not been built (there is no other
    implementation to fall back to)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with "
            "`python -m paper_2401_11029_amd.build` (hipcc, gfx950)")
    _torch_first()
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
