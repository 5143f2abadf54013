"""ctypes binding of libkappa.so (include/kappa.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.

Tensors are torch CUDA (HIP) tensors; weights travel as int32 tensors whose
bits the library reads as uint32.  Work is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass
from typing import List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkappa.so")
HEADER = os.path.join(HERE, "..", "include", "kappa.h")

OK, E_ARG, E_GRAPH, E_RANGE, E_NOMEM, E_CAPACITY, E_HIP = 0, -1, -2, -3, -4, -5, -6
EXPANSION_STAR2, INNER_OUTER, WEIGHT, EXPANSION, EXPANSION_STAR = 0, 1, 2, 3, 4
RATINGS = {"expansion*2": 0, "innerOuter": 1, "weight": 2, "expansion": 3, "expansion*": 4}
STOP_NONE, STOP_SIZE, STOP_EMPTY, STOP_STALL, STOP_MAXLEVEL = 0, 1, 2, 3, 4


class KappaError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        super().__init__(f"{fn} failed: {status} ({status_str(status)})")


TUNING_FIELDS = ("bin_small_max", "tail_max", "finish_max", "finish_max_big", "row_small_max",
                 "scan_one_block_max", "rounds_base", "rounds_n0", "rounds_growth", "rounds_cap")


class c_tuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in TUNING_FIELDS]


class c_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("xadj", ctypes.c_void_p),
                ("adj", ctypes.c_void_p), ("ew", ctypes.c_void_p), ("vw", ctypes.c_void_p)]


class c_graph_out(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("cap_n", ctypes.c_int32),
                ("cap_nnz", ctypes.c_int64), ("xadj", ctypes.c_void_p), ("adj", ctypes.c_void_p),
                ("ew", ctypes.c_void_p), ("vw", ctypes.c_void_p)]


class c_params(ctypes.Structure):
    _fields_ = [("rating", ctypes.c_int32), ("seed", ctypes.c_uint64), ("stop_n", ctypes.c_int32),
                ("stall_num", ctypes.c_uint32), ("stall_den", ctypes.c_uint32),
                ("max_levels", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("block_bits", ctypes.c_int32)]


COARSEN_TRUSTED = 1   # the graph passed kappa_validate: only its offsets are checked again
COARSEN_TWO_PHASE = 2   # every level matched by the two-phase matcher (blocks of 2^block_bits ids)
BLOCK_BITS_MAX = 11


class c_cut(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("cut", "total", "max_block", "max_node", "lmax_num",
                                                 "lmax_den", "imb_num", "bal_num", "bal_den")] + \
               [("feasible", ctypes.c_int64)]

    def as_tuple(self):
        return (self.cut, self.total, self.max_block, self.max_node, self.lmax_num, self.lmax_den,
                self.imb_num, self.bal_num, self.bal_den, int(self.feasible))


class c_refine_params(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("alpha_num", ctypes.c_uint32),
                ("alpha_den", ctypes.c_uint32), ("depth", ctypes.c_int32),
                ("max_local", ctypes.c_int32), ("max_global", ctypes.c_int32),
                ("stop_after", ctypes.c_int32)]


class c_refine_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("global_iterations", "searches", "moves", "kept",
                                               "adoptions", "colours", "bytes", "init_ticks",
                                               "move_ticks")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


# Presets of Table 2 (minimal, fast, strong): alpha, BFS depth, local
# iterations, max. global iterations, global iterations without change that end it
REFINE_PRESETS = {
    "minimal": dict(alpha_num=1, alpha_den=100, depth=1, max_local=1, max_global=1, stop_after=1),
    "fast": dict(alpha_num=5, alpha_den=100, depth=5, max_local=3, max_global=15, stop_after=1),
    "strong": dict(alpha_num=20, alpha_den=100, depth=20, max_local=5, max_global=15,
                   stop_after=2),
}
REFINE_K_MAX = 256


def refine_params(preset: str = "fast", seed: int = 1, **over) -> c_refine_params:
    d = dict(REFINE_PRESETS[preset])
    d.update(over)
    return c_refine_params(seed=seed & 0xFFFFFFFFFFFFFFFF, **d)


class c_level_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("matched", ctypes.c_int64), ("stop_reason", ctypes.c_int32),
                ("grid_rounds", ctypes.c_int32)]


_lib = None

# kappa_set_allocator callbacks (kept referenced while installed)
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_allocator = None


def declared_functions() -> List[str]:
    """Names of the functions declared in include/kappa.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kappa_[a-z_0-9]+)\s*\(", text)))


def lib():
    """Loads libkappa.so.  Raises if it is missing: there is no fallback.

    torch is imported first: its wheel carries its own HIP runtime, and the
    library must bind to that one (libamdhip64.so.7 already in the process)
    rather than load a second runtime from /opt/rocm, whose device memory and
    streams torch's tensors and streams would not belong to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_0910_2004_amd/build.py")
    import torch  # noqa: F401  (loads torch's HIP runtime before the library)
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    st = ctypes.c_int
    sig = {
        "kappa_validate": (st, [ctypes.POINTER(c_graph), P]),
        "kappa_rate": (st, [ctypes.POINTER(c_graph), i32, P, P, P]),
        "kappa_match": (st, [ctypes.POINTER(c_graph), i32, u64, P, ctypes.POINTER(i32),
                             ctypes.POINTER(i64), P]),
        "kappa_match_two_phase": (st, [ctypes.POINTER(c_graph), i32, u64, i32, P, P,
                                       ctypes.POINTER(i64), P]),
        "kappa_rcb_order": (st, [P, i32, i32, P, P]),
        "kappa_relabel": (st, [ctypes.POINTER(c_graph), P, ctypes.POINTER(c_graph_out), P]),
        "kappa_contract": (st, [ctypes.POINTER(c_graph), P, P, ctypes.POINTER(c_graph_out), P]),
        "kappa_coarsen": (st, [ctypes.POINTER(c_graph), ctypes.POINTER(c_params),
                               ctypes.POINTER(P), P]),
        "kappa_hierarchy_levels": (i32, [P]),
        "kappa_hierarchy_level": (st, [P, i32, ctypes.POINTER(c_graph), ctypes.POINTER(P),
                                       ctypes.POINTER(c_level_info)]),
        "kappa_hierarchy_round_stats": (i32, [P, i32, P, P, i32]),
        "kappa_hierarchy_rescan_stats": (i32, [P, i32, P, P, i32]),
        "kappa_hierarchy_free": (None, [P]),
        "kappa_initial_partition": (st, [i32, i32, u64, P, P]),
        "kappa_project": (st, [P, i32, i32, P, P, P]),
        "kappa_cut_balance": (st, [ctypes.POINTER(c_graph), P, i32, u32, u32, P,
                                   ctypes.POINTER(c_cut), P]),
        "kappa_cut_balance_noalloc": (st, [ctypes.POINTER(c_graph), P, i32, u32, u32, P,
                                           ctypes.POINTER(c_cut), P]),
        "kappa_uncoarsen": (st, [P, i32, u64, u32, u32, P, P, P]),
        "kappa_refine": (st, [ctypes.POINTER(c_graph), P, i32, u32, u32,
                              ctypes.POINTER(c_refine_params), ctypes.POINTER(c_refine_stats), P]),
        "kappa_uncoarsen_refined": (st, [P, i32, u64, u32, u32, ctypes.POINTER(c_refine_params),
                                         P, P, P, P]),
        "kappa_profile_enable": (None, [i32]),
        "kappa_profile_reset": (None, []),
        "kappa_profile_read": (i32, [P, P, P, i32]),
        "kappa_coarsen_batch": (st, [ctypes.POINTER(c_graph), i32, P, P, ctypes.POINTER(c_params),
                                     ctypes.POINTER(P), P]),
        "kappa_coarsen_graphs": (st, [P, i32, P, ctypes.POINTER(c_params), ctypes.POINTER(P), P]),
        "kappa_server_create": (st, [ctypes.POINTER(c_params), ctypes.POINTER(P), P]),
        "kappa_server_admit": (st, [P, ctypes.POINTER(c_graph), i32, ctypes.POINTER(ctypes.c_int64)]),
        "kappa_server_active": (i32, [P]),
        "kappa_server_step": (st, [P, P, i32, ctypes.POINTER(i32)]),
        "kappa_server_interrupt": (st, [P, i32]),
        "kappa_persistent_enable": (None, [i32]),
        "kappa_tuning_get": (st, [ctypes.POINTER(c_tuning)]),
        "kappa_tuning_set": (st, [ctypes.POINTER(c_tuning)]),
        "kappa_tuning_load": (st, [ctypes.c_char_p]),
        "kappa_server_take": (st, [P, ctypes.c_int64, ctypes.POINTER(P)]),
        "kappa_server_free": (None, [P]),
        "kappa_batch_count": (i32, [P]),
        "kappa_batch_graph_info": (st, [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "kappa_batch_hierarchy": (st, [P, i32, ctypes.POINTER(P), P]),
        "kappa_batch_free": (None, [P]),
        "kappa_cache_release": (st, []),
        "kappa_graphs_enable": (None, [i32]),
        "kappa_arena_first": (None, [u64]),
        "kappa_tail_enable": (None, [i32]),
        "kappa_set_allocator": (st, [_ALLOC_FN, _FREE_FN, P]),
        "kappa_status_str": (ctypes.c_char_p, [st]),
        "kappa_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def status_str(st: int) -> str:
    try:
        return lib().kappa_status_str(st).decode()
    except Exception:
        return "?"


def _check(fn: str, st: int):
    if st != OK:
        raise KappaError(fn, st)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# HIP runtime copy (used to read library-owned hierarchy arrays into tensors)
# ---------------------------------------------------------------------------
_hip = None


def _hip_rt():
    global _hip
    if _hip is None:
        lib()   # the runtime the library is bound to, not a second one
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.restype = ctypes.c_int
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int, ctypes.c_void_p]
    return _hip


def _copy_from_ptr(ptr: int, count: int, dtype, device):
    import torch
    out = torch.empty(max(count, 0), dtype=dtype, device=device)
    if count > 0 and ptr:
        nbytes = count * out.element_size()
        r = _hip_rt().hipMemcpyAsync(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr), nbytes,
                                     3, _stream())
        if r != 0:
            raise RuntimeError(f"hipMemcpyAsync failed: {r}")
    return out


# ---------------------------------------------------------------------------
# Graphs on the device
# ---------------------------------------------------------------------------
@dataclass
class DeviceGraph:
    n: int
    nnz: int
    xadj: object   # torch.int64 [n+1]
    adj: object    # torch.int32 [nnz]
    ew: object     # torch.int32 [nnz] (uint32 bits)
    vw: object     # torch.int32 [n]   (uint32 bits)

    def c(self) -> c_graph:
        return c_graph(self.n, self.nnz, self.xadj.data_ptr(),
                       self.adj.data_ptr() if self.nnz else None,
                       self.ew.data_ptr() if self.nnz else None,
                       self.vw.data_ptr() if self.n else None)

    @staticmethod
    def from_csr(g, device="cuda") -> "DeviceGraph":
        import numpy as np
        import torch
        # no host copy when the arrays already have these types (the weights'
        # uint32 bits travel as int32)
        xadj = torch.from_numpy(np.ascontiguousarray(g.xadj, dtype=np.int64)).to(device)
        adj = torch.from_numpy(np.ascontiguousarray(g.adj, dtype=np.int32)).to(device)
        ew = torch.from_numpy(np.ascontiguousarray(g.ew, dtype=np.uint32).view(np.int32)).to(device)
        vw = torch.from_numpy(np.ascontiguousarray(g.vw, dtype=np.uint32).view(np.int32)).to(device)
        return DeviceGraph(int(g.n), int(g.xadj[-1]), xadj, adj, ew, vw)

    @staticmethod
    def union(graphs, device="cuda"):
        """The block-diagonal union of host graphs on the device, and its
        node_off (the batched form's input)."""
        import numpy as np
        import torch
        n, xadj, adj, ew, vw, off = union_csr(graphs)
        dg = DeviceGraph(n, int(xadj[-1]), torch.from_numpy(xadj).to(device),
                         torch.from_numpy(adj).to(device),
                         torch.from_numpy(ew.view(np.int32)).to(device),
                         torch.from_numpy(vw.view(np.int32)).to(device))
        return dg, off

    def numpy(self):
        """(xadj, adj, ew, vw) as numpy arrays (ew, vw as uint32)."""
        import numpy as np
        return (self.xadj.cpu().numpy(), self.adj.cpu().numpy(),
                self.ew.cpu().numpy().view(np.uint32), self.vw.cpu().numpy().view(np.uint32))


def kappa_validate(g: DeviceGraph) -> int:
    return int(lib().kappa_validate(ctypes.byref(g.c()), _stream()))


def kappa_rate(g: DeviceGraph, rating: int):
    """Returns (num, den) as int64 tensors holding uint64 bits."""
    import torch
    num = torch.empty(max(g.nnz, 1), dtype=torch.int64, device=g.xadj.device)
    den = torch.empty(max(g.nnz, 1), dtype=torch.int64, device=g.xadj.device)
    _check("kappa_rate", lib().kappa_rate(ctypes.byref(g.c()), rating, _ptr(num), _ptr(den), _stream()))
    return num[:g.nnz], den[:g.nnz]


def kappa_match(g: DeviceGraph, rating: int, level_seed: int):
    import torch
    mate = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.xadj.device)
    rounds = ctypes.c_int32(0)
    matched = ctypes.c_int64(0)
    _check("kappa_match", lib().kappa_match(ctypes.byref(g.c()), rating,
                                            ctypes.c_uint64(level_seed & (2**64 - 1)), _ptr(mate),
                                            ctypes.byref(rounds), ctypes.byref(matched), _stream()))
    return mate[:g.n], int(rounds.value), int(matched.value)


def kappa_match_two_phase(g: DeviceGraph, rating: int, level_seed: int, block_bits: int):
    """Returns (mate, block-phase matching, |M|)."""
    import torch
    mate = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.xadj.device)
    loc = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.xadj.device)
    matched = ctypes.c_int64(0)
    _check("kappa_match_two_phase",
           lib().kappa_match_two_phase(ctypes.byref(g.c()), rating,
                                       ctypes.c_uint64(level_seed & (2**64 - 1)), block_bits,
                                       _ptr(mate), _ptr(loc), ctypes.byref(matched), _stream()))
    return mate[:g.n], loc[:g.n], int(matched.value)


def kappa_rcb_order(xy, leaf: int = 32):
    """Recursive coordinate bisection order of the points xy (float64 device
    tensor [n, 2]); returns order (int32 [n]), order[x] = the point at x."""
    import torch
    xy = xy.to(torch.float64).contiguous()
    n = int(xy.shape[0])
    order = torch.empty(max(n, 1), dtype=torch.int32, device=xy.device)
    _check("kappa_rcb_order", lib().kappa_rcb_order(_ptr(xy), n, leaf, _ptr(order), _stream()))
    return order[:n]


def kappa_relabel(g: DeviceGraph, order) -> DeviceGraph:
    """g renumbered: node x of the result is node order[x] of g."""
    import torch
    dev = g.xadj.device
    cx = torch.empty(g.n + 1, dtype=torch.int64, device=dev)
    ca = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
    ce = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
    cv = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    order = order.to(torch.int32).contiguous()
    out = c_graph_out(0, 0, g.n, g.nnz, cx.data_ptr(), ca.data_ptr(), ce.data_ptr(), cv.data_ptr())
    _check("kappa_relabel", lib().kappa_relabel(ctypes.byref(g.c()), _ptr(order), ctypes.byref(out),
                                                _stream()))
    return DeviceGraph(g.n, g.nnz, cx, ca[:g.nnz], ce[:g.nnz], cv[:g.n])


def kappa_contract(g: DeviceGraph, mate, cap_n: Optional[int] = None, cap_nnz: Optional[int] = None):
    """Returns (cmap, coarse DeviceGraph)."""
    import torch
    dev = g.xadj.device
    cap_n = g.n if cap_n is None else cap_n
    cap_nnz = g.nnz if cap_nnz is None else cap_nnz
    cmap = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    cx = torch.empty(cap_n + 1, dtype=torch.int64, device=dev)
    ca = torch.empty(max(cap_nnz, 1), dtype=torch.int32, device=dev)
    ce = torch.empty(max(cap_nnz, 1), dtype=torch.int32, device=dev)
    cv = torch.empty(max(cap_n, 1), dtype=torch.int32, device=dev)
    out = c_graph_out(0, 0, cap_n, cap_nnz, cx.data_ptr(), ca.data_ptr(), ce.data_ptr(), cv.data_ptr())
    _check("kappa_contract", lib().kappa_contract(ctypes.byref(g.c()), _ptr(mate), _ptr(cmap),
                                                  ctypes.byref(out), _stream()))
    n, m = int(out.n), int(out.nnz)
    return cmap[:g.n], DeviceGraph(n, m, cx[:n + 1], ca[:m], ce[:m], cv[:n])


@dataclass
class LevelView:
    graph: DeviceGraph
    cmap: object          # torch.int32 [n] or None on the coarsest level
    rounds: int
    matched: int
    stop_reason: int


class Hierarchy:
    """Owns a kappa_hierarchy handle (freed with the object).  Keeps the input
    graph alive: level 0 of the hierarchy refers to its arrays."""

    def __init__(self, handle, device, graph=None):
        self.handle = handle
        self.device = device
        self.graph = graph

    def __del__(self):
        try:
            if self.handle:
                lib().kappa_hierarchy_free(self.handle)
                self.handle = None
        except Exception:
            pass

    def __len__(self):
        return int(lib().kappa_hierarchy_levels(self.handle))

    def info(self, l: int) -> c_level_info:
        inf = c_level_info()
        _check("kappa_hierarchy_level", lib().kappa_hierarchy_level(self.handle, l, None, None,
                                                                    ctypes.byref(inf)))
        return inf

    def round_stats(self, l: int):
        import numpy as np
        p = np.zeros(64, dtype=np.int64)
        d = np.zeros(64, dtype=np.int64)
        r = lib().kappa_hierarchy_round_stats(self.handle, l, p.ctypes.data_as(ctypes.c_void_p),
                                              d.ctypes.data_as(ctypes.c_void_p), 64)
        k = min(r, 64)
        return int(r), p[:k].copy(), d[:k].copy()

    def rescan_stats(self, l: int):
        """(rounds, rows that scanned their row again per round, their degree sum)."""
        import numpy as np
        p = np.zeros(64, dtype=np.int64)
        d = np.zeros(64, dtype=np.int64)
        r = lib().kappa_hierarchy_rescan_stats(self.handle, l, p.ctypes.data_as(ctypes.c_void_p),
                                               d.ctypes.data_as(ctypes.c_void_p), 64)
        k = min(r, 64)
        return int(r), p[:k].copy(), d[:k].copy()

    def level(self, l: int) -> LevelView:
        """Copies level l into torch tensors."""
        import torch
        g = c_graph()
        cm = ctypes.c_void_p()
        inf = c_level_info()
        _check("kappa_hierarchy_level", lib().kappa_hierarchy_level(self.handle, l, ctypes.byref(g),
                                                                    ctypes.byref(cm), ctypes.byref(inf)))
        n, m = int(g.n), int(g.nnz)
        dg = DeviceGraph(n, m, _copy_from_ptr(g.xadj, n + 1, torch.int64, self.device),
                         _copy_from_ptr(g.adj, m, torch.int32, self.device),
                         _copy_from_ptr(g.ew, m, torch.int32, self.device),
                         _copy_from_ptr(g.vw, n, torch.int32, self.device))
        cmap = _copy_from_ptr(cm.value, n, torch.int32, self.device) if cm.value else None
        return LevelView(dg, cmap, int(inf.rounds), int(inf.matched), int(inf.stop_reason))


def kappa_coarsen(g: DeviceGraph, rating: int = EXPANSION_STAR2, seed: int = 42, stop_n: int = 256,
                  stall_num: int = 1, stall_den: int = 20, max_levels: int = 64,
                  trusted: bool = False, block_bits: Optional[int] = None) -> Hierarchy:
    """trusted: g passed kappa_validate and is unchanged since (the full
    structural check is skipped).  block_bits: match every level with the
    two-phase matcher, blocks of 2^block_bits consecutive ids."""
    flags = (COARSEN_TRUSTED if trusted else 0) | (COARSEN_TWO_PHASE if block_bits is not None else 0)
    p = c_params(rating, seed & (2**64 - 1), stop_n, stall_num, stall_den, max_levels, flags,
                 block_bits if block_bits is not None else 0)
    h = ctypes.c_void_p()
    _check("kappa_coarsen", lib().kappa_coarsen(ctypes.byref(g.c()), ctypes.byref(p), ctypes.byref(h),
                                                _stream()))
    return Hierarchy(h, g.xadj.device, g)


def union_csr(graphs):
    """Block-diagonal union of host CSR graphs (objects with n, xadj, adj, ew,
    vw numpy arrays), the input layout of the batched form: graph g's nodes
    follow those of graphs 0 .. g-1.  Returns (n, xadj, adj, ew, vw,
    node_off) as numpy arrays (node_off int32, count + 1)."""
    import numpy as np
    ns = np.array([int(g.n) for g in graphs], dtype=np.int64)
    es = np.array([int(g.xadj[-1]) if len(g.xadj) else 0 for g in graphs], dtype=np.int64)
    node_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    node_off[1:] = np.cumsum(ns)
    ent_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    ent_off[1:] = np.cumsum(es)
    n = int(node_off[-1])
    xadj = np.empty(n + 1, dtype=np.int64)
    adj = np.empty(int(ent_off[-1]), dtype=np.int32)
    ew = np.empty(int(ent_off[-1]), dtype=np.uint32)
    vw = np.empty(n, dtype=np.uint32)
    for i, g in enumerate(graphs):
        a, b = int(node_off[i]), int(node_off[i + 1])
        ea, eb = int(ent_off[i]), int(ent_off[i + 1])
        xadj[a:b] = np.asarray(g.xadj[:-1], dtype=np.int64) + ea
        adj[ea:eb] = np.asarray(g.adj, dtype=np.int64) + a
        ew[ea:eb] = g.ew
        vw[a:b] = g.vw
    xadj[n] = int(ent_off[-1])
    return n, xadj, adj, ew, vw, node_off.astype(np.int32)


class Batch:
    """Owns a kappa_batch handle (freed with the object); keeps the union
    graph alive (level 0 of the batch refers to its arrays)."""

    def __init__(self, handle, device, graph, count):
        self.handle = handle
        self.device = device
        self.graph = graph
        self.count = count

    def __del__(self):
        try:
            if self.handle:
                lib().kappa_batch_free(self.handle)
                self.handle = None
        except Exception:
            pass

    def __len__(self):
        return self.count

    def info(self, g: int):
        """(levels, stop reason) of graph g."""
        lv, st = ctypes.c_int32(), ctypes.c_int32()
        _check("kappa_batch_graph_info", lib().kappa_batch_graph_info(self.handle, g, ctypes.byref(lv),
                                                                      ctypes.byref(st)))
        return int(lv.value), int(st.value)

    def hierarchy(self, g: int) -> Hierarchy:
        """Graph g's hierarchy (local ids) as a standalone Hierarchy."""
        h = ctypes.c_void_p()
        _check("kappa_batch_hierarchy", lib().kappa_batch_hierarchy(self.handle, g, ctypes.byref(h),
                                                                    _stream()))
        return Hierarchy(h, self.device)   # a copy: independent of the batch


def kappa_coarsen_batch(u: DeviceGraph, node_off, rating: int = EXPANSION_STAR2, seed: int = 42,
                        stop_n=256, stall_num: int = 1, stall_den: int = 20,
                        max_levels: int = 64) -> Batch:
    """Coarsens the graphs of the block-diagonal union `u` (graph g owns nodes
    node_off[g] .. node_off[g+1]-1) together.  stop_n: one int for all graphs
    or a sequence with one per graph."""
    import numpy as np
    off = np.ascontiguousarray(np.asarray(node_off, dtype=np.int32))
    count = len(off) - 1
    sn = None
    if not np.isscalar(stop_n):
        sn = np.ascontiguousarray(np.asarray(stop_n, dtype=np.int32))
        stop_n = 0
    p = c_params(rating, seed & (2**64 - 1), int(stop_n), stall_num, stall_den, max_levels, 0)
    h = ctypes.c_void_p()
    _check("kappa_coarsen_batch", lib().kappa_coarsen_batch(
        ctypes.byref(u.c()), count, off.ctypes.data_as(ctypes.c_void_p),
        sn.ctypes.data_as(ctypes.c_void_p) if sn is not None else None, ctypes.byref(p),
        ctypes.byref(h), _stream()))
    return Batch(h, u.xadj.device, u, count)


def kappa_coarsen_graphs(graphs, rating: int = EXPANSION_STAR2, seed: int = 42, stop_n=256,
                         stall_num: int = 1, stall_den: int = 20, max_levels: int = 64,
                         trusted: bool = False) -> Batch:
    """The batched form over separate device graphs (a list of DeviceGraph):
    the library builds their union on the device.  stop_n: one int for all
    graphs or a sequence with one per graph."""
    import numpy as np
    count = len(graphs)
    descs = (c_graph * count)(*[g.c() for g in graphs])
    sn = None
    if not np.isscalar(stop_n):
        sn = np.ascontiguousarray(np.asarray(stop_n, dtype=np.int32))
        stop_n = 0
    p = c_params(rating, seed & (2**64 - 1), int(stop_n), stall_num, stall_den, max_levels,
                 COARSEN_TRUSTED if trusted else 0)
    h = ctypes.c_void_p()
    _check("kappa_coarsen_graphs", lib().kappa_coarsen_graphs(
        ctypes.cast(descs, ctypes.c_void_p), count,
        sn.ctypes.data_as(ctypes.c_void_p) if sn is not None else None, ctypes.byref(p),
        ctypes.byref(h), _stream()))
    return Batch(h, graphs[0].xadj.device, None, count)


class Server:
    """Level-granular continuous batching (kappa_server_*): the requests of
    one rating on one stream (the current stream when created).  admit()
    takes a device graph (copied by the library) and returns an id; step()
    advances every active request in one batched pass, up to the first level
    boundary at which a request finishes or an interrupt() was raised, and
    returns the ids that finished; take(id) gives a finished request's
    Hierarchy.  One thread drives a server; interrupt() may come from any."""

    def __init__(self, rating: int = EXPANSION_STAR2, seed: int = 42, stall_num: int = 1,
                 stall_den: int = 20, max_levels: int = 64, trusted: bool = False, device="cuda"):
        self.device = device
        p = c_params(rating, seed & (2**64 - 1), 0, stall_num, stall_den, max_levels,
                     COARSEN_TRUSTED if trusted else 0)
        h = ctypes.c_void_p()
        self.stream = _stream()
        _check("kappa_server_create", lib().kappa_server_create(ctypes.byref(p), ctypes.byref(h),
                                                                self.stream))
        self.handle = h
        self._fin = (ctypes.c_int64 * 4096)()

    def __del__(self):
        try:
            if self.handle:
                lib().kappa_server_free(self.handle)
                self.handle = None
        except Exception:
            pass

    def admit(self, g: "DeviceGraph", stop_n: int) -> int:
        rid = ctypes.c_int64()
        _check("kappa_server_admit", lib().kappa_server_admit(self.handle, ctypes.byref(g.c()),
                                                              int(stop_n), ctypes.byref(rid)))
        return int(rid.value)

    def active(self) -> int:
        return int(lib().kappa_server_active(self.handle))

    def interrupt(self, on: bool = True):
        """Ask the running (or next) step to end at its next level boundary;
        on=False clears the request.  Safe from any thread."""
        _check("kappa_server_interrupt", lib().kappa_server_interrupt(self.handle, 1 if on else 0))

    def step(self):
        nf = ctypes.c_int32()
        cap = max(1, self.active())   # no step finishes more requests than are active
        if len(self._fin) < cap:
            self._fin = (ctypes.c_int64 * cap)()
        _check("kappa_server_step", lib().kappa_server_step(
            self.handle, ctypes.cast(self._fin, ctypes.c_void_p), cap, ctypes.byref(nf)))
        return [int(self._fin[i]) for i in range(nf.value)]

    def take(self, rid: int) -> Hierarchy:
        h = ctypes.c_void_p()
        _check("kappa_server_take", lib().kappa_server_take(self.handle, ctypes.c_int64(rid),
                                                            ctypes.byref(h)))
        return Hierarchy(h, self.device)


def kappa_initial_partition(n: int, k: int, seed: int, device="cuda"):
    import torch
    part = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    _check("kappa_initial_partition", lib().kappa_initial_partition(n, k, ctypes.c_uint64(seed),
                                                                    _ptr(part), _stream()))
    return part[:n]


def kappa_project(cmap, n_coarse: int, part_coarse):
    import torch
    n = int(cmap.numel())
    out = torch.empty(max(n, 1), dtype=torch.int32, device=cmap.device)
    _check("kappa_project", lib().kappa_project(_ptr(cmap), n, n_coarse, _ptr(part_coarse),
                                                _ptr(out), _stream()))
    return out[:n]


def kappa_cut_balance(g: DeviceGraph, part, k: int, eps_num: int = 3, eps_den: int = 100):
    """Returns (c_cut result, block weights as an int64 tensor)."""
    import torch
    bw = torch.empty(max(k, 1), dtype=torch.int64, device=g.xadj.device)
    res = c_cut()
    _check("kappa_cut_balance", lib().kappa_cut_balance(ctypes.byref(g.c()), _ptr(part), k, eps_num,
                                                        eps_den, _ptr(bw), ctypes.byref(res),
                                                        _stream()))
    return res, bw[:k]


def kappa_cut_balance_noalloc(g: DeviceGraph, part, k: int, eps_num: int = 3, eps_den: int = 100,
                              block_w=None):
    """kappa_cut_balance through the allocation-free entry point: block_w
    (device int64 [k], may be None) is the caller's; returns the c_cut result."""
    res = c_cut()
    _check("kappa_cut_balance_noalloc",
           lib().kappa_cut_balance_noalloc(ctypes.byref(g.c()), _ptr(part), k, eps_num, eps_den,
                                           _ptr(block_w) if block_w is not None else None,
                                           ctypes.byref(res), _stream()))
    return res


def kappa_uncoarsen(h: Hierarchy, k: int, part_seed: int = 1, eps_num: int = 3, eps_den: int = 100,
                    part0=None):
    """Returns (level-0 partition tensor, [c_cut per level])."""
    import torch
    n0 = int(h.info(0).n)
    if part0 is None:
        part0 = torch.empty(max(n0, 1), dtype=torch.int32, device=h.device)
    L = len(h)
    res = (c_cut * L)()
    _check("kappa_uncoarsen", lib().kappa_uncoarsen(h.handle, k, ctypes.c_uint64(part_seed), eps_num,
                                                    eps_den, _ptr(part0), res, _stream()))
    return part0[:n0], list(res)


def kappa_refine(g: DeviceGraph, part, k: int, eps_num: int = 3, eps_den: int = 100,
                 preset: str = "fast", seed: int = 1, **over):
    """Pairwise refinement (Section 5) of the device partition `part`, in
    place.  Returns the stats as a dict."""
    p = refine_params(preset, seed, **over)
    out = c_refine_stats()
    _check("kappa_refine", lib().kappa_refine(ctypes.byref(g.c()), _ptr(part), k, eps_num, eps_den,
                                              ctypes.byref(p), ctypes.byref(out), _stream()))
    return out.as_dict()


def kappa_uncoarsen_refined(h: Hierarchy, k: int, part_seed: int = 1, eps_num: int = 3,
                            eps_den: int = 100, preset: str = "fast", seed: int = 1, part0=None,
                            **over):
    """The way back up with refinement.  Returns (level-0 partition tensor,
    [c_cut per level], [stats dict per level])."""
    import torch
    n0 = int(h.info(0).n)
    if part0 is None:
        part0 = torch.empty(max(n0, 1), dtype=torch.int32, device=h.device)
    L = len(h)
    res = (c_cut * L)()
    sts = (c_refine_stats * L)()
    p = refine_params(preset, seed, **over)
    _check("kappa_uncoarsen_refined",
           lib().kappa_uncoarsen_refined(h.handle, k, ctypes.c_uint64(part_seed), eps_num, eps_den,
                                         ctypes.byref(p), _ptr(part0), res, sts, _stream()))
    return part0[:n0], list(res), [x.as_dict() for x in sts]


def kappa_cache_release():
    """Frees the device memory the library keeps between calls."""
    _check("kappa_cache_release", lib().kappa_cache_release())


def tuning_get() -> dict:
    """The library's tuning table (kappa_tuning) as a dict."""
    t = c_tuning()
    _check("kappa_tuning_get", lib().kappa_tuning_get(ctypes.byref(t)))
    return {f: int(getattr(t, f)) for f in TUNING_FIELDS}


def tuning_set(table: Optional[dict] = None, **fields):
    """Sets the fields given (the others keep their values); raises
    KappaError (E_RANGE) on a value out of range."""
    cur = tuning_get()
    cur.update(table or {})
    cur.update(fields)
    unknown = set(cur) - set(TUNING_FIELDS)
    if unknown:
        raise KeyError(f"unknown tuning fields {sorted(unknown)}")
    t = c_tuning(*[int(cur[f]) for f in TUNING_FIELDS])
    _check("kappa_tuning_set", lib().kappa_tuning_set(ctypes.byref(t)))


def tuning_load(path: str):
    _check("kappa_tuning_load", lib().kappa_tuning_load(str(path).encode()))


def graphs_enable(on: bool = True):
    """Replay repeated launch sequences as HIP graphs (on) or launch every
    kernel directly (off, the library's default)."""
    lib().kappa_graphs_enable(1 if on else 0)


def use_torch_allocator(on: bool = True):
    """Let the library take its device memory (workspaces, hierarchy arenas,
    batch unions) from torch's caching allocator, on the stream of each call,
    so that it shows in torch's memory statistics and shares its pool; off:
    the device's stream-ordered pool (the library's default).  Switching
    releases the library's memory cache: no call may be running."""
    global _allocator
    import torch
    if on:
        def _alloc(nbytes, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                          int(stream or 0))
            except Exception:   # out of memory: the library reports KAPPA_E_NOMEM
                return None

        def _free(ptr, nbytes, stream, ctx):
            torch.cuda.caching_allocator_delete(int(ptr))

        cbs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
        _check("kappa_set_allocator", lib().kappa_set_allocator(cbs[0], cbs[1], None))
        _allocator = cbs
    else:
        _check("kappa_set_allocator", lib().kappa_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
        _allocator = None


def persistent_enable(on: bool = True):
    """Run a level's matching rounds after the first in one cooperative
    launch (on) or one launch per phase and round (off, the default)."""
    lib().kappa_persistent_enable(1 if on else 0)


def tail_enable(on: bool = True):
    """Run small levels (and every later one) in one workgroup (on) or every
    level with the grid kernels (off, the library's default)."""
    lib().kappa_tail_enable(1 if on else 0)


def arena_first(nbytes: int = 0):
    """First-attempt arena size of kappa_coarsen / kappa_coarsen_batch (0:
    the default sizing); a tight value sends calls through the retry path."""
    lib().kappa_arena_first(int(nbytes))


def profile_enable(on: bool = True):
    lib().kappa_profile_enable(1 if on else 0)


def profile_reset():
    lib().kappa_profile_reset()


def profile_read():
    """{kernel name: (launches, milliseconds)} since the last reset."""
    cap = 128
    names = (ctypes.c_char_p * cap)()
    launches = (ctypes.c_int64 * cap)()
    ms = (ctypes.c_double * cap)()
    n = lib().kappa_profile_read(names, launches, ms, cap)
    return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(min(n, cap))}
