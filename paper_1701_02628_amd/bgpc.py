"""Thin ctypes binding of libbgpc.so (argument marshalling only).

Every coloring step runs in the HIP library; this module only turns torch
device tensors into the pointers and structs of ``include/bgpc.h``.  It
raises if the library is missing or a tensor is not an int32 tensor on the
GPU: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbgpc.so")

OK = 0
E_INVALID, E_UNSORTED, E_NOT_TRANSPOSE, E_NOT_SYMMETRIC = -1, -2, -3, -4
E_OOM, E_NOT_CONVERGED, E_HIP, E_UNSUPPORTED, E_INTERNAL = -5, -6, -7, -8, -9
FIRST_FIT, B1, B2, B1_GLOBAL = 0, 1, 2, 3
STRICT, RESUME, NET_BALANCE = 1, 2, 8
NET_ALG8, NET_ALG6, NET_ALG6_REVERSE = 0, 1, 2
ROUTE_NET_MASKS, ROUTE_BITMAPS, ROUTE_DENSE, ROUTE_WHOLE_DEVICE = 0, 1, 2, 3
ALL_NET = 2 ** 64 - 1


class Csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("indices", ctypes.c_void_p)]


class RoundLog(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int32), ("n", ctypes.c_int32), ("mode", ctypes.c_void_p),
                ("w_size", ctypes.c_void_p), ("losers", ctypes.c_void_p), ("evicted", ctypes.c_void_p),
                ("max_color", ctypes.c_void_p), ("hash_t", ctypes.c_void_p), ("hash_c", ctypes.c_void_p),
                ("round_ms", ctypes.c_void_p)]


class Profile(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("launches", ctypes.c_int32), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("bytes_scanned", ctypes.c_double), ("bytes_states", ctypes.c_double)]


PROF_CONFLICT, PROF_COLOR = 0, 1
INCREMENTAL = 4


class Opts(ctypes.Structure):
    _fields_ = [("net_color_mask", ctypes.c_uint64), ("policy", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("start_round", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_int32), ("stream", ctypes.c_void_p), ("log", ctypes.POINTER(RoundLog)),
                ("rounds_out", ctypes.POINTER(ctypes.c_int32)), ("prof", ctypes.POINTER(Profile)),
                ("net_conflict_mask", ctypes.c_uint64), ("net_alg", ctypes.c_int32), ("reserved2", ctypes.c_int32),
                ("tuning", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("front", ctypes.c_int32), ("standing", ctypes.c_int32), ("planes", ctypes.c_int32),
                ("color_grid", ctypes.c_int32), ("removal_grid", ctypes.c_int32), ("apply_grid", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def tuning(front=-1, standing=-1, planes=-1, color_grid=0, removal_grid=0, apply_grid=0):
    return Tuning(front, standing, planes, color_grid, removal_grid, apply_grid)


class BatchItem(ctypes.Structure):
    _fields_ = [("csr_A", Csr), ("csr_B", Csr), ("colors_out", ctypes.c_void_p), ("status", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("order", ctypes.c_void_p), ("d2gc", ctypes.c_int32),
                ("route", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("n_a", ctypes.c_int32), ("n_b", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("a_off", ctypes.c_void_p), ("a_idx", ctypes.c_void_p), ("b_off", ctypes.c_void_p),
                ("b_idx", ctypes.c_void_p), ("colors_out", ctypes.c_void_p), ("tag", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


REQ_PINNED = 1


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n_distinct", ctypes.c_int64), ("max_color", ctypes.c_int64), ("card_min", ctypes.c_int64),
                ("card_max", ctypes.c_int64), ("n_empty_below_max", ctypes.c_int64),
                ("card_mean", ctypes.c_double), ("card_std", ctypes.c_double)]


_lib = None


def load():
    """Load libbgpc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1701_02628_amd/build.py "
                               "(the coloring path has no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.bgpc_opts_default.argtypes = [ctypes.POINTER(Opts)]
        lib.bgpc_opts_default.restype = None
        lib.bgpc_color.argtypes = [ctypes.POINTER(Csr), ctypes.POINTER(Csr), P, ctypes.POINTER(Opts), P]
        lib.bgpc_color.restype = ctypes.c_int
        lib.d2gc_color.argtypes = [ctypes.POINTER(Csr), P, ctypes.POINTER(Opts), P]
        lib.d2gc_color.restype = ctypes.c_int
        lib.color_stats.argtypes = [P, ctypes.c_int64, P, ctypes.POINTER(Stats)]
        lib.color_stats.restype = ctypes.c_int
        lib.bgpc_color_batch.argtypes = [ctypes.POINTER(BatchItem), ctypes.c_int32, ctypes.POINTER(Opts)]
        lib.bgpc_color_batch.restype = ctypes.c_int
        lib.bgpc_session_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.bgpc_session_create.restype = ctypes.c_void_p
        lib.bgpc_session_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(Request)]
        lib.bgpc_session_submit.restype = ctypes.c_int
        lib.bgpc_session_poll.argtypes = [ctypes.c_void_p, ctypes.POINTER(Completion), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
        lib.bgpc_session_poll.restype = ctypes.c_int
        lib.bgpc_session_destroy.argtypes = [ctypes.c_void_p]
        lib.bgpc_session_destroy.restype = None
        lib.bgpc_order_largest_first.argtypes = [ctypes.POINTER(Csr), ctypes.POINTER(Csr), P, P]
        lib.bgpc_order_largest_first.restype = ctypes.c_int
        lib.d2gc_order_largest_first.argtypes = [ctypes.POINTER(Csr), P, P]
        lib.d2gc_order_largest_first.restype = ctypes.c_int
        lib.bgpc_autotune.argtypes = [ctypes.POINTER(Csr), ctypes.POINTER(Csr), ctypes.POINTER(Opts), ctypes.c_int32,
                                      ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
        lib.bgpc_autotune.restype = ctypes.c_int
        lib.bgpc_order_smallest_last.argtypes = [ctypes.POINTER(Csr), ctypes.POINTER(Csr), ctypes.c_int32, P, P,
                                                 ctypes.POINTER(ctypes.c_int32)]
        lib.bgpc_order_smallest_last.restype = ctypes.c_int
        lib.d2gc_order_smallest_last.argtypes = [ctypes.POINTER(Csr), ctypes.c_int32, P, P,
                                                 ctypes.POINTER(ctypes.c_int32)]
        lib.d2gc_order_smallest_last.restype = ctypes.c_int
        lib.bgpc_color_noalloc.argtypes = [ctypes.POINTER(Csr), ctypes.POINTER(Csr), ctypes.POINTER(Opts), P]
        lib.bgpc_color_noalloc.restype = ctypes.c_int
        lib.bgpc_status_string.argtypes = [ctypes.c_int]
        lib.bgpc_status_string.restype = ctypes.c_char_p
        _lib = lib
    return _lib


EXPORTED = ("bgpc_opts_default", "bgpc_color", "d2gc_color", "color_stats", "bgpc_status_string",
            "bgpc_color_batch", "bgpc_session_create", "bgpc_session_submit", "bgpc_session_poll",
            "bgpc_session_destroy", "bgpc_order_largest_first", "d2gc_order_largest_first",
            "bgpc_order_smallest_last", "d2gc_order_smallest_last", "bgpc_autotune", "bgpc_color_noalloc")


def status_string(code: int) -> str:
    return load().bgpc_status_string(int(code)).decode()


def _dev_ptr(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int32 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class DeviceCsr:
    """int32 CSR resident on the GPU (offsets, indices) with its shape."""

    def __init__(self, offsets, indices, n_rows, n_cols):
        self.offsets, self.indices = offsets, indices
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)

    @property
    def nnz(self):
        return int(self.indices.numel())

    def as_struct(self) -> Csr:
        idx_ptr = self.indices.data_ptr() if self.indices.numel() else None
        return Csr(self.n_rows, self.n_cols, self.nnz, _dev_ptr(self.offsets, "offsets").value, idx_ptr)


def upload_csr(off, idx, n_rows, n_cols, device="cuda") -> DeviceCsr:
    import torch
    off = np.ascontiguousarray(off, dtype=np.int64)
    if off[-1] >= 2 ** 31:
        raise ValueError("more than 2^31 - 1 entries")
    o = torch.from_numpy(off.astype(np.int32)).to(device)
    i = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).to(device)
    return DeviceCsr(o, i, n_rows, n_cols)


def upload_bipartite(g, device="cuda"):
    """(csr_A, csr_B) on the GPU for a host graph with n_a, n_b, a_*, b_*."""
    A = upload_csr(g.a_off, g.a_idx, g.n_a, g.n_b, device)
    B = upload_csr(g.b_off, g.b_idx, g.n_b, g.n_a, device)
    return A, B


def upload_adjacency(adj, device="cuda") -> DeviceCsr:
    return upload_csr(adj.off, adj.idx, adj.n, adj.n, device)


class Result:
    def __init__(self, status, rounds, log):
        self.status, self.rounds, self.log = status, rounds, log

    def __repr__(self):
        return f"Result(status={self.status}, rounds={self.rounds})"


def _make_opts(net_color_mask, policy, chunk, max_rounds, start_round, flags, stream, log_cap, prof=None,
               net_conflict_mask=ALL_NET, net_alg=NET_ALG8, log_hashes=False, tune=None):
    lib = load()
    o = Opts()
    lib.bgpc_opts_default(ctypes.byref(o))
    o.net_color_mask = int(net_color_mask) & (2 ** 64 - 1)
    o.net_conflict_mask = int(net_conflict_mask) & (2 ** 64 - 1)
    o.net_alg = int(net_alg)
    o.policy, o.chunk, o.max_rounds = int(policy), int(chunk), int(max_rounds)
    o.start_round, o.flags = int(start_round), int(flags)
    o.stream = _stream_handle(stream)
    rounds = ctypes.c_int32(0)
    o.rounds_out = ctypes.pointer(rounds)
    keep = [rounds]
    if tune is not None:
        o.tuning = ctypes.cast(ctypes.pointer(tune), ctypes.c_void_p)
        keep.append(tune)
    log_arrays = None
    if log_cap:
        log_arrays = {"mode": np.zeros(log_cap, np.int32), "w": np.zeros(log_cap, np.int64),
                      "losers": np.zeros(log_cap, np.int64), "evicted": np.zeros(log_cap, np.int64),
                      "max_color": np.zeros(log_cap, np.int32), "round_ms": np.zeros(log_cap, np.float32)}
        if log_hashes:
            log_arrays["hash_t"] = np.zeros(log_cap, np.uint64)
            log_arrays["hash_c"] = np.zeros(log_cap, np.uint64)
        hp = (lambda k: log_arrays[k].ctypes.data if k in log_arrays else None)
        lg = RoundLog(log_cap, 0, log_arrays["mode"].ctypes.data, log_arrays["w"].ctypes.data,
                      log_arrays["losers"].ctypes.data, log_arrays["evicted"].ctypes.data,
                      log_arrays["max_color"].ctypes.data, hp("hash_t"), hp("hash_c"),
                      log_arrays["round_ms"].ctypes.data)
        o.log = ctypes.pointer(lg)
        keep.append(lg)
    if prof is not None:
        o.prof = ctypes.pointer(prof)
        keep.append(prof)
    return o, rounds, log_arrays, keep


def _finish(status, rounds, log_arrays, o):
    log = None
    if log_arrays is not None:
        n = o.log.contents.n
        log = {k: v[:n].copy() for k, v in log_arrays.items()}
    return Result(int(status), int(rounds.value), log)


def bgpc_color(csr_A: DeviceCsr, csr_B: DeviceCsr, order, colors_out, net_color_mask=0, policy=FIRST_FIT,
               chunk=64, max_rounds=0, start_round=0, flags=0, stream=None, log_cap=0, prof=None,
               net_conflict_mask=ALL_NET, net_alg=NET_ALG8, log_hashes=False, tune=None) -> Result:
    """Bipartite-graph partial coloring; colors_out is an int32 GPU tensor of |V_A|.
    prof: optional Profile struct (kernel timing), filled in place; tune:
    optional Tuning (result-invariant launch choices)."""
    lib = load()
    o, rounds, log_arrays, keep = _make_opts(net_color_mask, policy, chunk, max_rounds, start_round, flags,
                                             stream, log_cap, prof, net_conflict_mask, net_alg, log_hashes, tune)
    a, b = csr_A.as_struct(), csr_B.as_struct()
    order_p = _dev_ptr(order, "order") if order is not None else None
    st = lib.bgpc_color(ctypes.byref(a), ctypes.byref(b), order_p, ctypes.byref(o), _dev_ptr(colors_out, "colors_out"))
    del keep
    return _finish(st, rounds, log_arrays, o)


def bgpc_color_noalloc(csr_A: DeviceCsr, csr_B: DeviceCsr, colors_out, net_color_mask=0, policy=FIRST_FIT,
                       chunk=64, max_rounds=0, start_round=0, flags=0, stream=None, log_cap=0,
                       net_conflict_mask=ALL_NET, net_alg=NET_ALG8) -> Result:
    """bgpc_color without any allocation (natural order; workspace in the
    library's static device array)."""
    lib = load()
    o, rounds, log_arrays, keep = _make_opts(net_color_mask, policy, chunk, max_rounds, start_round, flags,
                                             stream, log_cap, None, net_conflict_mask, net_alg)
    if o.log:
        o.log.contents.round_ms = None   # per-round events are not created without allocation
    a, b = csr_A.as_struct(), csr_B.as_struct()
    st = lib.bgpc_color_noalloc(ctypes.byref(a), ctypes.byref(b), ctypes.byref(o), _dev_ptr(colors_out, "colors_out"))
    del keep
    res = _finish(st, rounds, log_arrays, o)
    if res.log is not None:
        res.log.pop("round_ms", None)
    return res


def d2gc_color(adj: DeviceCsr, order, colors_out, net_color_mask=0, policy=FIRST_FIT, chunk=64, max_rounds=0,
               start_round=0, flags=0, stream=None, log_cap=0, prof=None, net_conflict_mask=ALL_NET,
               net_alg=NET_ALG8, log_hashes=False, tune=None) -> Result:
    """Distance-2 coloring of a symmetric graph; colors_out is an int32 GPU tensor of n."""
    lib = load()
    o, rounds, log_arrays, keep = _make_opts(net_color_mask, policy, chunk, max_rounds, start_round, flags,
                                             stream, log_cap, prof, net_conflict_mask, net_alg, log_hashes, tune)
    a = adj.as_struct()
    order_p = _dev_ptr(order, "order") if order is not None else None
    st = lib.d2gc_color(ctypes.byref(a), order_p, ctypes.byref(o), _dev_ptr(colors_out, "colors_out"))
    del keep
    return _finish(st, rounds, log_arrays, o)


def order_largest_first(csr_A: DeviceCsr, csr_B: DeviceCsr, stream=None):
    """Largest-first order of V_A as an int32 GPU tensor (order[k] = vertex of rank k)."""
    import torch
    lib = load()
    out = torch.empty(max(csr_A.n_rows, 1), dtype=torch.int32, device=csr_A.offsets.device)[:csr_A.n_rows]
    a, b = csr_A.as_struct(), csr_B.as_struct()
    st = lib.bgpc_order_largest_first(ctypes.byref(a), ctypes.byref(b), _stream_handle(stream),
                                      _dev_ptr(out, "order_out") if csr_A.n_rows else None)
    if st != OK:
        raise RuntimeError(f"bgpc_order_largest_first failed: {status_string(st)}")
    return out


def d2gc_order_largest_first(adj: DeviceCsr, stream=None):
    """Largest-first order of a symmetric graph's vertices (closed neighbourhoods as nets)."""
    import torch
    lib = load()
    out = torch.empty(max(adj.n_rows, 1), dtype=torch.int32, device=adj.offsets.device)[:adj.n_rows]
    a = adj.as_struct()
    st = lib.d2gc_order_largest_first(ctypes.byref(a), _stream_handle(stream),
                                      _dev_ptr(out, "order_out") if adj.n_rows else None)
    if st != OK:
        raise RuntimeError(f"d2gc_order_largest_first failed: {status_string(st)}")
    return out


def autotune(csr_A: DeviceCsr, csr_B=None, trials=3, stream=None, **kw):
    """Tune the result-invariant choices for this graph (csr_B None: distance-2
    on the adjacency csr_A) under the given schedule (net_color_mask, policy,
    chunk, flags as for bgpc_color); returns (Tuning, default ms, tuned ms).
    The choice is cached in the library for graphs of the same shape."""
    lib = load()
    o, rounds, _, keep = _make_opts(kw.get("net_color_mask", 0), kw.get("policy", FIRST_FIT), kw.get("chunk", 64),
                                    0, 0, kw.get("flags", 0), stream, 0)
    best = Tuning()
    md, mb = ctypes.c_double(0), ctypes.c_double(0)
    a = csr_A.as_struct()
    b = csr_B.as_struct() if csr_B is not None else None
    st = lib.bgpc_autotune(ctypes.byref(a), ctypes.byref(b) if b is not None else None, ctypes.byref(o), int(trials),
                           ctypes.byref(best), ctypes.byref(md), ctypes.byref(mb))
    del keep
    if st != OK:
        raise RuntimeError(f"bgpc_autotune failed: {status_string(st)}")
    return best, md.value, mb.value


def order_smallest_last(csr_A: DeviceCsr, csr_B: DeviceCsr, slack_shift=3, stream=None, with_steps=False):
    """Smallest-last order of V_A by removal steps (int32 GPU tensor, order[k] = vertex of rank k)."""
    import torch
    lib = load()
    out = torch.empty(max(csr_A.n_rows, 1), dtype=torch.int32, device=csr_A.offsets.device)[:csr_A.n_rows]
    steps = ctypes.c_int32(0)
    a, b = csr_A.as_struct(), csr_B.as_struct()
    st = lib.bgpc_order_smallest_last(ctypes.byref(a), ctypes.byref(b), int(slack_shift), _stream_handle(stream),
                                      _dev_ptr(out, "order_out") if csr_A.n_rows else None, ctypes.byref(steps))
    if st != OK:
        raise RuntimeError(f"bgpc_order_smallest_last failed: {status_string(st)}")
    return (out, steps.value) if with_steps else out


def d2gc_order_smallest_last(adj: DeviceCsr, slack_shift=3, stream=None, with_steps=False):
    """Smallest-last order of a symmetric graph's vertices (closed neighbourhoods as nets)."""
    import torch
    lib = load()
    out = torch.empty(max(adj.n_rows, 1), dtype=torch.int32, device=adj.offsets.device)[:adj.n_rows]
    steps = ctypes.c_int32(0)
    a = adj.as_struct()
    st = lib.d2gc_order_smallest_last(ctypes.byref(a), int(slack_shift), _stream_handle(stream),
                                      _dev_ptr(out, "order_out") if adj.n_rows else None, ctypes.byref(steps))
    if st != OK:
        raise RuntimeError(f"d2gc_order_smallest_last failed: {status_string(st)}")
    return (out, steps.value) if with_steps else out


def color_stats(colors, stream=None) -> dict:
    """Color-set statistics of an int32 GPU tensor of colors."""
    lib = load()
    out = Stats()
    st = lib.color_stats(_dev_ptr(colors, "colors"), int(colors.numel()), _stream_handle(stream), ctypes.byref(out))
    if st != OK:
        raise RuntimeError(f"color_stats failed: {status_string(st)}")
    return {"n_distinct": out.n_distinct, "max_color": out.max_color, "card_min": out.card_min,
            "card_max": out.card_max, "n_empty_below_max": out.n_empty_below_max,
            "card_mean": out.card_mean, "card_std": out.card_std}


def bgpc_color_batch(graphs, colors, max_rounds=0, stream=None, orders=None, with_routes=False, **opts):
    """Color many graphs in one call.

    graphs: list of (csr_A, csr_B) DeviceCsr pairs, or a DeviceCsr adjacency
    for a distance-2 item; colors: list of int32 GPU tensors; orders: None or
    a list of None / int32 GPU permutations; opts: net_color_mask, policy,
    chunk, flags, net_conflict_mask, net_alg as for bgpc_color.  Returns
    (status, per-item statuses, per-item rounds[, per-item routes]).
    """
    lib = load()
    n = len(graphs)
    items = (BatchItem * max(n, 1))()
    for i, (gr, c) in enumerate(zip(graphs, colors)):
        if isinstance(gr, DeviceCsr):
            items[i].csr_A = gr.as_struct()
            items[i].d2gc = 1
        else:
            items[i].csr_A = gr[0].as_struct()
            items[i].csr_B = gr[1].as_struct()
        items[i].colors_out = _dev_ptr(c, "colors").value
        if orders is not None and orders[i] is not None:
            items[i].order = _dev_ptr(orders[i], "order").value
    o, rounds, _, keep = _make_opts(opts.get("net_color_mask", 0), opts.get("policy", FIRST_FIT),
                                    opts.get("chunk", 64), max_rounds, 0, opts.get("flags", 0), stream, 0,
                                    None, opts.get("net_conflict_mask", ALL_NET), opts.get("net_alg", NET_ALG8))
    st = lib.bgpc_color_batch(items, n, ctypes.byref(o))
    del keep
    out = (int(st), [items[i].status for i in range(n)], [items[i].rounds for i in range(n)])
    return out + ([items[i].route for i in range(n)],) if with_routes else out


class Session:
    """Serving session (continuous batching) over host-resident requests.

    submit() takes numpy int32 arrays; they and the colors array returned are
    kept alive here until the request's completion has been polled.
    """

    def __init__(self, mem_budget: int, max_slots: int = 512, max_group: int = 256, max_rounds: int = 0):
        self._lib = load()
        self._h = self._lib.bgpc_session_create(int(mem_budget), int(max_slots), int(max_group), int(max_rounds))
        if not self._h:
            raise RuntimeError("bgpc_session_create failed")
        self._live = {}

    def submit(self, tag: int, n_a: int, n_b: int, a_off, a_idx, b_off, b_idx, colors=None):
        """numpy arrays (staged by the session), or pinned int32 CPU torch
        tensors with a pinned `colors` tensor (uploaded directly)."""
        import torch
        if isinstance(a_off, torch.Tensor):
            arrs = [a_off, a_idx, b_off, b_idx]
            for t in arrs + [colors]:
                if t.dtype != torch.int32 or t.is_cuda or not t.is_pinned() or not t.is_contiguous():
                    raise TypeError("pinned requests need contiguous pinned int32 CPU tensors")
            ptrs = [t.data_ptr() for t in arrs]
            nnz, cptr, flags = int(a_idx.numel()), colors.data_ptr(), REQ_PINNED
        else:
            arrs = [np.ascontiguousarray(x, dtype=np.int32) for x in (a_off, a_idx, b_off, b_idx)]
            colors = np.empty(max(n_a, 1), dtype=np.int32)
            ptrs = [x.ctypes.data for x in arrs]
            nnz, cptr, flags = int(arrs[1].shape[0]), colors.ctypes.data, 0
        r = Request(int(n_a), int(n_b), nnz, ptrs[0], ptrs[1], ptrs[2], ptrs[3], cptr, int(tag), flags, 0)
        self._live[int(tag)] = (arrs, colors)
        st = self._lib.bgpc_session_submit(self._h, ctypes.byref(r))
        if st != OK:
            del self._live[int(tag)]
        return st

    def poll(self, cap: int = 256, wait_ms: int = 0):
        """List of (tag, status, rounds, t_submit, t_admit, t_done, colors)."""
        buf = (Completion * cap)()
        n = ctypes.c_int32(0)
        err = self._lib.bgpc_session_poll(self._h, buf, cap, ctypes.byref(n), int(wait_ms))
        if err != OK:
            raise RuntimeError(f"serving session error: {status_string(err)}")
        out = []
        for i in range(n.value):
            c = buf[i]
            arrs, colors = self._live.pop(int(c.tag))
            out.append((int(c.tag), int(c.status), int(c.rounds), c.t_submit, c.t_admit, c.t_done, colors))
        return out

    def close(self):
        if self._h:
            self._lib.bgpc_session_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
