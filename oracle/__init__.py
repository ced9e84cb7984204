"""CPU oracle for the speculative coloring rounds -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain C, built
with gcc) through ctypes and shares no code with the device library.

Graph arguments are duck-typed: a bipartite graph exposes
``n_a, n_b, a_off, a_idx, b_off, b_idx``; a symmetric graph for distance-2
coloring exposes ``n, off, idx``.  A caller ``order`` (order[k] = the vertex
of rank k) is applied by relabelling vertices to their ranks, re-sorting every
member list, running the natural-order oracle and mapping the colors back.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OK, E_INVALID, E_NOT_CONVERGED, E_INTERNAL = 0, -1, -6, -8
FIRST_FIT, B1, B2, B1_GLOBAL = 0, 1, 2, 3
NET_ALG8, NET_ALG6, NET_ALG6_REVERSE = 0, 1, 2


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        lib.oracle_color.argtypes = [i32, i32, P, P, P, P, i32, u64, i32, i32, i32, i32, i32,
                                     i32, i32, u64, P, P, i32, P, P, P, P, P, P, P]
        lib.oracle_color.restype = ctypes.c_int
        lib.oracle_seq_greedy.argtypes = [i32, i32, P, P, P, P, i32, P]
        lib.oracle_seq_greedy.restype = ctypes.c_int
        lib.oracle_count_violations.argtypes = [i32, i32, P, P, i32, P]
        lib.oracle_count_violations.restype = ctypes.c_int64
        lib.oracle_color_stats.argtypes = [P, i64, P, P]
        lib.oracle_color_stats.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_order_smallest_last.argtypes = [i32, i32, P, P, P, P, i32, i32, i32, P]
        lib.oracle_order_smallest_last.restype = ctypes.c_int64
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (0 leaves them)."""
    _load().oracle_set_threads(int(n))


# ---------------------------------------------------------------------------
# relabelling by rank (plain data movement)


def _relabel_lists(n_rows, off, idx, inv_cols, row_order=None):
    """Rows reordered by row_order (if given), entries mapped through inv_cols
    and re-sorted within each row."""
    off = np.asarray(off, dtype=np.int64)
    idx = np.asarray(idx)
    counts = np.diff(off)
    if row_order is None:
        row_order = np.arange(n_rows)
    new_counts = counts[row_order]
    new_off = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(new_counts, out=new_off[1:])
    new_rows = np.repeat(np.arange(n_rows, dtype=np.int64), new_counts)
    src_pos = np.concatenate([np.arange(off[r], off[r + 1]) for r in row_order]) if n_rows else np.zeros(0, np.int64)
    vals = inv_cols[idx[src_pos]] if idx.size else np.zeros(0, np.int64)
    key = np.lexsort((vals, new_rows))
    return new_off, _c32(vals[key])


def _inverse(order, n):
    order = np.asarray(order, dtype=np.int64)
    if order.shape != (n,) or not np.array_equal(np.sort(order), np.arange(n)):
        raise ValueError("order must be a permutation of the colored vertices")
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n)
    return order, inv


# ---------------------------------------------------------------------------
# the rounds


class Result:
    def __init__(self, status, colors, rounds, log):
        self.status = status
        self.colors = colors
        self.rounds = rounds
        self.log = log

    def __repr__(self):
        return f"Result(status={self.status}, rounds={self.rounds})"


def _run(n_a, n_b, a_off, a_idx, b_off, b_idx, d2, net_color_mask, policy, chunk,
         max_rounds, start_round, init_colors, log_cap, literal_ff=False, net_alg=NET_ALG8,
         net_balance=False, vertex_removal_mask=0):
    lib = _load()
    a_off, b_off = _c64(a_off), _c64(b_off)
    a_idx, b_idx = _c32(a_idx), _c32(b_idx)
    colors = np.full(n_a, -1, dtype=np.int32) if init_colors is None else _c32(init_colors).copy()
    rounds = np.zeros(1, dtype=np.int32)
    lm = np.zeros(log_cap, dtype=np.int32)
    lw = np.zeros(log_cap, dtype=np.int64)
    ll = np.zeros(log_cap, dtype=np.int64)
    le = np.zeros(log_cap, dtype=np.int64)
    lc = np.zeros(log_cap, dtype=np.int32)
    ht = np.zeros(log_cap, dtype=np.uint64)
    hc = np.zeros(log_cap, dtype=np.uint64)
    st = lib.oracle_color(n_a, n_b, _ptr(a_off), _ptr(a_idx), _ptr(b_off), _ptr(b_idx),
                          int(d2), ctypes.c_uint64(net_color_mask & (2 ** 64 - 1)), int(policy), int(chunk),
                          int(max_rounds), int(start_round), int(bool(literal_ff)), int(net_alg),
                          int(bool(net_balance)), ctypes.c_uint64(vertex_removal_mask & (2 ** 64 - 1)),
                          _ptr(colors), _ptr(rounds),
                          log_cap, _ptr(lm), _ptr(lw), _ptr(ll), _ptr(le), _ptr(lc), _ptr(ht), _ptr(hc))
    r = int(rounds[0])
    k = min(r, log_cap)
    log = {"mode": lm[:k].copy(), "w": lw[:k].copy(), "losers": ll[:k].copy(),
           "evicted": le[:k].copy(), "max_color": lc[:k].copy(), "hash_t": ht[:k].copy(),
           "hash_c": hc[:k].copy()}
    return int(st), colors, r, log


def bgpc(g, net_color_mask: int = 0, policy: int = FIRST_FIT, chunk: int = 64,
         max_rounds: int = 0, order=None, init_colors=None, start_round: int = 0,
         log_cap: int = 4096, literal_ff: bool = False, net_alg: int = NET_ALG8,
         net_balance: bool = False, vertex_removal_mask: int = 0) -> Result:
    """Bipartite-graph partial coloring of V_A (Sections II-III, V).
    literal_ff: first-fit rounds gather F(w) member by member instead of
    through per-net color sets (same result, much slower on large nets).
    net_alg: the net-based coloring of Algorithm 8 (default), Algorithm 6, or
    Algorithm 6 with the reverse start; net_balance: net-based rounds choose
    by the policy (Section V).  vertex_removal_mask: rounds whose conflicts
    are checked in the vertex form where that form is exact (same results)."""
    n_a, n_b = int(g.n_a), int(g.n_b)
    a_off, a_idx, b_off, b_idx = g.a_off, g.a_idx, g.b_off, g.b_idx
    inv = None
    if order is not None:
        order, inv = _inverse(order, n_a)
        b_off, b_idx = _relabel_lists(n_b, b_off, b_idx, inv)
        a_off, a_idx = _relabel_lists(n_a, a_off, a_idx, np.arange(n_b, dtype=np.int64), row_order=order)
        if init_colors is not None:
            init_colors = np.asarray(init_colors)[order]
    st, colors, r, log = _run(n_a, n_b, a_off, a_idx, b_off, b_idx, 0, net_color_mask, policy, chunk,
                              max_rounds, start_round, init_colors, log_cap, literal_ff, net_alg,
                              net_balance, vertex_removal_mask)
    if inv is not None:
        colors = colors[inv]
    return Result(st, colors, r, log)


def d2gc(adj, net_color_mask: int = 0, policy: int = FIRST_FIT, chunk: int = 64,
         max_rounds: int = 0, order=None, init_colors=None, start_round: int = 0,
         log_cap: int = 4096, literal_ff: bool = False, net_alg: int = NET_ALG8,
         net_balance: bool = False, vertex_removal_mask: int = 0) -> Result:
    """Distance-2 coloring of a symmetric graph without self loops (Section IV)."""
    n = int(adj.n)
    off, idx = adj.off, adj.idx
    inv = None
    if order is not None:
        order, inv = _inverse(order, n)
        off, idx = _relabel_lists(n, off, idx, inv, row_order=order)
        if init_colors is not None:
            init_colors = np.asarray(init_colors)[order]
    st, colors, r, log = _run(n, n, off, idx, off, idx, 1, net_color_mask, policy, chunk,
                              max_rounds, start_round, init_colors, log_cap, literal_ff, net_alg,
                              net_balance, vertex_removal_mask)
    if inv is not None:
        colors = colors[inv]
    return Result(st, colors, r, log)


def seq_greedy(g, order=None) -> np.ndarray:
    """Sequential first-fit in rank order (bipartite graph)."""
    lib = _load()
    n_a, n_b = int(g.n_a), int(g.n_b)
    a_off, a_idx, b_off, b_idx = g.a_off, g.a_idx, g.b_off, g.b_idx
    inv = None
    if order is not None:
        order, inv = _inverse(order, n_a)
        b_off, b_idx = _relabel_lists(n_b, b_off, b_idx, inv)
        a_off, a_idx = _relabel_lists(n_a, a_off, a_idx, np.arange(n_b, dtype=np.int64), row_order=order)
    a_off, b_off, a_idx, b_idx = _c64(a_off), _c64(b_off), _c32(a_idx), _c32(b_idx)
    out = np.empty(n_a, dtype=np.int32)
    st = lib.oracle_seq_greedy(n_a, n_b, _ptr(a_off), _ptr(a_idx), _ptr(b_off), _ptr(b_idx), 0, _ptr(out))
    if st:
        raise RuntimeError(f"oracle_seq_greedy failed: {st}")
    return out[inv] if inv is not None else out


def seq_greedy_d2(adj) -> np.ndarray:
    lib = _load()
    n = int(adj.n)
    off, idx = _c64(adj.off), _c32(adj.idx)
    out = np.empty(n, dtype=np.int32)
    st = lib.oracle_seq_greedy(n, n, _ptr(off), _ptr(idx), _ptr(off), _ptr(idx), 1, _ptr(out))
    if st:
        raise RuntimeError(f"oracle_seq_greedy failed: {st}")
    return out


def violations(g, colors) -> int:
    """Shared-net color repeats plus uncolored vertices (0 = valid coloring)."""
    lib = _load()
    colors = _c32(colors)
    if hasattr(g, "n_b"):
        b_off, b_idx = _c64(g.b_off), _c32(g.b_idx)
        return int(lib.oracle_count_violations(int(g.n_a), int(g.n_b), _ptr(b_off), _ptr(b_idx), 0, _ptr(colors)))
    off, idx = _c64(g.off), _c32(g.idx)
    return int(lib.oracle_count_violations(int(g.n), int(g.n), _ptr(off), _ptr(idx), 1, _ptr(colors)))


def color_stats(colors) -> dict:
    """Non-empty color sets and their cardinalities (the balancing metrics)."""
    lib = _load()
    colors = _c32(colors)
    oi = np.zeros(5, dtype=np.int64)
    od = np.zeros(2, dtype=np.float64)
    st = lib.oracle_color_stats(_ptr(colors), colors.shape[0], _ptr(oi), _ptr(od))
    if st:
        raise RuntimeError("oracle_color_stats failed")
    return {"n_distinct": int(oi[0]), "max_color": int(oi[1]), "card_min": int(oi[2]),
            "card_max": int(oi[3]), "n_empty_below_max": int(oi[4]),
            "card_mean": float(od[0]), "card_std": float(od[1])}


def order_largest_first(g) -> np.ndarray:
    """Largest-first processing order of a bipartite graph: vertices by
    decreasing key(u) = sum over the nets v of u of (|vtxs(v)| - 1), an upper
    bound of u's distance-2 degree, ties by increasing id.  The paper's
    experiments compare processing orders (Section VI: natural and
    smallest-last); this degree order is the cheap one.  Returns order[k] =
    the vertex of rank k."""
    n_a = int(g.n_a)
    a_off = np.asarray(g.a_off, dtype=np.int64)
    sizes = np.diff(np.asarray(g.b_off, dtype=np.int64))
    key = np.zeros(n_a, dtype=np.int64)
    owner = np.repeat(np.arange(n_a), np.diff(a_off))   # vertex of each (vertex, net) incidence
    np.add.at(key, owner, sizes[np.asarray(g.a_idx, dtype=np.int64)] - 1)
    return np.lexsort((np.arange(n_a), -key)).astype(np.int32)


def d2gc_order_largest_first(adj) -> np.ndarray:
    """The same order for distance-2 coloring: the nets are the closed
    neighbourhoods N[x], so key(u) = sum over x in N[u] of |nbor(x)|."""
    n = int(adj.n)
    off = np.asarray(adj.off, dtype=np.int64)
    deg = np.diff(off)
    key = deg.copy()   # x = u itself
    owner = np.repeat(np.arange(n), deg)
    np.add.at(key, owner, deg[np.asarray(adj.idx, dtype=np.int64)])
    return np.lexsort((np.arange(n), -key)).astype(np.int32)


def _smallest_last(n, a_off, a_idx, b_off, b_idx, n_b, d2, batched, slack_shift=63):
    lib = _load()
    a_off, b_off, a_idx, b_idx = _c64(a_off), _c64(b_off), _c32(a_idx), _c32(b_idx)
    out = np.empty(max(n, 1), dtype=np.int32)
    steps = lib.oracle_order_smallest_last(int(n), int(n_b), _ptr(a_off), _ptr(a_idx), _ptr(b_off), _ptr(b_idx),
                                           int(d2), int(bool(batched)), int(slack_shift), _ptr(out))
    if steps < 0:
        raise RuntimeError("oracle_order_smallest_last failed")
    return out[:n], int(steps)


def order_smallest_last(g, batched: bool = True, with_steps: bool = False, slack_shift: int = 63):
    """Smallest-last order of a bipartite graph (Section VI's other order):
    vertices are removed smallest key first -- key(u) = sum over the nets of u
    of (members still present - 1) -- and ranked in reverse removal order.
    batched: every vertex at the current minimum key leaves in one step (ranks
    of a step ascending by id); with slack_shift < 63 a step takes every key
    up to d + (d >> slack_shift), d the minimum; else one vertex per step,
    ties to the lowest id (quadratic: small graphs only).  Returns order[k] =
    vertex of rank k (and the number of steps with with_steps)."""
    o, st = _smallest_last(g.n_a, g.a_off, g.a_idx, g.b_off, g.b_idx, g.n_b, 0, batched, slack_shift)
    return (o, st) if with_steps else o


def d2gc_order_smallest_last(adj, batched: bool = True, with_steps: bool = False, slack_shift: int = 63):
    """The same order for distance-2 coloring (nets = closed neighbourhoods)."""
    o, st = _smallest_last(adj.n, adj.off, adj.idx, adj.off, adj.idx, adj.n, 1, batched, slack_shift)
    return (o, st) if with_steps else o
