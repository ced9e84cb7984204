"""Seeded synthetic bipartite graphs for the coloring workloads.

This module only draws inputs.  It holds none of the coloring method's
arithmetic, imports nothing from the HIP binding or from the CPU oracle, and
is the one piece of code that both sides (tests, benchmark, oracle runs) share.

Vocabulary follows Section II of the paper: a bipartite graph
G = (V_A u V_B, E) whose V_A side is colored ("vertices") and whose V_B side
defines the neighbourhoods ("nets").  ``b_off/b_idx`` is the row-major CSR of
nets -> vertices (vtxs(v)), ``a_off/a_idx`` its transpose (nets(u)).  Every
member list is sorted ascending and holds no duplicates.  Offsets are int64 on
the host so that the batched workload can be concatenated without overflow;
the device library takes int32 offsets per graph.

Workload recipes (all with numpy's PCG64 bit generator):

* ``random_uniform``  -- each net draws k ~ U{kmin..kmax} distinct vertices,
  uniformly at random (the small plain workload and every batched graph).
* ``stencil27``       -- 3D 27-point stencil Jacobian pattern on a g^3 grid,
  net p = the 3x3x3 box around grid point p truncated at the boundary, vertex
  id x + g*y + g*g*z.
* ``skewed``          -- net sizes from P(k) ~ k^-2.1 on {2..10,000}; vertex
  popularity density ~ (j+1)^(-2/3) on [0, n_A) (a column-degree tail of
  exponent 2.5); distinct members drawn by repeated top-up sampling.
* ``rmat``            -- R-MAT edge list, symmetrised, self loops and duplicate
  edges removed: the adjacency of a unipartite graph for distance-2 coloring.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np


@dataclasses.dataclass
class Bipartite:
    """A bipartite graph in CSR (nets -> vertices) plus CSC (vertices -> nets)."""

    n_a: int
    n_b: int
    b_off: np.ndarray  # int64[n_b + 1]
    b_idx: np.ndarray  # int32[nnz]
    a_off: np.ndarray  # int64[n_a + 1]
    a_idx: np.ndarray  # int32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.b_idx.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for arr in (self.b_off, self.b_idx, self.a_off, self.a_idx):
            h.update(np.ascontiguousarray(arr).tobytes())
        return h.hexdigest()


@dataclasses.dataclass
class Adjacency:
    """A symmetric unipartite graph without self loops, CSR."""

    n: int
    off: np.ndarray  # int64[n + 1]
    idx: np.ndarray  # int32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.idx.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for arr in (self.off, self.idx):
            h.update(np.ascontiguousarray(arr).tobytes())
        return h.hexdigest()


def _offsets_from_counts(counts: np.ndarray) -> np.ndarray:
    off = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def transpose(n_rows: int, n_cols: int, off: np.ndarray, idx: np.ndarray):
    """CSR of the transpose; each output row lists source rows ascending."""
    counts = np.bincount(idx, minlength=n_cols).astype(np.int64)
    t_off = _offsets_from_counts(counts)
    rows = np.repeat(np.arange(n_rows, dtype=np.int32), np.diff(off))
    perm = np.argsort(idx, kind="stable")
    t_idx = rows[perm].astype(np.int32, copy=False)
    return t_off, t_idx


def from_net_lists(n_a: int, n_b: int, b_off, b_idx, name="") -> Bipartite:
    b_off = np.asarray(b_off, dtype=np.int64)
    b_idx = np.asarray(b_idx, dtype=np.int32)
    a_off, a_idx = transpose(n_b, n_a, b_off, b_idx)
    return Bipartite(n_a, n_b, b_off, b_idx, a_off, a_idx, name)


def from_nets(n_a: int, nets, name="") -> Bipartite:
    """Build from a Python list of member lists (small hand-written graphs)."""
    sizes = [len(m) for m in nets]
    b_off = _offsets_from_counts(np.asarray(sizes, dtype=np.int64))
    flat = [int(x) for m in nets for x in sorted(m)]
    b_idx = np.asarray(flat, dtype=np.int32)
    return from_net_lists(n_a, len(nets), b_off, b_idx, name)


def adjacency_from_edges(n: int, edges, name="") -> Adjacency:
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return _symmetrize(n, e[:, 0], e[:, 1], name)


def _symmetrize(n: int, src: np.ndarray, dst: np.ndarray, name="") -> Adjacency:
    keep = src != dst
    src = src[keep].astype(np.int64)
    dst = dst[keep].astype(np.int64)
    keys = np.concatenate([src * n + dst, dst * n + src])
    keys = np.unique(keys)
    rows = keys // n
    cols = (keys % n).astype(np.int32)
    counts = np.bincount(rows, minlength=n).astype(np.int64)
    return Adjacency(n, _offsets_from_counts(counts), cols, name)


# ---------------------------------------------------------------------------
# distinct uniform rows


def _distinct_uniform_rows(rng: np.random.Generator, n_cols: int, k: np.ndarray) -> tuple:
    """For every row i draw k[i] distinct columns uniformly from [0, n_cols).

    A row is redrawn whole while it holds a repeated column, which leaves every
    k-subset equally likely.  Returns (offsets int64, sorted members int32).
    """
    n_rows = k.shape[0]
    kmax = int(k.max()) if n_rows else 0
    out = np.empty((n_rows, kmax), dtype=np.int64)
    todo = np.arange(n_rows)
    sentinel = np.int64(n_cols)
    col_pos = np.arange(kmax)
    while todo.size:
        draw = rng.integers(0, n_cols, size=(todo.size, kmax), dtype=np.int64)
        draw[col_pos[None, :] >= k[todo][:, None]] = sentinel
        draw.sort(axis=1)
        dup = (draw[:, 1:] == draw[:, :-1]) & (draw[:, 1:] != sentinel)
        bad = dup.any(axis=1)
        good = ~bad
        out[todo[good]] = draw[good]
        todo = todo[bad]
    off = _offsets_from_counts(k.astype(np.int64))
    mask = col_pos[None, :] < k[:, None]
    idx = out[mask].astype(np.int32)
    return off, idx


def random_uniform(n_a: int, n_b: int, kmin: int, kmax: int, seed: int, name="") -> Bipartite:
    """Each net takes k ~ U{kmin..kmax} distinct uniformly drawn vertices."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(kmin, kmax + 1, size=n_b, dtype=np.int64)
    b_off, b_idx = _distinct_uniform_rows(rng, n_a, k)
    return from_net_lists(n_a, n_b, b_off, b_idx, name or f"random_{n_a}x{n_b}_k{kmin}-{kmax}_s{seed}")


# ---------------------------------------------------------------------------
# 27-point stencil


def stencil27(g: int, name="") -> Bipartite:
    """Nets = 3x3x3 boxes of a g^3 grid truncated at the boundary.

    The relation is symmetric, so CSC equals CSR.  Offsets (dz, dy, dx) are
    enumerated lexicographically, which lists box members by ascending id.
    """
    n = g * g * g
    ids = np.arange(n, dtype=np.int64)
    x = ids % g
    y = (ids // g) % g
    z = ids // (g * g)
    cols = []
    valids = []
    for dz in (-1, 0, 1):
        vz = (z + dz >= 0) & (z + dz < g)
        for dy in (-1, 0, 1):
            vy = vz & (y + dy >= 0) & (y + dy < g)
            for dx in (-1, 0, 1):
                v = vy & (x + dx >= 0) & (x + dx < g)
                valids.append(v)
                cols.append(ids + dx + g * dy + g * g * dz)
    valid = np.stack(valids, axis=1)
    col = np.stack(cols, axis=1)
    counts = valid.sum(axis=1).astype(np.int64)
    off = _offsets_from_counts(counts)
    idx = col[valid].astype(np.int32)
    del valid, col
    return Bipartite(n, n, off, idx, off.copy(), idx.copy(), name or f"stencil27_{g}^3")


# ---------------------------------------------------------------------------
# skewed nets with power-law vertex popularity


def _zipf_sizes(rng, n: int, exponent: float, kmin: int, kmax: int) -> np.ndarray:
    support = np.arange(kmin, kmax + 1, dtype=np.float64)
    w = support ** (-exponent)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(n)
    pos = np.searchsorted(cdf, u, side="right")
    pos = np.minimum(pos, support.shape[0] - 1)
    return (kmin + pos).astype(np.int64)


def _popular_columns(rng, m: int, n_cols: int) -> np.ndarray:
    """Inverse CDF of the density ~ (x+1)^(-2/3) on [0, n_cols), floored."""
    top = (n_cols + 1.0) ** (1.0 / 3.0) - 1.0
    u = rng.random(m)
    x = np.floor((1.0 + u * top) ** 3 - 1.0)
    return np.clip(x, 0, n_cols - 1).astype(np.int64)


def skewed(n_a: int, n_b: int, seed: int, exponent: float = 2.1, kmin: int = 2, kmax: int = 10000,
           name="") -> Bipartite:
    """Zipf-sized nets whose members follow power-law vertex popularity.

    Each net first draws its size, then draws that many members; repeated
    members are dropped and the shortfall is drawn again until every net holds
    exactly its size in distinct members.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    k = _zipf_sizes(rng, n_b, exponent, kmin, kmax)
    k = np.minimum(k, n_a)
    rows = np.repeat(np.arange(n_b, dtype=np.int64), k)
    cols = _popular_columns(rng, rows.shape[0], n_a)
    while True:
        key = rows * n_a + cols
        key = np.unique(key)
        rows = key // n_a
        cols = key % n_a
        have = np.bincount(rows, minlength=n_b).astype(np.int64)
        short = k - have
        if not short.any():
            break
        extra_rows = np.repeat(np.arange(n_b, dtype=np.int64), short)
        extra_cols = _popular_columns(rng, extra_rows.shape[0], n_a)
        rows = np.concatenate([rows, extra_rows])
        cols = np.concatenate([cols, extra_cols])
    b_off = _offsets_from_counts(k)
    return from_net_lists(n_a, n_b, b_off, cols.astype(np.int32), name or f"skewed_{n_a}x{n_b}_s{seed}")


# ---------------------------------------------------------------------------
# R-MAT


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int, name="") -> Adjacency:
    """R-MAT edges, symmetrised, with self loops and duplicates removed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 1 << scale
    m = edge_factor * n
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    for level in range(scale):
        u = rng.random(m)
        bit = np.int64(1) << np.int64(scale - 1 - level)
        down = u >= ab                      # quadrants c and d: source bit set
        right = ((u >= a) & (u < ab)) | (u >= abc)  # quadrants b and d: target bit set
        src += down.astype(np.int64) * bit
        dst += right.astype(np.int64) * bit
        del u, down, right
    return _symmetrize(n, src, dst, name or f"rmat_s{scale}_ef{edge_factor}_s{seed}")


# ---------------------------------------------------------------------------
# the five named workloads


def log_uniform_int(rng, lo: int, hi: int) -> int:
    return int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_graph(i: int) -> Bipartite:
    """Graph i of the batched workload (seed 1000 + i)."""
    rng = np.random.Generator(np.random.PCG64(1000 + i))
    n_a = log_uniform_int(rng, 1000, 200000)
    n_b = log_uniform_int(rng, 1000, 200000)
    k = rng.integers(3, 31, size=n_b, dtype=np.int64)
    b_off, b_idx = _distinct_uniform_rows(rng, n_a, k)
    return from_net_lists(n_a, n_b, b_off, b_idx, f"batch_{i}")


def batch_sizes(i: int) -> tuple:
    """(n_A, n_B) of batched graph i without drawing its edges."""
    rng = np.random.Generator(np.random.PCG64(1000 + i))
    return log_uniform_int(rng, 1000, 200000), log_uniform_int(rng, 1000, 200000)


def config(i: int, scale_down: int = 0):
    """The named workloads.  ``scale_down`` shrinks the large ones for tests."""
    if i == 0:
        return random_uniform(20000, 20000, 2, 8, seed=1, name="random20k")
    if i == 1:
        g = 128 >> scale_down
        return stencil27(g)
    if i == 2:
        n = 4194304 >> scale_down
        return skewed(n, n, seed=3, kmax=min(10000, n), name=f"skewed_{n}")
    if i == 3:
        return rmat(22 - scale_down, 16, 0.57, 0.19, 0.19, seed=4)
    raise ValueError("config index must be 0..3 (the batched workload is batch_graph(i))")
