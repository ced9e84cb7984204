"""Parity of the HIP coloring library with the CPU oracle (bit-exact).

Every case runs the C ABI through the ctypes binding on cuda:0 and compares
whole color arrays with the oracle on the same seeded input, round by round
where the case is small, and always on the final coloring, the number of
rounds and the per-round log.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1701_02628_amd import bgpc, synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _gpu_bgpc(cuda, g, dev=None, **kw):
    import torch
    A, B = dev if dev is not None else bgpc.upload_bipartite(g)
    out = torch.full((g.n_a,), -7, dtype=torch.int32, device=cuda)
    init = kw.pop("init_colors", None)
    if init is not None:
        out.copy_(torch.from_numpy(np.asarray(init, np.int32)))
    order = kw.pop("order", None)
    if order is not None:
        order = torch.from_numpy(np.asarray(order, np.int32)).to(cuda)
    res = bgpc.bgpc_color(A, B, order, out, log_cap=kw.pop("log_cap", 4096), **kw)
    torch.cuda.synchronize()
    return res, out.cpu().numpy()


def _gpu_d2(cuda, adj, dev=None, **kw):
    import torch
    D = dev if dev is not None else bgpc.upload_adjacency(adj)
    out = torch.full((adj.n,), -7, dtype=torch.int32, device=cuda)
    init = kw.pop("init_colors", None)
    if init is not None:
        out.copy_(torch.from_numpy(np.asarray(init, np.int32)))
    order = kw.pop("order", None)
    if order is not None:
        order = torch.from_numpy(np.asarray(order, np.int32)).to(cuda)
    res = bgpc.d2gc_color(D, order, out, log_cap=kw.pop("log_cap", 4096), **kw)
    torch.cuda.synchronize()
    return res, out.cpu().numpy()


def _compare_full(res, colors, ref):
    assert res.status == ref.status, (res.status, ref.status)
    assert res.rounds == ref.rounds, (res.rounds, ref.rounds)
    assert np.array_equal(colors, ref.colors), np.flatnonzero(colors != ref.colors)[:10]
    for key in ("mode", "w", "losers", "evicted", "max_color"):
        assert np.array_equal(res.log[key], ref.log[key]), (key, res.log[key][:20], ref.log[key][:20])


def _worked_cases():
    with open(os.path.join(HERE, "golden", "worked_examples.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _worked_cases(), ids=lambda c: c["name"])
def test_worked_examples_round_by_round(cuda, case):
    if case["kind"] == "bgpc":
        g = synth.from_nets(case["n"], case["nets"])
        dev = bgpc.upload_bipartite(g)
        run = lambda **kw: _gpu_bgpc(cuda, g, dev, **kw)
    else:
        g = synth.adjacency_from_edges(case["n"], case["edges"])
        dev = bgpc.upload_adjacency(g)
        run = lambda **kw: _gpu_d2(cuda, g, dev, **kw)
    states = case["states"]
    extra = dict(net_alg=case.get("net_alg", 0), flags=bgpc.NET_BALANCE if case.get("net_balance") else 0)
    if "init_colors" in case:
        extra["init_colors"] = case["init_colors"]
        extra["flags"] |= bgpc.RESUME
    for k, expect in enumerate(states, start=1):
        res, colors = run(net_color_mask=case["net_color_mask"], policy=case["policy"], chunk=case["chunk"],
                          max_rounds=k, **extra)
        assert colors.tolist() == expect, (k, colors.tolist(), expect)
        assert res.status == (bgpc.OK if k == len(states) else bgpc.E_NOT_CONVERGED)
        assert res.rounds == k


def test_config0_round_by_round(cuda):
    g = synth.config(0)
    dev = bgpc.upload_bipartite(g)
    full = oracle.bgpc(g)
    assert full.status == 0
    for k in range(1, full.rounds + 1):
        ref = oracle.bgpc(g, max_rounds=k)
        res, colors = _gpu_bgpc(cuda, g, dev, max_rounds=k)
        assert np.array_equal(colors, ref.colors), (k, np.flatnonzero(colors != ref.colors)[:10])
        assert res.rounds == ref.rounds
    res, colors = _gpu_bgpc(cuda, g, dev)
    _compare_full(res, colors, full)


SCHEDULES = [
    ("V-V", dict(net_color_mask=0)),
    ("N1", dict(net_color_mask=0b1)),
    ("V-then-N", dict(net_color_mask=0b10)),
    ("N2", dict(net_color_mask=0b11)),
    ("N-every-5th", dict(net_color_mask=0b100001)),
    ("B1", dict(policy=1, chunk=64)),
    ("B2", dict(policy=2, chunk=64)),
    ("B1-T7", dict(policy=1, chunk=7)),
    ("B2-T100", dict(policy=2, chunk=100)),
    ("N1-B1", dict(net_color_mask=1, policy=1, chunk=64)),
    ("N1-B2", dict(net_color_mask=1, policy=2, chunk=64)),
    ("B1G", dict(policy=3, chunk=64)),
    ("N1-B1G-T5", dict(net_color_mask=1, policy=3, chunk=5)),
]

GRAPHS = [
    # (n_a, n_b, kmin, kmax, seed): several compaction tiles and a ragged tail
    (5003, 4001, 2, 8, 11),
    (20481, 9000, 3, 30, 12),
    (3000, 6000, 1, 5, 13),
]


@pytest.mark.parametrize("shape", GRAPHS, ids=lambda s: f"{s[0]}x{s[1]}k{s[2]}-{s[3]}")
@pytest.mark.parametrize("sched", SCHEDULES, ids=lambda s: s[0])
def test_random_schedules(cuda, shape, sched):
    n_a, n_b, kmin, kmax, seed = shape
    g = synth.random_uniform(n_a, n_b, kmin, kmax, seed)
    ref = oracle.bgpc(g, **sched[1])
    res, colors = _gpu_bgpc(cuda, g, **sched[1])
    _compare_full(res, colors, ref)
    assert oracle.violations(g, colors) == 0


def test_colors_beyond_64(cuda):
    """Dense nets push first-fit past 63: the wide paths and pairwise checks."""
    g = synth.random_uniform(3000, 2500, 40, 90, 21)
    for kw in (dict(), dict(net_color_mask=1), dict(policy=1), dict(policy=2), dict(net_color_mask=0b11),
               dict(policy=3)):
        ref = oracle.bgpc(g, **kw)
        res, colors = _gpu_bgpc(cuda, g, **kw)
        _compare_full(res, colors, ref)
        assert int(colors.max()) >= 64


def test_big_nets(cuda):
    """Nets above 64 members (LDS hash) and above 4096 members (color windows)."""
    rng = np.random.Generator(np.random.PCG64(5))
    n_a = 12000
    nets = [rng.choice(n_a, size=int(s), replace=False) for s in (5000, 4200, 700, 130, 65)]
    nets += [rng.choice(n_a, size=int(rng.integers(2, 9)), replace=False) for _ in range(6000)]
    g = synth.from_nets(n_a, nets)
    for kw in (dict(), dict(net_color_mask=1), dict(net_color_mask=0b101), dict(policy=2, net_color_mask=1)):
        ref = oracle.bgpc(g, **kw)
        res, colors = _gpu_bgpc(cuda, g, **kw)
        _compare_full(res, colors, ref)


def test_skewed_small(cuda):
    """Vertices of up to 1,603 nets: under B1/B2 their color words are
    precomputed per round (more than 128 nets) and searched as one row."""
    g = synth.skewed(30000, 30000, seed=3, kmax=3000)
    for kw in (dict(net_color_mask=1), dict(net_color_mask=1, policy=1), dict(net_color_mask=1, policy=2),
               dict(net_color_mask=1, policy=1, chunk=7), dict(policy=2, chunk=200), dict(net_color_mask=1, policy=3)):
        ref = oracle.bgpc(g, **kw)
        res, colors = _gpu_bgpc(cuda, g, **kw)
        _compare_full(res, colors, ref)


def test_d2gc_hubs(cuda):
    """Two hubs whose closed neighbourhoods exceed 4,096 members: removal in
    those nets lists the proposals in LDS, or sweeps color windows when there
    are too many of them."""
    rng = np.random.Generator(np.random.PCG64(8))
    n = 8000
    edges = [(0, i) for i in range(1, 5001)] + [(n - 1, i) for i in range(2000, n - 1)]
    e = rng.integers(1, n, size=(20000, 2))
    edges += [(int(a), int(b)) for a, b in e if a != b]
    adj = synth.adjacency_from_edges(n, edges)
    assert int((np.diff(adj.off) + 1 > 4096).sum()) == 2
    # (first-fit on this graph costs the oracle minutes; the full-size R-MAT
    # case covers first-fit with such nets)
    for kw in (dict(policy=1, net_color_mask=1), dict(policy=2, chunk=16, net_color_mask=1)):
        ref = oracle.d2gc(adj, log_cap=8192, **kw)
        res, colors = _gpu_d2(cuda, adj, log_cap=8192, **kw)
        _compare_full(res, colors, ref)


@pytest.mark.parametrize("mask", [0, 1, 0b10, 0b11])
def test_d2gc_rmat_small(cuda, mask):
    adj = synth.rmat(11, 8, 0.57, 0.19, 0.19, seed=9)
    ref = oracle.d2gc(adj, net_color_mask=mask)
    res, colors = _gpu_d2(cuda, adj, net_color_mask=mask)
    _compare_full(res, colors, ref)
    assert oracle.violations(adj, colors) == 0


@pytest.mark.parametrize("mask", [0, 1, 0b10, 0b101])
def test_standing_proposals_mixed_schedules(cuda, mask):
    """Standing proposals forced on small graphs with nets above 64 members
    (pending lists, nets left with one pending member skipped by vertex
    rounds, first-fit skips through zf) under schedules that alternate
    vertex- and net-based rounds, distance-1 and distance-2: colors, rounds
    and round log equal the oracle's."""
    t = bgpc.tuning(standing=1)
    adj = synth.rmat(11, 8, 0.57, 0.19, 0.19, seed=9)
    ref = oracle.d2gc(adj, net_color_mask=mask)
    res, colors = _gpu_d2(cuda, adj, net_color_mask=mask, tune=t)
    _compare_full(res, colors, ref)
    if mask:
        g = synth.skewed(30000, 30000, seed=5, kmax=3000, name="skewed30k")
        ref = oracle.bgpc(g, net_color_mask=mask)
        res, colors = _gpu_bgpc(cuda, g, net_color_mask=mask, tune=t)
        _compare_full(res, colors, ref)


def test_d2gc_policies(cuda):
    adj = synth.rmat(10, 4, 0.57, 0.19, 0.19, seed=10)
    for kw in (dict(policy=1), dict(policy=2), dict(policy=1, net_color_mask=1), dict(policy=3, net_color_mask=1)):
        ref = oracle.d2gc(adj, **kw)
        res, colors = _gpu_d2(cuda, adj, **kw)
        _compare_full(res, colors, ref)
    adj = synth.rmat(11, 8, 0.57, 0.19, 0.19, seed=9)   # 21 vertices of more than 128 closed neighbourhoods
    for kw in (dict(policy=1, net_color_mask=1), dict(policy=2, net_color_mask=1), dict(policy=2, chunk=5)):
        ref = oracle.d2gc(adj, **kw)
        res, colors = _gpu_d2(cuda, adj, **kw)
        _compare_full(res, colors, ref)


def test_edge_cases(cuda):
    import torch
    # no vertices
    g = synth.from_nets(0, [])
    A, B = bgpc.upload_bipartite(g)
    out = torch.zeros(1, dtype=torch.int32, device=cuda)
    r = bgpc.bgpc_color(A, B, None, out)
    assert r.status == bgpc.OK and r.rounds == 0
    # no nets: everything isolated -> color 0 in one round, under every schedule
    g = synth.from_nets(777, [])
    for kw in (dict(), dict(net_color_mask=1), dict(policy=1), dict(policy=2)):
        ref = oracle.bgpc(g, **kw)
        res, colors = _gpu_bgpc(cuda, g, **kw)
        _compare_full(res, colors, ref)
        assert colors.tolist() == [0] * 777 and res.rounds == 1
    # empty and single-member nets, vertices without nets
    g = synth.from_nets(50, [[], [3], [1, 2, 3], [], [40], [0, 49]] + [[i, i + 1] for i in range(10, 30)])
    for kw in (dict(), dict(net_color_mask=1), dict(net_color_mask=0b11), dict(policy=1, chunk=3)):
        ref = oracle.bgpc(g, **kw)
        res, colors = _gpu_bgpc(cuda, g, **kw)
        _compare_full(res, colors, ref)
    # one vertex, one net
    g = synth.from_nets(1, [[0]])
    res, colors = _gpu_bgpc(cuda, g, net_color_mask=1)
    assert colors.tolist() == [0] and res.rounds == 1


def test_strict_validation(cuda):
    import torch
    g = synth.from_nets(6, [[0, 1, 2], [2, 3], [4, 5]])
    A, B = bgpc.upload_bipartite(g)
    out = torch.zeros(6, dtype=torch.int32, device=cuda)
    assert bgpc.bgpc_color(A, B, None, out, flags=bgpc.STRICT).status == bgpc.OK
    bad = B.indices.clone()
    bad[0], bad[1] = bad[1].item(), bad[0].item()
    Bu = bgpc.DeviceCsr(B.offsets, bad, B.n_rows, B.n_cols)
    assert bgpc.bgpc_color(A, Bu, None, out, flags=bgpc.STRICT).status == bgpc.E_UNSORTED
    g2 = synth.from_nets(6, [[0, 1, 2], [2, 4], [4, 5]])
    A2, _ = bgpc.upload_bipartite(g2)
    assert bgpc.bgpc_color(A2, B, None, out, flags=bgpc.STRICT).status == bgpc.E_NOT_TRANSPOSE
    adj = synth.adjacency_from_edges(4, [(0, 1), (1, 2)])
    D = bgpc.upload_adjacency(adj)
    out4 = torch.zeros(4, dtype=torch.int32, device=cuda)
    assert bgpc.d2gc_color(D, None, out4, flags=bgpc.STRICT).status == bgpc.OK
    # drop one direction of an edge -> not symmetric
    off = np.array([0, 1, 2, 3, 3]); idx = np.array([1, 0, 1])  # 0-1, 1-0, 2-1 (missing 1-2)
    Dn = bgpc.upload_csr(off, idx, 4, 4)
    assert bgpc.d2gc_color(Dn, None, out4, flags=bgpc.STRICT).status == bgpc.E_NOT_SYMMETRIC
    off = np.array([0, 1, 2, 2, 2]); idx = np.array([0, 1])   # self loops
    Ds = bgpc.upload_csr(off, idx, 4, 4)
    assert bgpc.d2gc_color(Ds, None, out4, flags=bgpc.STRICT).status == bgpc.E_NOT_SYMMETRIC
    # bad options
    assert bgpc.bgpc_color(A, B, None, out, policy=7).status == bgpc.E_INVALID
    assert bgpc.bgpc_color(A, B, None, out, chunk=0).status == bgpc.E_INVALID


@pytest.mark.parametrize("mask", [0, 0b1, 0b110])
def test_resume_matches_uninterrupted(cuda, mask):
    g = synth.random_uniform(9000, 7000, 2, 12, 31)
    full = oracle.bgpc(g, net_color_mask=mask)
    for k in (1, 2, 4):
        part, colors_k = _gpu_bgpc(cuda, g, net_color_mask=mask, max_rounds=k)
        assert part.status == bgpc.E_NOT_CONVERGED
        res, colors = _gpu_bgpc(cuda, g, net_color_mask=mask, init_colors=colors_k, start_round=k,
                                flags=bgpc.RESUME)
        assert res.status == bgpc.OK
        assert np.array_equal(colors, full.colors)
        assert res.rounds + k == full.rounds
        ref = oracle.bgpc(g, net_color_mask=mask, init_colors=colors_k, start_round=k)
        _compare_full(res, colors, ref)


def test_color_stats(cuda):
    import torch
    rng = np.random.Generator(np.random.PCG64(77))
    for colors in (rng.integers(-1, 300, size=100000), np.array([5, 5, 5, -1]), np.arange(1000) % 7,
                   rng.integers(0, 3, size=17)):
        colors = colors.astype(np.int32)
        got = bgpc.color_stats(torch.from_numpy(colors).to(cuda))
        ref = oracle.color_stats(colors)
        for k in ("n_distinct", "max_color", "card_min", "card_max", "n_empty_below_max"):
            assert got[k] == ref[k], (k, got[k], ref[k])
        assert abs(got["card_mean"] - ref["card_mean"]) <= 1e-12 * max(1.0, abs(ref["card_mean"]))
        assert abs(got["card_std"] - ref["card_std"]) <= 1e-12 * max(1.0, abs(ref["card_std"]))


def test_repeatable(cuda):
    g = synth.random_uniform(30000, 30000, 3, 30, 41)
    dev = bgpc.upload_bipartite(g)
    first = None
    for _ in range(3):
        res, colors = _gpu_bgpc(cuda, g, dev, net_color_mask=1)
        if first is None:
            first = colors
        assert np.array_equal(colors, first)


@pytest.mark.parametrize("mask", [0, 0b1, 0b10, 0b11])
def test_stencil_small(cuda, mask):
    g = synth.stencil27(24)
    ref = oracle.bgpc(g, net_color_mask=mask)
    res, colors = _gpu_bgpc(cuda, g, net_color_mask=mask)
    _compare_full(res, colors, ref)


@pytest.mark.parametrize("shape", GRAPHS + [(4000, 4000, 30, 60, 14)], ids=lambda s: f"{s[0]}x{s[1]}k{s[2]}-{s[3]}")
@pytest.mark.parametrize("mask", [0, 0b1, 0b101])
def test_incremental_rounds(cuda, shape, mask):
    """BGPC_INCREMENTAL recomputes only changed vertices: same results."""
    n_a, n_b, kmin, kmax, seed = shape
    g = synth.random_uniform(n_a, n_b, kmin, kmax, seed)
    ref = oracle.bgpc(g, net_color_mask=mask)
    res, colors = _gpu_bgpc(cuda, g, net_color_mask=mask, flags=bgpc.INCREMENTAL)
    _compare_full(res, colors, ref)
    for k in (1, 2, 3, 5):
        part = oracle.bgpc(g, net_color_mask=mask, max_rounds=k)
        res, colors = _gpu_bgpc(cuda, g, net_color_mask=mask, flags=bgpc.INCREMENTAL, max_rounds=k)
        assert np.array_equal(colors, part.colors) and res.status == part.status


def test_incremental_stencil_and_d2(cuda):
    g = synth.stencil27(20)
    ref = oracle.bgpc(g)
    res, colors = _gpu_bgpc(cuda, g, flags=bgpc.INCREMENTAL)
    _compare_full(res, colors, ref)
    adj = synth.adjacency_from_edges(3000, [(i, (i * 7 + 3) % 3000) for i in range(3000)] +
                                     [(i, (i + 1) % 3000) for i in range(3000)])
    ref = oracle.d2gc(adj)
    res, colors = _gpu_d2(cuda, adj, flags=bgpc.INCREMENTAL)
    _compare_full(res, colors, ref)


def test_profile_counters(cuda):
    import torch
    g = synth.stencil27(32)
    A, B = bgpc.upload_bipartite(g)
    out = torch.empty(g.n_a, dtype=torch.int32, device=cuda)
    for kid in (bgpc.PROF_CONFLICT, bgpc.PROF_COLOR):
        pr = bgpc.Profile(kid, 0, 0.0, 0.0, 0.0)
        r = bgpc.bgpc_color(A, B, None, out, prof=pr)
        assert r.status == 0
        # the lookahead may queue a few empty rounds after the last one
        assert r.rounds <= pr.launches <= r.rounds + 8 and pr.ms > 0 and pr.bytes > 0
        # the removal scan reads no more than the round's nets
        assert 0 < pr.bytes_scanned <= pr.bytes * (1 + 1e-9)


@pytest.mark.parametrize("shape", [(300, 20000, 3, 30, 5), (1200, 60000, 3, 30, 6), (64, 5000, 2, 9, 7)],
                         ids=lambda s: f"{s[0]}x{s[1]}")
def test_dense_small_graphs(cuda, shape):
    """Few vertices, many nets: nearly every pair conflicts (one-workgroup
    dense route); round by round on the first rounds, then whole."""
    n_a, n_b, kmin, kmax, seed = shape
    g = synth.random_uniform(n_a, n_b, kmin, kmax, seed)
    ref = oracle.bgpc(g)
    res, colors = _gpu_bgpc(cuda, g)
    _compare_full(res, colors, ref)
    for k in (1, 2, 7):
        part = oracle.bgpc(g, max_rounds=k)
        res, colors = _gpu_bgpc(cuda, g, max_rounds=k)
        assert res.status == part.status and np.array_equal(colors, part.colors)
        for key in ("w", "losers", "max_color"):
            assert np.array_equal(res.log[key], part.log[key]), key


def _degree_order(off):
    """Largest degree first, ties by id (a simple caller ordering)."""
    deg = np.diff(np.asarray(off, dtype=np.int64))
    return np.lexsort((np.arange(deg.shape[0]), -deg)).astype(np.int32)


@pytest.mark.parametrize("mask,policy", [(0, 0), (0b1, 0), (0, 1), (0b11, 2)], ids=["vv", "n1", "b1", "n1n2_b2"])
def test_caller_order(cuda, mask, policy):
    """Ranks from a caller permutation (random, and degree-descending): the
    library relabels on the device; the oracle relabels on the host."""
    g = synth.random_uniform(3000, 2500, 2, 12, 21)
    perms = [np.random.Generator(np.random.PCG64(5)).permutation(g.n_a).astype(np.int32), _degree_order(g.a_off)]
    for perm in perms:
        ref = oracle.bgpc(g, net_color_mask=mask, policy=policy, order=perm)
        res, colors = _gpu_bgpc(cuda, g, net_color_mask=mask, policy=policy, order=perm)
        _compare_full(res, colors, ref)


def test_caller_order_big_nets_d2_resume(cuda):
    """Nets above 64 members under an order (rows re-sorted on the device),
    distance-2 under an order, and resuming from partial colors with one."""
    g = synth.skewed(6000, 6000, seed=23, kmax=600, name="skewed_small_order")
    perm = np.random.Generator(np.random.PCG64(6)).permutation(g.n_a).astype(np.int32)
    ref = oracle.bgpc(g, net_color_mask=1, order=perm)
    res, colors = _gpu_bgpc(cuda, g, net_color_mask=1, order=perm)
    _compare_full(res, colors, ref)
    adj = synth.rmat(10, 8, 0.57, 0.19, 0.19, seed=7)
    dperm = _degree_order(adj.off)
    for mask in (0, 0b1):
        ref = oracle.d2gc(adj, net_color_mask=mask, order=dperm)
        res, colors = _gpu_d2(cuda, adj, net_color_mask=mask, order=dperm)
        _compare_full(res, colors, ref)
    part = oracle.bgpc(g, net_color_mask=1, order=perm, max_rounds=2)
    ref = oracle.bgpc(g, order=perm, init_colors=part.colors, start_round=2, net_color_mask=1)
    res, colors = _gpu_bgpc(cuda, g, order=perm, init_colors=part.colors, start_round=2, net_color_mask=1,
                            flags=bgpc.RESUME)
    _compare_full(res, colors, ref)


def test_caller_order_rejected_when_not_a_permutation(cuda):
    g = synth.random_uniform(500, 400, 2, 6, 22)
    bad = np.arange(g.n_a, dtype=np.int32)
    bad[7] = bad[8]
    res, _ = _gpu_bgpc(cuda, g, order=bad)
    assert res.status == bgpc.E_INVALID
    bad[7] = g.n_a + 3
    res, _ = _gpu_bgpc(cuda, g, order=bad)
    assert res.status == bgpc.E_INVALID


def test_caller_order_edge_cases(cuda):
    """Vertices in no net, and a single vertex, under a reversing order."""
    for g in (synth.from_nets(6, []), synth.from_nets(5, [[1, 3], [], [0, 1, 2, 3, 4]]), synth.from_nets(1, [[0]])):
        perm = np.arange(g.n_a, dtype=np.int32)[::-1].copy()
        for mask in (0, 1):
            ref = oracle.bgpc(g, net_color_mask=mask, order=perm)
            res, colors = _gpu_bgpc(cuda, g, net_color_mask=mask, order=perm)
            _compare_full(res, colors, ref)


def test_largest_first_orders(cuda):
    """Device largest-first orders equal the oracle's, and coloring under them
    matches the oracle's run under the same order."""
    cases = [synth.random_uniform(5003, 4001, 2, 8, 11), synth.skewed(6000, 6000, seed=23, kmax=600, name="sk6k"),
             synth.stencil27(12), synth.from_nets(7, []), synth.from_nets(5, [[0, 1, 2], [1, 3], [2, 3, 4], [0, 4]])]
    for g in cases:
        A, B = bgpc.upload_bipartite(g)
        got = bgpc.order_largest_first(A, B)
        ref = oracle.order_largest_first(g)
        assert np.array_equal(got.cpu().numpy(), ref)
        for kw in (dict(), dict(net_color_mask=1)):
            res, colors = _gpu_bgpc(cuda, g, (A, B), order=ref, **kw)
            _compare_full(res, colors, oracle.bgpc(g, order=ref, **kw))
    adj = synth.rmat(11, 8, 0.57, 0.19, 0.19, seed=9)
    D = bgpc.upload_adjacency(adj)
    got = bgpc.d2gc_order_largest_first(D)
    ref = oracle.d2gc_order_largest_first(adj)
    assert np.array_equal(got.cpu().numpy(), ref)
    res, colors = _gpu_d2(cuda, adj, D, order=ref, net_color_mask=1)
    _compare_full(res, colors, oracle.d2gc(adj, order=ref, net_color_mask=1))


def test_net_round_size_limit(cuda):
    """A net-based round needs the largest net's bitmap in LDS: a net of
    230,000 members is past that limit and the call says so before any round."""
    g = synth.from_nets(230000, [list(range(230000))])
    res, _ = _gpu_bgpc(cuda, g, net_color_mask=1)
    assert res.status == bgpc.E_UNSUPPORTED and res.rounds == 0
    res, colors = _gpu_bgpc(cuda, g, net_color_mask=1 << 5)   # a net-based round later on: refused up front
    assert res.status == bgpc.E_UNSUPPORTED and res.rounds == 0


def test_b1_global_resume(cuda):
    """B1G reads col_max from the colors already present: resuming must see
    the ones it was handed."""
    g = synth.random_uniform(9000, 7000, 2, 12, 31)
    part = oracle.bgpc(g, policy=3, max_rounds=3)
    ref = oracle.bgpc(g, policy=3, init_colors=part.colors, start_round=3)
    res, colors = _gpu_bgpc(cuda, g, policy=3, init_colors=part.colors, start_round=3, flags=bgpc.RESUME)
    _compare_full(res, colors, ref)
    assert np.array_equal(colors, oracle.bgpc(g, policy=3).colors)


# ---------------------------------------------------------------------------
# net-based variants (Algorithm 6, net-based balancing), removal forms, hashes


def _oracle_kw(kw):
    """bgpc_color keyword arguments -> the oracle's."""
    out = {k: v for k, v in kw.items() if k in ("net_color_mask", "policy", "chunk", "net_alg", "max_rounds")}
    if kw.get("flags", 0) & bgpc.NET_BALANCE:
        out["net_balance"] = True
    return out


NET_VARIANTS = [
    ("alg6-N1", dict(net_color_mask=1, net_alg=1)),
    ("alg6r-N1", dict(net_color_mask=1, net_alg=2)),
    ("alg6-N2", dict(net_color_mask=0b11, net_alg=1)),
    ("alg6-V-then-N", dict(net_color_mask=0b10, net_alg=1)),
    ("alg6r-every-3rd", dict(net_color_mask=0b1001001, net_alg=2)),
    ("netB1-N1", dict(net_color_mask=1, policy=1, flags=8)),
    ("netB2-N2", dict(net_color_mask=0b11, policy=2, flags=8)),
    ("netB1G-N1", dict(net_color_mask=1, policy=3, flags=8)),
    ("netB2-T5", dict(net_color_mask=0b101, policy=2, chunk=5, flags=8)),
    ("netFF-N1", dict(net_color_mask=1, policy=0, flags=8)),
]


@pytest.mark.parametrize("shape", GRAPHS[:2] + [(2000, 1500, 60, 140, 15)], ids=lambda s: f"{s[0]}x{s[1]}k{s[2]}-{s[3]}")
@pytest.mark.parametrize("var", NET_VARIANTS, ids=lambda v: v[0])
def test_net_variants(cuda, shape, var):
    n_a, n_b, kmin, kmax, seed = shape
    g = synth.random_uniform(n_a, n_b, kmin, kmax, seed)
    ref = oracle.bgpc(g, **_oracle_kw(var[1]))
    res, colors = _gpu_bgpc(cuda, g, **var[1])
    _compare_full(res, colors, ref)


@pytest.mark.parametrize("var", NET_VARIANTS, ids=lambda v: v[0])
def test_net_variants_skewed_and_d2(cuda, var):
    g = synth.skewed(30000, 30000, seed=5, kmax=3000, name="skewed30k")
    ref = oracle.bgpc(g, **_oracle_kw(var[1]))
    res, colors = _gpu_bgpc(cuda, g, **var[1])
    _compare_full(res, colors, ref)
    adj = synth.rmat(11, 8, 0.57, 0.19, 0.19, seed=4)
    ref = oracle.d2gc(adj, **_oracle_kw(var[1]))
    res, colors = _gpu_d2(cuda, adj, **var[1])
    _compare_full(res, colors, ref)


@pytest.mark.parametrize("sched", [("V-V", dict()), ("N1", dict(net_color_mask=1)), ("B2", dict(policy=2)),
                                   ("V-then-N", dict(net_color_mask=0b10)), ("alg6-N1", dict(net_color_mask=1, net_alg=1))],
                         ids=lambda s: s[0])
def test_vertex_form_removal(cuda, sched):
    """net_conflict_mask = 0: the vertex form (Algorithm 5) wherever it is
    exact, the net form elsewhere; same rounds and colors as the oracle."""
    for g in (synth.random_uniform(5003, 4001, 2, 8, 11), synth.stencil27(24)):
        ref = oracle.bgpc(g, **sched[1])
        res, colors = _gpu_bgpc(cuda, g, net_conflict_mask=0, **sched[1])
        _compare_full(res, colors, ref)
        # every other round in the vertex form
        res, colors = _gpu_bgpc(cuda, g, net_conflict_mask=0x5555555555555555, **sched[1])
        _compare_full(res, colors, ref)
    adj = synth.rmat(11, 8, 0.57, 0.19, 0.19, seed=4)
    ref = oracle.d2gc(adj, net_color_mask=1)
    res, colors = _gpu_d2(cuda, adj, net_color_mask=1, net_conflict_mask=0)
    _compare_full(res, colors, ref)


@pytest.mark.parametrize("kw", [dict(), dict(net_color_mask=0b101), dict(policy=2, chunk=9),
                                dict(net_color_mask=1, flags=8, policy=1)], ids=str)
def test_round_hashes_and_times(cuda, kw):
    """FNV-1a-64 of the tentative colors after each round's coloring step and
    of the colors after each round, against the oracle's; per-round event
    times are positive and sum to at most the call."""
    g = synth.random_uniform(5003, 4001, 2, 8, 11)
    ref = oracle.bgpc(g, **_oracle_kw(kw))
    res, colors = _gpu_bgpc(cuda, g, log_hashes=True, **kw)
    _compare_full(res, colors, ref)
    assert np.array_equal(res.log["hash_t"], ref.log["hash_t"])
    assert np.array_equal(res.log["hash_c"], ref.log["hash_c"])
    big = synth.stencil27(40)
    res, _ = _gpu_bgpc(cuda, big)
    assert (res.log["round_ms"] > 0).all() and len(res.log["round_ms"]) == res.rounds


def test_smallest_last_orders(cuda):
    """The device's smallest-last orders (removal steps, with and without the
    slack) equal the oracle's, bipartite and distance-2; coloring in that order
    equals the oracle's coloring in it."""
    import torch
    for g in (synth.random_uniform(5003, 4001, 2, 8, 11), synth.stencil27(20),
              synth.skewed(30000, 30000, seed=5, kmax=3000, name="skewed30k"), synth.from_nets(7, [])):
        A, B = bgpc.upload_bipartite(g)
        for shift in (3, 63):
            got, steps = bgpc.order_smallest_last(A, B, slack_shift=shift, with_steps=True)
            want, wsteps = oracle.order_smallest_last(g, with_steps=True, slack_shift=shift)
            assert steps == wsteps and np.array_equal(got.cpu().numpy(), want), (g.name, shift)
        order = want
        ref = oracle.bgpc(g, order=order, net_color_mask=1)
        res, colors = _gpu_bgpc(cuda, g, order=order, net_color_mask=1)
        _compare_full(res, colors, ref)
    adj = synth.rmat(12, 8, 0.57, 0.19, 0.19, seed=4)
    D = bgpc.upload_adjacency(adj)
    got, steps = bgpc.d2gc_order_smallest_last(D, slack_shift=3, with_steps=True)
    want, wsteps = oracle.d2gc_order_smallest_last(adj, with_steps=True, slack_shift=3)
    assert steps == wsteps and np.array_equal(got.cpu().numpy(), want)
    ref = oracle.d2gc(adj, order=want, net_color_mask=1)
    res, colors = _gpu_d2(cuda, adj, order=want, net_color_mask=1)
    _compare_full(res, colors, ref)


def _grid7(g):
    """Adjacency of the 7-point stencil on a g^3 grid (degree <= 6)."""
    ids = np.arange(g ** 3).reshape(g, g, g)
    e = [np.stack([ids[:, :, :-1].ravel(), ids[:, :, 1:].ravel()], 1),
         np.stack([ids[:, :-1, :].ravel(), ids[:, 1:, :].ravel()], 1),
         np.stack([ids[:-1, :, :].ravel(), ids[1:, :, :].ravel()], 1)]
    return synth.adjacency_from_edges(g ** 3, np.concatenate(e))


def test_front_driven_rounds(cuda):
    """Front-driven first-fit rounds (only vertices whose nets hold color 0
    are recolored, removal over the listed dirty nets, winners streamed) on
    graphs of at least 2^20 small nets: every round's record and hashes equal
    the oracle's, also when stopped after a few rounds; the default rounds
    give the same."""
    t = bgpc.tuning(front=1)
    g = synth.stencil27(102)
    ref = oracle.bgpc(g)
    res, colors = _gpu_bgpc(cuda, g, log_hashes=True, tune=t)
    _compare_full(res, colors, ref)
    assert np.array_equal(res.log["hash_t"], ref.log["hash_t"])
    assert np.array_equal(res.log["hash_c"], ref.log["hash_c"])
    res, colors = _gpu_bgpc(cuda, g)
    _compare_full(res, colors, ref)
    for k in (1, 2, 7):
        refk = oracle.bgpc(g, max_rounds=k)
        res, colors = _gpu_bgpc(cuda, g, max_rounds=k, tune=t)
        _compare_full(res, colors, refk)
    r = synth.random_uniform(1100000, 1050000, 2, 8, 61)
    ref = oracle.bgpc(r)
    res, colors = _gpu_bgpc(cuda, r, tune=t)
    _compare_full(res, colors, ref)
    adj = _grid7(102)
    ref = oracle.d2gc(adj)
    res, colors = _gpu_d2(cuda, adj, tune=t)
    _compare_full(res, colors, ref)


FORCED = [dict(front=1), dict(front=0, standing=1), dict(standing=0), dict(planes=1), dict(planes=0),
          dict(color_grid=8, removal_grid=2, apply_grid=2), dict(front=1, color_grid=64, removal_grid=32)]


@pytest.mark.parametrize("forced", FORCED, ids=str)
def test_tuning_choices_keep_results(cuda, forced):
    """Every result-invariant choice, forced on graphs of every kind (front-
    driven rounds and standing proposals also on small graphs, color words on
    and off, extreme grids): colors, rounds and round log equal the oracle's."""
    t = bgpc.tuning(**forced)
    cases = [(synth.random_uniform(5003, 4001, 2, 8, 11), dict()),
             (synth.random_uniform(3000, 2500, 40, 90, 21), dict()),     # colors past 63
             (synth.stencil27(24), dict()),
             (synth.random_uniform(20481, 9000, 3, 30, 12), dict(net_color_mask=0b101)),
             (synth.skewed(30000, 30000, seed=5, kmax=3000, name="skewed30k"), dict(net_color_mask=1, policy=2))]
    for g, kw in cases:
        ref = oracle.bgpc(g, **kw)
        res, colors = _gpu_bgpc(cuda, g, tune=t, **kw)
        _compare_full(res, colors, ref)
    for adj in (_grid7(20), synth.rmat(11, 8, 0.57, 0.19, 0.19, seed=4)):
        ref = oracle.d2gc(adj)
        res, colors = _gpu_d2(cuda, adj, tune=t)
        _compare_full(res, colors, ref)


def test_autotune(cuda):
    """The autotuner returns a choice no slower than the library's own (it
    checks every candidate's colors against the default's itself); the tuned
    choice, explicit or from the shape cache, gives the oracle's colors."""
    for g, kw in ((synth.stencil27(48), dict()), (synth.random_uniform(20000, 20000, 2, 8, 1), dict()),
                  (synth.random_uniform(30000, 30000, 3, 30, 41), dict(net_color_mask=1))):
        A, B = bgpc.upload_bipartite(g)
        best, ms_default, ms_best = bgpc.autotune(A, B, trials=2, **kw)
        assert ms_best <= ms_default
        ref = oracle.bgpc(g, **kw)
        res, colors = _gpu_bgpc(cuda, g, (A, B), tune=best, **kw)
        _compare_full(res, colors, ref)
        res, colors = _gpu_bgpc(cuda, g, (A, B), **kw)   # the cached choice
        _compare_full(res, colors, ref)
    adj = _grid7(24)
    D = bgpc.upload_adjacency(adj)
    best, _, _ = bgpc.autotune(D, None, trials=1)
    res, colors = _gpu_d2(cuda, adj, D, tune=best)
    _compare_full(res, colors, oracle.d2gc(adj))
