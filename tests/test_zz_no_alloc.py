"""The allocation-free entry point (bgpc_color_noalloc) against bgpc_color:
same colors, rounds and round log, on two calls in a row on one GPU (the
second on a smaller graph, so the static workspace holds the first call's
leftovers), under several schedules; sizes past its limits are refused."""
import numpy as np
import pytest

from paper_1701_02628_amd import bgpc, synth

pytestmark = pytest.mark.gpu

CASES = [("V-V", dict()), ("N1", dict(net_color_mask=1)), ("B2", dict(policy=2, chunk=9)),
         ("V-then-N", dict(net_color_mask=0b10)), ("strict-B1G", dict(policy=3, flags=1)),
         ("alg6-vertex-removal", dict(net_color_mask=1, net_alg=1, net_conflict_mask=0))]


def _pair(cuda, g, kw):
    import torch
    A, B = bgpc.upload_bipartite(g)
    o1 = torch.full((g.n_a,), -7, dtype=torch.int32, device=cuda)
    o2 = torch.full((g.n_a,), -7, dtype=torch.int32, device=cuda)
    r1 = bgpc.bgpc_color(A, B, None, o1, log_cap=4096, **kw)
    r2 = bgpc.bgpc_color_noalloc(A, B, o2, log_cap=4096, **kw)
    torch.cuda.synchronize()
    return r1, o1.cpu().numpy(), r2, o2.cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_noalloc_equals_bgpc_color_twice(cuda, case):
    big = synth.random_uniform(120000, 110000, 3, 30, 91)
    small = synth.random_uniform(5003, 4001, 2, 8, 11)
    for g in (big, small):
        r1, c1, r2, c2 = _pair(cuda, g, case[1])
        assert r2.status == r1.status == 0, (r1.status, r2.status)
        assert r2.rounds == r1.rounds
        assert np.array_equal(c1, c2)
        for k in ("mode", "w", "losers", "evicted", "max_color"):
            assert np.array_equal(r1.log[k], r2.log[k]), k


def test_noalloc_colors_past_63_and_stencil(cuda):
    for g in (synth.random_uniform(3000, 2500, 40, 90, 21), synth.stencil27(40), synth.random_uniform(900, 800, 2, 5, 3)):
        r1, c1, r2, c2 = _pair(cuda, g, {})
        assert r2.status == r1.status == 0 and r2.rounds == r1.rounds and np.array_equal(c1, c2)


def test_noalloc_refuses_past_its_limits(cuda):
    import torch
    g = synth.random_uniform(1100000, 1000, 1, 2, 5)    # more vertices than the limit
    A, B = bgpc.upload_bipartite(g)
    out = torch.empty(g.n_a, dtype=torch.int32, device=cuda)
    assert bgpc.bgpc_color_noalloc(A, B, out).status == bgpc.E_UNSUPPORTED
    small = synth.random_uniform(500, 400, 2, 6, 1)
    A, B = bgpc.upload_bipartite(small)
    out = torch.empty(small.n_a, dtype=torch.int32, device=cuda)
    assert bgpc.bgpc_color_noalloc(A, B, out, flags=4).status == bgpc.E_UNSUPPORTED   # incremental rounds
