"""Host logic of bench.py (no GPU): the one-GPU refusal and the calibrated
counter arithmetic behind the bench line's HBM fractions."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_calibrated_traffic_arithmetic():
    """A copy of 256 MiB read as 128 MiB by FETCH_SIZE (the counter sees half
    the bytes read) and 256 MiB by WRITE_SIZE gives factors 2 and 1; round 0
    runs from the first coloring launch through the first compaction."""
    kib = 1024.0
    fetch = [("__amd_rocclr_copyBuffer", 128 * kib),
             ("bgpc::k_fill_i32(int*, int, long)", 1.0),
             ("void bgpc::k_vcolor_ff<false, false>(bgpc::Graph, ...)", 10.0),
             ("void bgpc::k_conflict_small<false, true, true, false>(bgpc::Graph, ...)", 20.0),
             ("void bgpc::k_apply<false>(bgpc::Graph, ...)", 3.0),
             ("void bgpc::k_compact<false>(int const*, ...)", 1.0),
             ("void bgpc::k_vcolor_ff<false, false>(bgpc::Graph, ...)", 6.0),
             ("void bgpc::k_conflict_small<false, true, true, false>(bgpc::Graph, ...)", 12.0),
             ("void bgpc::k_apply<false>(bgpc::Graph, ...)", 1.0),
             ("void bgpc::k_compact<false>(int const*, ...)", 1.0),
             ("at::native::some_torch_kernel", 99.0)]
    write = [(n, v / 2.0) for n, v in fetch]
    write[0] = (fetch[0][0], 256 * kib)
    f_read, f_write, kernels, round0 = bench.calibrated_traffic(fetch, write)
    assert f_read == pytest.approx(2.0)
    assert f_write == pytest.approx(1.0)
    assert set(kernels) == {"k_fill_i32", "k_vcolor_ff", "k_conflict_small", "k_apply", "k_compact"}
    assert kernels["k_vcolor_ff"]["launches_per_call"] == 2
    # bytes = 1024 * (fetch * 2 + write * 1) = 1024 * 2.5 * fetch
    assert kernels["k_vcolor_ff"]["bytes_per_launch"] == pytest.approx(1024 * 2.5 * (10 + 6) / 2)
    assert kernels["k_conflict_small"]["bytes_per_launch"] == pytest.approx(1024 * 2.5 * 16)
    assert round0 == pytest.approx(1024 * 2.5 * (10 + 20 + 3 + 1))


def test_calibrated_traffic_needs_the_copy():
    rows = [("void bgpc::k_apply<false>(bgpc::Graph, ...)", 1.0)]
    with pytest.raises(SystemExit):
        bench.calibrated_traffic(rows, rows)
