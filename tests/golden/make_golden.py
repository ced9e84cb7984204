"""Writes tests/golden/workloads.json: oracle results on the full-size workloads.

Calls only the CPU oracle (oracle/) and the input generators; nothing here
comes from the HIP library.  Each entry stores the SHA-256 of the generated
input arrays (to catch generator drift), the rounds, the per-round worklist
sizes and the SHA-256 of the int32 colors.  Slow (the skewed and R-MAT
workloads take many minutes on 8 cores), so entries can be (re)made one
group at a time:

    python tests/golden/make_golden.py stencil skewed rmat batch
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1701_02628_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "workloads.json")
BATCH_SAMPLE = list(range(0, 4096, 128)) + [5, 7, 8]


def batch_large_sample(k: int = 24) -> list:
    """k graphs of the batched workload spread over the sizes above 1.2e6
    expected memberships (n_B times the mean net size 16.5) with more than
    20,000 vertices, chosen from the generator's sizes alone: large sparse
    graphs, the ones one workgroup would take longest on."""
    sizes = np.array([synth.batch_sizes(i) for i in range(4096)])
    na, nb = sizes[:, 0], sizes[:, 1]
    big = np.nonzero((nb * 16.5 > 1.2e6) & (na > 20000))[0]
    by_size = big[np.argsort(nb[big], kind="stable")]
    return sorted(int(i) for i in by_size[np.linspace(0, len(by_size) - 1, k).astype(int)])


def colors_sha(colors) -> str:
    return hashlib.sha256(np.ascontiguousarray(colors, dtype=np.int32).tobytes()).hexdigest()


def entry(g_digest, r, colors_extra=None):
    e = {"input_sha256": g_digest, "status": r.status, "rounds": r.rounds, "w": [int(x) for x in r.log["w"]],
         "colors_sha256": colors_sha(r.colors), "n_distinct": int(len(np.unique(r.colors))),
         "max_color": int(r.colors.max()) if r.colors.size else -1}
    if colors_extra:
        e.update(colors_extra)
    return e


def make(groups):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    if "random20k" in groups:
        g = synth.config(0)
        d = g.digest()
        data["random20k"] = {"vv": entry(d, oracle.bgpc(g)), "n1": entry(d, oracle.bgpc(g, net_color_mask=1))}
    if "stencil" in groups:
        g = synth.config(1)
        d = g.digest()
        out = {}
        # mask 0b1 is the paper's N1-N2 (net-based coloring in the first
        # round), 0b11 its N2-N2 (the first two rounds)
        for name, mask in (("vv", 0), ("n1", 0b1), ("v_then_n", 0b10), ("n2n2", 0b11)):
            t = time.time()
            out[name] = entry(d, oracle.bgpc(g, net_color_mask=mask))
            print("stencil", name, out[name]["rounds"], f"{time.time() - t:.1f}s", flush=True)
        out["seq_greedy_colors"] = int(len(np.unique(oracle.seq_greedy(g))))
        data["stencil128"] = out
    if "skewed" in groups:
        g = synth.config(2)
        d = g.digest()
        out = {}
        for name, pol in (("n1_ff", 0), ("n1_b1", 1), ("n1_b2", 2)):
            t = time.time()
            r = oracle.bgpc(g, net_color_mask=1, policy=pol)
            out[name] = entry(d, r, {"stats": oracle.color_stats(r.colors)})
            print("skewed", name, r.rounds, f"{time.time() - t:.1f}s", flush=True)
        data.setdefault("skewed4m", {}).update(out)
    if "skewed_b1g" in groups:
        # B1 with one col_max per round (policy 3), net-based first round
        g = synth.config(2)
        t = time.time()
        r = oracle.bgpc(g, net_color_mask=1, policy=3)
        data.setdefault("skewed4m", {})["n1_b1g"] = entry(g.digest(), r, {"stats": oracle.color_stats(r.colors)})
        print("skewed n1_b1g", r.rounds, f"{time.time() - t:.1f}s", flush=True)
    if "rmat" in groups:
        a = synth.config(3)
        d = a.digest()
        t = time.time()
        r = oracle.d2gc(a, net_color_mask=1)
        data["rmat22_d2"] = {"n1": entry(d, r), "max_degree": int(np.diff(a.off).max())}
        print("rmat", r.rounds, f"{time.time() - t:.1f}s", flush=True)
    if "batch" in groups:
        out = {}
        for i in BATCH_SAMPLE:
            g = synth.batch_graph(i)
            t = time.time()
            out[str(i)] = entry(g.digest(), oracle.bgpc(g))
            print("batch", i, out[str(i)]["rounds"], f"{time.time() - t:.1f}s", flush=True)
        data["batch4096_sample"] = out
    if "batch_large" in groups:
        out = data.setdefault("batch4096_sample", {})
        for i in batch_large_sample():
            if str(i) in out:
                continue
            g = synth.batch_graph(i)
            t = time.time()
            out[str(i)] = entry(g.digest(), oracle.bgpc(g))
            print("batch", i, out[str(i)]["rounds"], f"{time.time() - t:.1f}s", flush=True)
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    make(sys.argv[1:] or ["random20k", "stencil", "skewed", "skewed_b1g", "rmat", "batch", "batch_large"])
