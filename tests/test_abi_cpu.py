"""The C ABI library loads on the CPU and exports every entry point that
include/bgpc.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re
import subprocess

from paper_1701_02628_amd import bgpc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    with open(os.path.join(ROOT, "include", "bgpc.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"BGPC_API\s+[\w\s\*]+?\b(\w+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_entry_points()
    for must in ("bgpc_color", "d2gc_color", "color_stats", "bgpc_status_string", "bgpc_opts_default"):
        assert must in names, names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(bgpc.LIB_PATH)
    for name in declared_entry_points():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", bgpc.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(declared_entry_points()) <= exported


def test_binding_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the sizes and field offsets gcc gives the C structs."""
    src = tmp_path / "layout.c"
    src.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "bgpc.h"
int main(void) {
  printf("csr %zu %zu %zu\n", sizeof(bgpc_csr), offsetof(bgpc_csr, nnz), offsetof(bgpc_csr, indices));
  printf("log %zu %zu %zu\n", sizeof(bgpc_round_log), offsetof(bgpc_round_log, max_color),
         offsetof(bgpc_round_log, round_ms));
  printf("prof %zu %zu %zu\n", sizeof(bgpc_profile), offsetof(bgpc_profile, bytes), offsetof(bgpc_profile, bytes_scanned));
  printf("opts %zu %zu %zu %zu %zu %zu\n", sizeof(bgpc_opts), offsetof(bgpc_opts, stream), offsetof(bgpc_opts, log),
         offsetof(bgpc_opts, prof), offsetof(bgpc_opts, net_conflict_mask), offsetof(bgpc_opts, net_alg));
  printf("item %zu %zu %zu %zu\n", sizeof(bgpc_batch_item), offsetof(bgpc_batch_item, order),
         offsetof(bgpc_batch_item, d2gc), offsetof(bgpc_batch_item, route));
  printf("stats %zu %zu\n", sizeof(bgpc_stats), offsetof(bgpc_stats, card_std));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        k, *vals = line.split()
        got[k] = [int(v) for v in vals]
    assert got["csr"] == [ctypes.sizeof(bgpc.Csr), bgpc.Csr.nnz.offset, bgpc.Csr.indices.offset]
    assert got["log"] == [ctypes.sizeof(bgpc.RoundLog), bgpc.RoundLog.max_color.offset,
                          bgpc.RoundLog.round_ms.offset]
    assert got["prof"] == [ctypes.sizeof(bgpc.Profile), bgpc.Profile.bytes.offset, bgpc.Profile.bytes_scanned.offset]
    assert got["opts"] == [ctypes.sizeof(bgpc.Opts), bgpc.Opts.stream.offset, bgpc.Opts.log.offset,
                           bgpc.Opts.prof.offset, bgpc.Opts.net_conflict_mask.offset, bgpc.Opts.net_alg.offset]
    assert got["item"] == [ctypes.sizeof(bgpc.BatchItem), bgpc.BatchItem.order.offset, bgpc.BatchItem.d2gc.offset,
                           bgpc.BatchItem.route.offset]
    assert got["stats"] == [ctypes.sizeof(bgpc.Stats), bgpc.Stats.card_std.offset]


def test_status_strings_and_defaults():
    lib = bgpc.load()
    assert bgpc.status_string(0) == "ok"
    assert "max_rounds" in bgpc.status_string(-6)
    o = bgpc.Opts()
    lib.bgpc_opts_default(ctypes.byref(o))
    assert o.policy == 0 and o.chunk == 64 and o.net_color_mask == 0 and o.flags == 0
    assert o.net_conflict_mask == 2 ** 64 - 1 and o.net_alg == 0
