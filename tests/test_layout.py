"""Host-side checks: the ctypes mirrors of the C structs match the header's
layout (compiled with the host C compiler), and the benchmark refuses a GPU
count it does not measure."""
import ctypes
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _c_layout(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "bh.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(bh_stats), sizeof(bh_options),\n'
        "         offsetof(bh_stats, t_particle_ms), offsetof(bh_stats, n_neighbor_calls),\n"
        "         offsetof(bh_stats, neighbor_tests), offsetof(bh_options, quadrupole),\n"
        "         offsetof(bh_options, curve), offsetof(bh_options, list_tile), offsetof(bh_stats, n_theta_fallback));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


def test_ctypes_structs_match_header(tmp_path):
    from paper_0909_0541_amd import bh
    size_s, size_o, off_tp, off_nc, off_nt, off_q, off_c, off_lt, off_tf = _c_layout(tmp_path)
    assert ctypes.sizeof(bh._Stats) == size_s
    assert ctypes.sizeof(bh._Options) == size_o
    assert bh._Stats.t_particle_ms.offset == off_tp
    assert bh._Stats.n_neighbor_calls.offset == off_nc
    assert bh._Stats.neighbor_tests.offset == off_nt
    assert bh._Options.quadrupole.offset == off_q
    assert bh._Options.curve.offset == off_c
    assert bh._Options.list_tile.offset == off_lt
    assert bh._Stats.n_theta_fallback.offset == off_tf
    # the Stats record lists every field of the C struct, in order
    assert [f for f, _ in bh._Stats._fields_] == list(bh.Stats.__dataclass_fields__)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
