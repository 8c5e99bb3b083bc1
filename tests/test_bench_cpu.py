"""CPU checks of the benchmark's host logic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_counts():
    ai = dict(n=10, nnz=40, nnz_l=20, nnz_u=30, updates=100)
    # per-stage byte counts: triangle values + indices, row pointers, 2 vectors; factor read,
    # pattern, factor write, update list; K values + indices, row pointers, 3 vectors
    assert bench.algorithmic_bytes("trsv_l", ai) == 20 * 12 + 11 * 4 + 10 * 16
    assert bench.algorithmic_bytes("trsv_u", ai) == 30 * 12 + 11 * 4 + 10 * 16
    assert bench.algorithmic_bytes("refactor", ai) == 50 * 20 + 100 * 4
    assert bench.algorithmic_bytes("spmv", ai) == 40 * 12 + 11 * 4 + 10 * 24
    with pytest.raises(KeyError):
        bench.algorithmic_bytes("nope", ai)


def test_percentile():
    assert bench.percentile([1, 2, 3, 4], 50) == 2.5
    assert bench.percentile([5], 99) == 5


def test_cpu_baseline_compares_solutions():
    import numpy as np
    import kkt_synth as ks
    import oracle
    p = ks.make_pattern(1)
    systems = [p.system(k) for k in (1, 2)]
    Q = oracle.order(p.rowptr, p.colidx)
    xs = [oracle.direct_solve(p.rowptr, p.colidx, v, b, Q=Q)[0] for v, b in systems]
    done, el, cmp = bench.cpu_baseline(p, systems, 0.0, gpu_xs=xs)
    assert done == 1 and el > 0 and len(cmp) == 1
    assert cmp[0][0] == 0.0 and cmp[0][1] > 1.0
    bad = [xs[0] * (1 + 1e-3), xs[1]]
    _, _, cmp = bench.cpu_baseline(p, systems[:1], 0.0, gpu_xs=bad)
    assert abs(cmp[0][0] - 1e-3) < 1e-9


def test_host_cpu_reports_cores():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["cpu_count"] >= h["nproc"]
