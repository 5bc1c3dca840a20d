"""Host-side behaviour of bench.py that needs no GPU: the refusal of more
than one GPU, the timing statistics, the algorithmic byte counts, and the
trace summariser on a small synthetic trace database."""
from __future__ import annotations

import os
import sqlite3
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
    assert r.stdout == ""


def test_stats_and_algorithmic_bytes():
    s = bench.stats([5.0, 1.0, 3.0, 2.0, 4.0])
    assert s == {"median_ms": 3.0, "min_ms": 1.0, "p90_ms": 5.0, "calls": 5}
    n, k = 1 << 30, 56308200
    assert bench.algorithmic_bytes("k_local", n, k) == 4 * n
    assert bench.algorithmic_bytes("k_write", n, k) == 4 * n + 8 * k
    assert bench.algorithmic_bytes("k_merge", n, k) == 0


def test_trace_summary_sections(tmp_path, monkeypatch):
    """Kernels in dispatch order: labelling, then the I == I0 labelling and
    the decision, then the droplet statistics, then anything else."""
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start int, end int, grid_x int, workgroup_x int)")
    seq = [("hk::k_local<3>(hk::Geo)", 100), ("hk::k_write(hk::Geo)", 50),
           ("void hk::k_local<1>(hk::Geo)", 10), ("hk::(anonymous namespace)::k_cls_count<true>(x)", 5),
           ("hk::(anonymous namespace)::k_cls_decide(x)", 1),
           ("hk::k_local<3>(hk::Geo)", 20), ("hk::(anonymous namespace)::k_ds_stats(x)", 2),
           ("hk::k_local<3>(hk::Geo)", 7)]
    t = 0
    for name, dur in seq:
        con.execute("insert into kernels values (?, ?, ?, ?, ?)", (name, t, t + dur * 1000, 512, 256))
        t += dur * 1000 + 10
    con.commit()
    con.close()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    bench.summarize_trace(str(db))
    label = (tmp_path / "profiles" / "kernel_trace_hk_label_percolation1024.txt").read_text()
    cls = (tmp_path / "profiles" / "kernel_trace_hk_classify_capsules512.txt").read_text()
    drop = (tmp_path / "profiles" / "kernel_trace_hk_droplet_stats_droplets512.txt").read_text()
    assert "hk::k_local<3>" in label and "k_cls" not in label and "k_local<1>" not in label
    assert "k_cls_count<true>" in cls and "k_cls_decide" in cls and "k_local<1>" in cls
    assert "k_ds_stats" in drop and "k_local<3>" in drop and "k_cls" not in drop
    # the dispatch after the droplet statistics belongs to no section
    assert " 20.0 " in drop and " 7.0 " not in drop
