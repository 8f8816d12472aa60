"""CPU checks of the benchmark's bookkeeping: the algorithmic bytes per cell are the
figures the kernel design states, the roofline object follows from a profile by
the contract's arithmetic, counter traffic and VALU issue are used only for the
kernel sources they were taken on, and a multi-GPU request is refused."""

import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_per_cell():
    """The hot-path definition: residual (2 + 2/3) S + 128 B, filter 2 S + 160 B, with
    S = 4 x 6 x 8 = 192 B at P2 FP64 (640 and 544 B) and 4 x (8 + 5 x 4) = 112 B mixed;
    as stored, the kernels read 52 and 108 B of geometry."""
    b = bench.algorithmic_bytes_per_cell(2, "fp64")
    assert set(b) == {"residual", "filter"}
    assert b["residual"] == pytest.approx(640.0)
    assert b["filter"] == 544
    m = bench.algorithmic_bytes_per_cell(2, "mixed")
    assert m["residual"] == pytest.approx(112 * (2 + 2 / 3) + 128)
    assert m["filter"] == 2 * 112 + 160
    p1 = bench.algorithmic_bytes_per_cell(1, "fp64")
    assert p1["filter"] == 2 * 96 + 160
    # per DOF-stage at P2 FP64 (24 DOF per cell): 1184 B / 24 = 49.3 B
    assert sum(b.values()) / 24 == pytest.approx(1184 / 24)
    st = bench.stored_bytes_per_cell(2, "fp64")
    assert st["residual"] == pytest.approx(192 * (2 + 2 / 3) + 52) and st["filter"] == 2 * 192 + 108


def test_roofline_from_profile():
    """achieved = algorithmic bytes per launch / mean launch time of the kernel with the
    largest total time; frac against 8 TB/s."""
    n_cell = 100_000
    prof = {"residual": (50e-3 * 30, 30), "filter": (60e-3 * 30, 30)}
    roof, per_k = bench.roofline(prof, 2, n_cell, "no_such_workload", "fp64")
    assert roof["kernel"] == "filter" and roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    alg = 544 * n_cell
    assert roof["alg_bytes_per_launch"] == alg
    assert roof["achieved"] == pytest.approx(alg / 60e-6 / 1e9, rel=1e-3)
    assert roof["peak"] == 8000.0
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0, rel=1e-3)
    assert roof["traffic"] is None                  # no counters for this workload
    assert roof["as_stored"]["bytes_per_cell"] == 492
    assert set(per_k) == {"residual", "filter"}


def test_cpu_model_and_threads():
    model, usable = bench.host_cpu()
    assert isinstance(model, str) and model and usable >= 1


def test_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    rec = {"kernel_source_sha": bench.kernel_source_hash(), "fetch_factor": 2.0, "write_factor": 1.0,
           "workloads": {"w": {"filter": {"hbm_bytes_per_launch": 123, "read_bytes": 100, "write_bytes": 23}}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic("filter", "w") == 123
    assert bench.load_traffic("residual", "w") is None
    assert bench.load_valu("filter", "w") is None    # no VALU counters in this record
    rec["workloads"]["w"]["filter"]["valu"] = {"insts_per_launch": 7, "busy_frac": 0.5, "clock_ghz": 2.1}
    f.write_text(json.dumps(rec))
    assert bench.load_valu("filter", "w") == {"insts_per_launch": 7, "busy_frac": 0.5, "clock_ghz": 2.1}
    prof = {"residual": (0.05, 1), "filter": (0.06, 1)}
    roof, _ = bench.roofline(prof, 2, 1000, "w", "fp64")
    assert roof["traffic"] == 123 and roof["valu"]["busy_frac"] == 0.5
    rec["kernel_source_sha"] = "0" * 16              # counters of other kernel sources
    f.write_text(json.dumps(rec))
    assert bench.load_traffic("filter", "w") is None
    assert bench.load_valu("filter", "w") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
