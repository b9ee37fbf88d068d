"""Host-side logic of bench.py (no GPU): the one-GPU contract, the counter
summary reader and the CPU-baseline record."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def _summary(tmp_path, sha, cells=4194304, traffic=123456789):
    p = tmp_path / "pmc.txt"
    p.write_text(f"header line\ncells: {cells}\ntraffic_bytes_per_launch: {traffic}\n"
                 f"source_sha256: {sha}\n")
    return str(p)


def test_traffic_is_read_only_for_the_current_sources(tmp_path, monkeypatch):
    sha = bench.stage_source_hash()
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, sha))
    assert bench.read_traffic(4194304) == 123456789.0
    assert bench.read_traffic(65536) is None  # counters of another workload
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, "0" * 64))
    assert bench.read_traffic(4194304) is None  # kernel sources changed since
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.read_traffic(4194304) is None


def test_cpu_baseline_record():
    from workloads import make_workload
    w = make_workload("shell32")
    rec = bench.cpu_baseline(w, 50.0, budget_s=0.0, max_steps=1)
    assert rec["kind"] == "oracle" and rec["cores"] == 1
    assert rec["unit"] == "cell-stage updates/s" and rec["value"] > 0
    assert "shell32" in rec["sample"] and "s=14" in rec["sample"]


@pytest.mark.parametrize("flag", ["--steps", "--warmup", "--march-steps"])
def test_arguments_parse(flag, monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", flag, "3"])
    a = bench.parse()
    assert getattr(a, flag.lstrip("-").replace("-", "_")) == 3 and a.gpus == 1


def test_cpu_baseline_slab_sample():
    """Large grids are sampled by their innermost r-planes."""
    from workloads import make_workload
    w = make_workload("shell32")
    rec = bench.cpu_baseline(w, 50.0, budget_s=0.0, max_steps=1, max_cells=8 * 32 * 64)
    assert rec["value"] > 0
    assert "the 8 innermost r-planes (8x32x64 = 16384 cells) of shell32" in rec["sample"]


def test_median():
    assert bench.median([3.0, 1.0, 2.0]) == 2.0
    assert bench.median([4.0, 1.0, 3.0, 2.0]) == 2.5


def test_host_fields_pool_equals_in_process():
    """The training fields of the learned guess are the same whether a pool
    of fresh processes or this process generates them."""
    from paper_1610_01265_amd import learned
    a = learned.host_fields((4, 6, 8), range(5), workers=2)
    b = learned.host_fields((4, 6, 8), range(5), workers=1)
    assert [s for s, _ in a] == list(range(5))
    assert all(sa == sb and (ta == tb).all() for (sa, ta), (sb, tb) in zip(a, b))
