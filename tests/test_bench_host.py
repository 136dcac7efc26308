"""CPU: the host-side logic of bench.py (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

OPTS = {"texture_format": 2, "points_per_thread": 16, "tile_order": 1, "persistent": 2}


def test_counters_are_used_only_for_the_measured_kernel(tmp_path, monkeypatch):
    """The committed counter summary feeds the bench line only while it was
    taken on the current kernel source, workload, schedule and size."""
    rec = {"kernel_hash": bench.kernel_source_hash(), "workload": "c4", "options": OPTS,
           "n_residuals": 1000, "hbm_bytes_per_launch": 123.0,
           "l2_read_requests_per_launch": 7.0, "l2_hit_rate": 0.5, "l2_channel_busy": 0.9}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_counters("c4", OPTS, 1000)["hbm_bytes_per_launch"] == 123.0
    assert bench.measured_counters("c3", OPTS, 1000) is None
    assert bench.measured_counters("c4", dict(OPTS, points_per_thread=8), 1000) is None
    assert bench.measured_counters("c4", OPTS, 999) is None
    f.write_text(json.dumps(dict(rec, kernel_hash="0" * 16)))
    assert bench.measured_counters("c4", OPTS, 1000) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_counters("c4", OPTS, 1000) is None


def test_committed_counter_summary_is_well_formed():
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    for k in ("kernel_hash", "workload", "options", "n_residuals", "hbm_bytes_per_launch",
              "fetch_scale", "write_scale", "l2_hit_rate"):
        assert k in rec, k
    assert 0 < rec["hbm_bytes_per_launch"] < 24 * rec["n_residuals"] * 4
    assert 1.9 < rec["fetch_scale"] < 2.1 and 0.9 < rec["write_scale"] < 1.1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_hash_covers_only_the_fused_kernels_device_code(tmp_path, monkeypatch):
    """Host-side edits (the launch code, the plan structure) keep the committed
    counters valid; edits of the kernel's device code or of the data layout it
    reads invalidate them."""
    import shutil
    src = os.path.join(ROOT, "paper_2607_00579_amd", "csrc")
    dst = tmp_path / "paper_2607_00579_amd" / "csrc"
    shutil.copytree(src, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()

    def edit(name, old, new):
        p = dst / name
        text = p.read_text()
        assert old in text
        p.write_text(text.replace(old, new, 1))

    edit("edge_cost.hip", "namespace epo {", "namespace epo {\n// host-side note")
    edit("epo_internal.h", "struct Plan {", "// plan note\nstruct Plan {")
    assert bench.kernel_source_hash() == h0
    edit("epo_internal.h", "struct Tile {", "// layout note\nstruct Tile {")
    h1 = bench.kernel_source_hash()
    assert h1 != h0
    edit("fused_kernel.h", "namespace fused {", "namespace fused {\n// kernel note")
    assert bench.kernel_source_hash() not in (h0, h1)


def test_cpu_baseline_reports_the_host(monkeypatch):
    """The oracle baseline on the host's cores: a positive rate, the worker
    count as cores, and the host description (core count, CPU model, NumPy)."""
    from synth import make
    r = bench.cpu_baseline(make("c1"), budget_s=0.5)
    assert r["kind"] == "oracle" and r["value"] > 0
    assert 1 <= r["cores"] <= 16
    for k in ("nproc", "affinity", "cpu_model", "numpy"):
        assert r["host"][k], k
    assert "directed pairs" in r["sample"]
