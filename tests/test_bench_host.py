"""CPU: the host-side logic of bench.py (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

OPTS = {"texture_format": 2, "points_per_thread": 16, "tile_order": 1, "persistent": 2,
        "record_order": 1, "resort_interval": 8}


def test_counters_are_used_only_for_the_measured_kernel(tmp_path, monkeypatch):
    """The committed counter summary feeds the bench line only while it was
    taken on the current kernel source, workload, schedule and size."""
    rec = {"kernel_hash": bench.kernel_source_hash(), "workload": "c4", "options": OPTS,
           "n_residuals": 1000, "hbm_bytes_per_launch": 123.0,
           "l2_read_requests_per_launch": 7.0, "l2_hit_rate": 0.5, "l2_channel_busy": 0.9}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"records": [rec]}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_counters("c4", OPTS, 1000)["hbm_bytes_per_launch"] == 123.0
    assert bench.measured_counters("c3", OPTS, 1000) is None
    assert bench.measured_counters("c4", dict(OPTS, points_per_thread=8), 1000) is None
    assert bench.measured_counters("c4", OPTS, 999) is None
    f.write_text(json.dumps({"records": [dict(rec, kernel_hash="0" * 16)]}))
    assert bench.measured_counters("c4", OPTS, 1000) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_counters("c4", OPTS, 1000) is None


def test_committed_counter_summary_is_well_formed():
    recs = bench.load_counter_records()
    assert recs
    for rec in recs:
        for k in ("kernel_hash", "workload", "options", "n_residuals", "hbm_bytes_per_launch",
                  "fetch_scale", "write_scale", "l2_hit_rate", "valu_insts_per_launch",
                  "l2_read_requests_per_launch"):
            assert k in rec, k
        assert 0 < rec["hbm_bytes_per_launch"] < 24 * rec["n_residuals"] * 4
        assert 1.9 < rec["fetch_scale"] < 2.1 and 0.9 < rec["write_scale"] < 1.1
    # one record per workload and schedule
    keys = [(r["workload"], json.dumps(r["options"], sort_keys=True)) for r in recs]
    assert len(keys) == len(set(keys))


def _pmc_csv(path, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    head = '"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n'
    path.write_text(head + "".join(f'{d},"{k}","{c}",{v}\n' for d, k, c, v in rows))


def test_counter_summary_from_rocprof_runs(tmp_path, monkeypatch):
    """summarize_counters averages each counter over the fused kernel's
    dispatches (other kernels ignored), scales the byte counters by the
    calibration copy and keeps one record per workload and schedule."""
    kern = "void epo::fused::" + bench.KERNEL_NAME + "(args)"
    other = "void epo::pair_setup_kernel(args)"
    copy = "__amd_rocclr_copyBuffer"
    vals = {"FETCH_SIZE": 1000.0, "WRITE_SIZE": 10.0, "TCC_HIT_sum": 80.0, "TCC_MISS_sum": 20.0,
            "TCC_REQ_sum": 100.0, "TCC_BUSY_sum": 128.0 * 90, "GRBM_GUI_ACTIVE": 800.0,
            "SQ_INSTS_VALU": 5e6, "TCP_TCC_READ_REQ_sum": 64.0,
            "TCP_TCC_READ_REQ_LATENCY_sum": 6400.0, "TA_TA_BUSY_sum": 256 * 50.0,
            "TD_TD_BUSY_sum": 256 * 60.0, "TD_TC_STALL_sum": 256 * 30.0,
            "TCP_PENDING_STALL_CYCLES_sum": 256 * 20.0}
    for d, names in bench.COUNTER_PASSES.items():
        rows = []
        for disp in (3, 7):
            for c in names.split():
                # the two dispatches differ by +-10 %: the record holds the mean
                rows.append((disp, kern, c, vals.get(c, 1.0) * (0.9 if disp == 3 else 1.1)))
                rows.append((disp + 1, other, c, 1e9))
        _pmc_csv(tmp_path / d / "x" / "run_counter_collection.csv", rows)
    half = bench.CALIBRATION_BYTES / 1024 / 2
    _pmc_csv(tmp_path / "copy_fetch" / "run_counter_collection.csv", [(1, copy, "FETCH_SIZE", half)])
    _pmc_csv(tmp_path / "copy_write" / "run_counter_collection.csv",
             [(1, copy, "WRITE_SIZE", 2 * half)])
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"records": [{"workload": "c1", "options": OPTS, "stale": True},
                                         {"workload": "c2", "options": OPTS}]}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    bench.summarize_counters(str(tmp_path), "c1", OPTS, bench.KERNEL_NAME)
    recs = json.loads(f.read_text())["records"]
    assert [r["workload"] for r in recs] == ["c2", "c1"] and "stale" not in recs[1]
    r = recs[1]
    assert abs(r["fetch_scale"] - 2.0) < 1e-12 and abs(r["write_scale"] - 1.0) < 1e-12
    assert abs(r["hbm_read_bytes_per_launch"] - 1000.0 * 1024 * 2) < 1e-6
    assert abs(r["hbm_write_bytes_per_launch"] - 10.0 * 1024) < 1e-6
    assert abs(r["l2_hit_rate"] - 0.8) < 1e-12
    assert abs(r["valu_insts_per_launch"] - 5e6) < 1e-3
    assert abs(r["l2_read_latency_cycles"] - 100.0) < 1e-9
    assert abs(r["l2_channel_busy"] - 90.0 / 100.0) < 1e-12
    assert r["dispatches"]["fetch"] == 2
    assert bench.measured_counters("c1", OPTS, r["n_residuals"]) == r


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_hash_covers_only_the_fused_kernels_device_code(tmp_path, monkeypatch):
    """Host-side edits (the launch code, the plan structure) and comment edits
    keep the committed counters valid; edits of the kernel's device code or of
    the data layout it reads invalidate them."""
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

    edit("edge_cost.hip", "namespace epo {", "namespace epo {\nconstexpr int kHostOnly = 1;")
    edit("epo_internal.h", "struct Plan {", "struct PlanNote {};\nstruct Plan {")
    # comments and layout inside the hashed files do not count either
    edit("epo_internal.h", "struct Tile {", "// layout note\nstruct Tile {")
    edit("fused_kernel.h", "namespace fused {", "namespace fused {\n/* kernel\n   note */  ")
    assert bench.kernel_source_hash() == h0
    edit("epo_internal.h", "struct Tile {", "struct TileNote {};\nstruct Tile {")
    h1 = bench.kernel_source_hash()
    assert h1 != h0
    edit("fused_kernel.h", "namespace fused {", "namespace fused {\nconstexpr int kNote = 1;")
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


@pytest.mark.parametrize("steps,warmup,want", [(20, 20, 10), (20, 21, 1), (5, 1, 1), (30, 20, 10),
                                               (12, 8, 4), (7, 14, 7), (1, 0, 1), (100, 50, 10)])
def test_graph_steps_divide_timed_and_warmup_steps(steps, warmup, want):
    """The bench runs steps / g timed and warmup / g warm-up graph launches of
    g iterations each: g divides both counts, at most 10."""
    g = bench.graph_steps_for(steps, warmup)
    assert g == want
    assert steps % g == 0 and warmup % g == 0 and 1 <= g <= 10
