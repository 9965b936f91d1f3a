"""The measurement helpers of bench.py (CPU only): the copy-calibrated HBM
traffic summary behind the roofline's `traffic` field, its guard against a
changed sweep source, and the host description of the CPU baseline."""
import csv
import hashlib
import json
import os
import shutil

import bench

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
SWEEP = "void (anonymous namespace)::k_sweep<float, false, 0>((anonymous namespace)::SweepArgs, float const*)"
OTHER = "void (anonymous namespace)::k_sweep<float, false, 1>((anonymous namespace)::SweepArgs, float const*)"


def _csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_summary_scales_by_the_copy_calibration(tmp_path):
    copy_bytes = 1 << 28
    # the copy reads half its bytes under FETCH_SIZE (factor 2) and all of
    # them under WRITE_SIZE (factor 1); the sweep's medians are 800 and 1100
    # KiB, the evaluation-mode sweep and the outlier must not enter them
    _csv(tmp_path / "cf.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 131072.0)] * 3)
    _csv(tmp_path / "cw.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 262144.0)] * 3)
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(SWEEP, 790.0), (SWEEP, 800.0), (SWEEP, 5000.0), (OTHER, 1e9)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(SWEEP, 1100.0), (SWEEP, 1090.0), (SWEEP, 1200.0), (OTHER, 1e9)])
    out = tmp_path / "t.json"
    bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                             str(tmp_path / "cw.csv"), str(out), copy_bytes, "cmd", "w")
    rec = json.load(open(out))
    assert rec["copy_calibration"]["fetch_factor"] == 2.0 and rec["copy_calibration"]["write_factor"] == 1.0
    assert rec["dispatches"] == [3, 3]
    assert rec["fetch_bytes"] == 800 * 2 * 1024 and rec["write_bytes"] == 1100 * 1024
    assert rec["bytes_per_launch"] == rec["fetch_bytes"] + rec["write_bytes"]
    assert len(rec["dual_hip_sha256"]) == 64


def test_traffic_field_follows_the_profiled_source(tmp_path, monkeypatch):
    # a tree whose traffic summary was taken on its own sweep source gives the
    # stored figure; once the source changes the counters no longer describe it
    (tmp_path / "profiles").mkdir()
    src_dir = tmp_path / "paper_2310_08230_amd" / "csrc"
    src_dir.mkdir(parents=True)
    shutil.copy(os.path.join(bench.ROOT, "paper_2310_08230_amd", "csrc", "dual.hip"), src_dir)
    sha = hashlib.sha256(open(src_dir / "dual.hip", "rb").read()).hexdigest()
    rec = {"bytes_per_launch": 28401200, "dual_hip_sha256": sha}
    with open(tmp_path / "profiles" / "sweep_plain_fp32_500_hbm_traffic.json", "w") as f:
        json.dump(rec, f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench._traffic() == 28401200
    with open(src_dir / "dual.hip", "a") as f:
        f.write("\n// changed\n")
    assert bench._traffic() is None


def test_host_cpu_names_model_and_cores():
    h = bench.host_cpu()
    assert isinstance(h["cpu_model"], str) and h["cpu_model"]
    assert h["cores_available"] >= 1


SOFT = "void (anonymous namespace)::k_sweep<float, true, 0, 0>((anonymous namespace)::SweepArgs, float const*)"
SOFT_BOUND = "void (anonymous namespace)::k_sweep<float, true, 2, 0>((anonymous namespace)::SweepArgs, float const*)"


def test_valu_summary_takes_the_smoothed_update_sweep(tmp_path):
    # medians per dispatch of the smoothed update sweep only: the hard sweep
    # and the smoothed bound-only launch must not enter them
    path = tmp_path / "c.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        rows = [(SOFT, "SQ_INSTS_VALU", v) for v in (70.0e6, 71.0e6, 90.0e6)]
        rows += [(SOFT, "SQ_INSTS_VALU_TRANS_F32", v) for v in (4.1e6, 4.2e6, 4.3e6)]
        rows += [(SOFT, "SQ_WAVES", 68800.0)] * 3
        rows += [(SWEEP, "SQ_INSTS_VALU", 1e9), (SOFT_BOUND, "SQ_INSTS_VALU", 1e9)]
        for i, (name, counter, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})
    out = tmp_path / "v.json"
    bench.summarize_valu(str(path), str(out), "w", "cmd")
    rec = json.load(open(out))
    assert rec["dispatches"] == 3
    assert rec["valu_insts_per_launch"] == 71.0e6 and rec["trans_insts_per_launch"] == 4.2e6
    assert rec["waves_per_launch"] == 68800.0
    assert abs(rec["valu_issue_peak_G_per_s"] - 614.4) < 1e-9
    assert len(rec["dual_hip_sha256"]) == 64


def test_committed_valu_summary_matches_the_sweep_source():
    # the smoothed entry's roofline is reported only while the summary
    # describes the current source; the committed one must
    rec = bench._smoothed_valu()
    assert rec is not None and rec["valu_insts_per_launch"] > 0


def test_committed_traffic_summaries_match_the_sweep_source():
    # every per-pair traffic figure the bench line can carry comes from a
    # summary taken on the current sweep source
    for name in bench.TRAFFIC_PROFILES.values():
        assert bench._traffic(name) > 0, name
