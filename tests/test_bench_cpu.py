"""Host-side rules of bench.py: the counted HBM traffic is reported only while the committed
counter record matches the kernel source and the tile schedules it was taken with, and a
run asked for more than one GPU stops with a message."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

REC = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def _record():
    return json.load(open(REC))


def test_traffic_of_the_recorded_schedules():
    rec = _record()
    tuning = dict(rec["tuning"])
    expect = sum(mb for k, mb in rec["hbm_MB_per_launch"].items() if k.startswith("k_freq_bwd<"))
    assert expect > 0
    assert bench.hbm_traffic("freq_bwd", tuning) == round(expect * 1e6)


def test_traffic_is_null_for_other_backward_schedules():
    tuning = dict(_record()["tuning"])
    tuning["bwd_rows_k"] = [v * 2 for v in tuning["bwd_rows_k"]]
    assert bench.hbm_traffic("freq_bwd", tuning) is None
    # the forward's figure does not depend on the backward's schedules
    assert bench.hbm_traffic("freq_fwd", tuning) is not None


def test_traffic_is_null_once_the_kernel_source_changed(tmp_path, monkeypatch):
    rec = _record()
    (tmp_path / "profiles").mkdir()
    src = tmp_path / rec["source"]
    src.parent.mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, rec["source"]), src)
    shutil.copy(REC, tmp_path / "profiles" / "hbm_traffic.json")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    tuning = dict(rec["tuning"])
    assert bench.hbm_traffic("freq_bwd", tuning) is not None      # an exact copy still matches
    with open(src, "a") as f:
        f.write("\n// edited\n")
    assert bench.hbm_traffic("freq_bwd", tuning) is None


def test_traffic_is_null_without_a_record(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.hbm_traffic("freq_bwd", dict(_record()["tuning"])) is None


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout == ""


def test_default_run_uses_the_recorded_schedules():
    """A default bench run (library schedules) reports counted traffic: the committed record
    was taken with exactly those schedules."""
    assert bench.effective_tuning(None) == _record()["tuning"]


def test_decoder_bound_hand_cases():
    """The decoder's combined bound against sums worked by hand: a 4-channel first layer
    (every kernel HBM-bound) and a stride-1, 128-channel stack (the MFMA term wins where
    the kernel moves fewer than 312 bytes per 1e5 flops)."""
    # hidden 4 -> 128 at stride 2 on 8 frames, output layer on 16 samples, batch 1:
    # bytes 8256 (forward), 4160 (weight gradient); output 4160, 12352, 4160; all at 8 TB/s
    got = bench.decoder_bound_ms([(128, 4, 2), (1, 128, 1)], 8, 1)
    assert abs(got - 33088 / 8e12 * 1e3) < 1e-15
    # two 128 -> 128 stride-1 layers on 8 frames, batch 2: forward and weight gradient of
    # both at 4 718 592 flops and 2.5 PFLOP/s (1.8874368 ns each); the second layer's data
    # gradient moves 16 384 bytes (2.048 ns; the first layer has none); output layer
    # 0.52 + 1.544 + 0.52 ns
    got = bench.decoder_bound_ms([(128, 128, 1), (128, 128, 1), (1, 128, 1)], 8, 2)
    expect = (4 * 1.8874368e-9 + 2.048e-9 + 0.52e-9 + 1.544e-9 + 0.52e-9) * 1e3
    assert abs(got - expect) < 1e-9 * expect
