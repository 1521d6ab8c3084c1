"""CPU checks of bench.py's host-side parts: the oracle baseline runs and
reports the fields of its JSON object."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2605_27323_amd import scenes  # noqa: E402


def test_cpu_baseline_runs_on_a_short_budget():
    scene, cam = scenes.cornell()
    cam = dict(cam, width=bench.W, height=bench.H)
    res = bench.cpu_baseline(scene, cam, budget_s=0.05, single_s=0.05)
    assert res["kind"] == "oracle" and res["unit"] == "path-samples/s"
    assert res["value"] > 0 and res["cores"] >= 1 and res["single_thread"]["value"] > 0
    assert "paths" in res["sample"]


def test_gpu_count_other_than_one_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
