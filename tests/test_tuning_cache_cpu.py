"""Host logic of the FFT launch-shape cache file (no GPU: the measurement and the
device query are replaced by stand-ins that record their calls)."""
import json
import os

import torch

from paper_2404_02783_amd import tuning


class _Plan:
    def __init__(self, n, dtype, batch):
        self.n, self.dtype, self.batch, self.device = n, dtype, batch, torch.device("cpu")


def test_tune_measures_once_then_reads_the_file(tmp_path, monkeypatch):
    calls = {"autotune": 0, "set": []}

    def fake_autotune(plan, reps=3, use_cache=True, mesh_scratch=None):
        calls["autotune"] += 1
        return [4, 8, 2, 16], [0.5, 0.6, 0.1, 0.2]

    monkeypatch.setattr(tuning, "pm_plan_autotune", fake_autotune)
    monkeypatch.setattr(tuning, "pm_plan_set_tuning", lambda plan, shapes: calls["set"].append(list(shapes)))
    monkeypatch.setattr(tuning.torch.cuda, "get_device_name", lambda dev=None: "AMD Instinct MI355X")
    path = os.path.join(tmp_path, "shapes.json")
    p64 = _Plan(64, torch.float32, 16)
    assert tuning.tune(p64, path) == ([4, 8, 2, 16], "measured")
    assert calls["autotune"] == 1 and calls["set"] == []
    # a second plan with the same key is served from the file, without measuring
    assert tuning.tune(_Plan(64, torch.float32, 16), path) == ([4, 8, 2, 16], "file")
    assert calls["autotune"] == 1 and calls["set"] == [[4, 8, 2, 16]]
    # another dtype or batch is another key: measured and added, the first entry kept
    tuning.tune(_Plan(64, torch.float64, 16), path)
    tuning.tune(_Plan(64, torch.float32, 8), path)
    assert calls["autotune"] == 3
    with open(path) as f:
        table = json.load(f)
    assert set(table) == {"AMD Instinct MI355X|n=64|f32|boxes=16", "AMD Instinct MI355X|n=64|f64|boxes=16",
                          "AMD Instinct MI355X|n=64|f32|boxes=8"}
    assert table["AMD Instinct MI355X|n=64|f32|boxes=16"]["shapes"] == [4, 8, 2, 16]
    assert not os.path.exists(path + ".tmp")


def test_tune_without_a_file_reports_the_process_cache(monkeypatch):
    monkeypatch.setattr(tuning, "pm_plan_autotune", lambda plan, reps=3, use_cache=True, mesh_scratch=None:
                        ([1, 2, 4, 8], [-1.0, -1.0, -1.0, -1.0]))
    monkeypatch.setattr(tuning.torch.cuda, "get_device_name", lambda dev=None: "gpu")
    assert tuning.tune(_Plan(32, torch.float32, 1)) == ([1, 2, 4, 8], "process")
