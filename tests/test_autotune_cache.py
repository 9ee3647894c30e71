"""Host side of the autotuner (no GPU): cache keys and the JSON round trip."""
from paper_1507_04941_amd import autotune

import torch


def test_keys_name_device_class_bank_box_dtype():
    k = autotune.entry_key("AMD Instinct MI355X", 28,
                           [(4.0, 8.0), (1.0, 2.0), (2.0, 2.0)], (64, 64, 64), torch.float16)
    assert k == "AMD Instinct MI355X|28|3/6,6/6,12/24|64x64x64|f16"
    assert autotune.bank_key([(1.0, 1.0)]) == "3/3"
    assert autotune.entry_key("d", 3, [(1, 1)], 8, torch.float32) == "d|3|3/3|8x8x8|f32"


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("GSF_TUNE_CACHE", str(tmp_path / "sub" / "t.json"))
    assert autotune.load() == {}
    c = {"d|3|3/3|8x8x8|f32": {"config": dict(autotune.DEFAULT), "ms": 1.0, "trials": []}}
    p = autotune.save(c)
    assert p.endswith("t.json")
    assert autotune.load() == c
