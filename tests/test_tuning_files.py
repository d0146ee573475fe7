"""CPU checks of the autotuner's result files: each workload has its own file,
named by the workload (names may contain underscores), holding the workload's
signature, and the shipped files load for the workloads they were tuned on."""
import json
import os

from paper_2605_10457_amd import autotune


def test_save_load_by_workload_name(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "TUNING_DIR", str(tmp_path))
    a = {"options": {"bounds_block": 128}, "ms": 1.0}
    b = {"options": {"bounds_block": 256}, "ms": 2.0}
    pa = autotune.save(a, "gfx950", "config4", "config4_1_8x8")
    pb = autotune.save(b, "gfx950", "config4_colocated", "config4_colocated_1_8x8")
    assert pa != pb
    assert autotune.load("gfx950", "config4")["options"]["bounds_block"] == 128
    got = autotune.load("gfx950", "config4_colocated")
    assert got["options"]["bounds_block"] == 256 and got["signature"] == "config4_colocated_1_8x8"
    assert autotune.load("gfx950", "config9") is None


def test_shipped_tuning_files_match_their_workloads():
    d = autotune.TUNING_DIR
    for f in sorted(os.listdir(d)):
        if not f.endswith(".json"):
            continue
        t = json.load(open(os.path.join(d, f)))
        arch, name = f[:-5].split("_", 1)
        assert t["arch"] == arch
        # the signature starts with the workload name the file is named after
        assert t["signature"].startswith(name + "_"), (f, t["signature"])
        assert set(t["options"]) <= set(autotune.SPACE) | {"group_cull"}, f
