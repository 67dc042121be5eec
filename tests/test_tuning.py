"""The autotuner's table: bucket keys and the nearest-bucket lookup that
pphd.Filter and pphd.Batch apply at creation (host logic, no GPU)."""
import json

from paper_1503_03769_amd import pphd


def test_bucket_keys():
    assert pphd.tuning_bucket(pphd.PPHD_FP32, False, 64, 32768, 60.0) == "fp32/g6/cap15/m6"
    assert pphd.tuning_bucket(pphd.PPHD_FP64, True, 256, 300000, 65.0) == "fp64_batch/g8/cap18/m6"


def test_lookup_exact_then_nearest_of_the_same_kind(tmp_path, monkeypatch):
    table = {
        "fp32/g6/cap15/m6": {"pt_cz": 4, "pt_weight": 4, "pass_workgroups": 1024, "rs_tiles": 2},
        "fp32/g4/cap15/m6": {"pt_cz": 8, "pt_weight": 4, "pass_workgroups": 512, "rs_tiles": 1},
        "fp32_batch/g8/cap18/m6": {"pt_cz": 8, "pt_weight": 8, "pass_workgroups": 2048, "rs_tiles": 2},
    }
    path = tmp_path / "tuning.json"
    path.write_text(json.dumps(table))
    monkeypatch.setattr(pphd, "TUNING_PATH", str(path))
    assert pphd.lookup_tuning(pphd.PPHD_FP32, False, 64, 32768, 60.0) == table["fp32/g6/cap15/m6"]
    # 16 groups: nearer to g4 than to g6
    assert pphd.lookup_tuning(pphd.PPHD_FP32, False, 18, 32768, 60.0) == table["fp32/g4/cap15/m6"]
    # a batch never takes a single filter's shape, and no FP64 entry exists
    assert pphd.lookup_tuning(pphd.PPHD_FP32, True, 1, 4096, 20.0) == table["fp32_batch/g8/cap18/m6"]
    assert pphd.lookup_tuning(pphd.PPHD_FP64, False, 64, 32768, 60.0) is None
