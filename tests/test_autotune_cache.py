"""The autotuner's on-disk cache (host logic, no GPU): keys by job class,
values written atomically and merged with what another process wrote."""
import json

import paper_2208_06970_amd.autotune as at


def test_cache_roundtrip_and_merge(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("LSRVT_AUTOTUNE_CACHE", str(path))
    monkeypatch.setattr(at, "_CACHE", None)
    k1 = at.job_class((64, 64, 64), 512, 5)
    assert k1 != at.job_class((64, 64, 64), 8, 5)          # voxels per site is part of the class
    assert k1 == at.job_class((64, 64, 64), 500, 5)         # same power-of-two bucket
    at._store(k1, {"engine": 2})
    # another process adds its own key meanwhile
    disk = json.loads(path.read_text())
    disk["other"] = {"engine": 1}
    path.write_text(json.dumps(disk))
    at._store("mine", {"engine": 1})
    disk = json.loads(path.read_text())
    assert disk[k1] == {"engine": 2} and disk["other"] == {"engine": 1} and disk["mine"] == {"engine": 1}
    # a fresh process reads the file
    monkeypatch.setattr(at, "_CACHE", None)
    assert at._load()[k1]["engine"] == 2


def test_unwritable_cache_keeps_results_in_memory(tmp_path, monkeypatch):
    blocker = tmp_path / "file"
    blocker.write_text("x")
    monkeypatch.setenv("LSRVT_AUTOTUNE_CACHE", str(blocker / "sub" / "tune.json"))
    monkeypatch.setattr(at, "_CACHE", None)
    at._store("k", {"engine": 1})
    assert at._load()["k"] == {"engine": 1}
