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


def test_br_grid_times_a_short_loop_and_caches(tmp_path, monkeypatch):
    """The relaxation-grid choice (host logic; the library calls and the
    clock are replaced): with the components given, each candidate is timed
    on a two-update Lloyd loop, the fastest is kept, and the cached choice is
    returned later without timing."""
    import types

    import paper_2208_06970_amd as L
    monkeypatch.setenv("LSRVT_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(at, "_CACHE", None)
    monkeypatch.setattr(at, "_device_name", lambda: "dev")
    state = {"grid": 0, "engine": 0}
    calls = []

    def set_tuning(knob, value):
        assert knob == at.TUNE_BR_GRID
        prev, state["grid"] = state["grid"], value
        return prev

    def set_engine(e):
        prev, state["engine"] = state["engine"], e
        return prev

    def fake_cvt(band, comp, sites, weights, iters, want_mean_ds=True):
        calls.append(("cvt", state["grid"], state["engine"], iters))

    def fake_vt(band, sites):
        calls.append(("vt", state["grid"], state["engine"], None))

    cost = {1024: 3.0, 2048: 2.0, 4096: 1.0, 8192: 1.5}

    def fake_time(fn, reps=2):
        fn()
        return cost[state["grid"]]

    monkeypatch.setattr(at, "lsrvt_set_tuning", set_tuning)
    monkeypatch.setattr(at, "lsrvt_set_vt_engine", set_engine)
    monkeypatch.setattr(at, "lsrvt_vt", fake_vt)
    monkeypatch.setattr(L, "lsrvt_cvt", fake_cvt)
    monkeypatch.setattr(at, "_time", fake_time)
    band = types.SimpleNamespace(shape=(64, 64, 64))
    sites = types.SimpleNamespace(numel=lambda: 512)
    assert at.br_grid(band, sites, 5, comp=object()) == 4096
    assert [c[0] for c in calls] == ["cvt"] * 4 and {c[3] for c in calls} == {2}
    assert {c[2] for c in calls} == {at.VT_BRICKS}         # timed with the brick relaxation
    assert state == {"grid": 0, "engine": 0}                # knobs restored
    calls.clear()
    assert at.br_grid(band, sites, 5, tune=False) == 4096 and not calls   # from the cache
    monkeypatch.setattr(at, "_CACHE", None)
    assert at.br_grid(band, sites, 5, tune=False) == 4096   # from the file
    # another class, without components: one Voronoi pass per candidate
    other = types.SimpleNamespace(numel=lambda: 8)
    assert at.br_grid(band, other, 5) == 4096
    assert [c[0] for c in calls] == ["vt"] * 4
