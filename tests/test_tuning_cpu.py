"""Host logic of the launch-shape cache (paper_2403_12179_amd.tuning): the
candidate grid, the cache file's round trip, atomic rewrites that keep other
processes' entries, stale formats and corrupt files, and the cache keys."""
import json
import os

import pytest

from paper_2403_12179_amd import tuning


def test_candidates_cover_the_grid():
    c = tuning.candidates()
    assert len(c) == len(tuning.PLANES) * len(tuning.ROWS_LOG2) * len(tuning.ADDRESSING) == 24
    assert len({tuple(sorted(x.items())) for x in c}) == 24
    assert tuning.DEFAULT_SHAPE in c


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    tc = tuning.TuneCache(path)
    assert len(tc) == 0 and tc.get("k") is None
    tc.put("k", {"planes_per_thread": 2, "buffer_addressing": 0, "tile_rows_log2_cap": 3})
    again = tuning.TuneCache(path)
    assert again.get("k")["planes_per_thread"] == 2 and again.get("k")["format"] == tuning.FORMAT
    assert [f for f in os.listdir(tmp_path / "sub")] == ["tune.json"]  # no temporaries left


def test_put_keeps_entries_written_meanwhile(tmp_path):
    path = str(tmp_path / "tune.json")
    a = tuning.TuneCache(path)
    b = tuning.TuneCache(path)
    a.put("x", dict(tuning.DEFAULT_SHAPE))
    b.put("y", dict(tuning.DEFAULT_SHAPE))  # b loaded before a wrote
    d = json.load(open(path))
    assert set(d) == {"x", "y"}


def test_stale_format_and_corrupt_file(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"old": {"planes_per_thread": 1, "format": tuning.FORMAT + 1},
                                "cur": {"planes_per_thread": 8, "format": tuning.FORMAT}, "junk": 3}))
    tc = tuning.TuneCache(str(path))
    assert tc.get("old") is None and tc.get("junk") is None and tc.get("cur")["planes_per_thread"] == 8
    path.write_text("{not json")
    assert len(tuning.TuneCache(str(path))) == 0
    path.write_text("[1, 2]")
    assert len(tuning.TuneCache(str(path))) == 0


def test_env_path(monkeypatch, tmp_path):
    monkeypatch.setenv("BXMG_TUNE_CACHE", str(tmp_path / "e.json"))
    assert tuning.default_cache_path() == str(tmp_path / "e.json")
    monkeypatch.delenv("BXMG_TUNE_CACHE")
    assert tuning.default_cache_path().endswith(os.path.join(".cache", "bxmg", "tune.json"))


class _Box:
    def __init__(self, size):
        self.size = size


class _BA:
    def __init__(self, dom, boxes):
        self.domain = _Box(dom)
        self.boxes = [_Box(b) for b in boxes]

    def __len__(self):
        return len(self.boxes)


def test_keys():
    one = tuning._geom_one(_BA((64, 64, 32), [(32, 32, 32)] * 4))
    assert one == "dom64x64x32/b4/e32"
    many = tuning._geom_many([_BA((32,) * 3, [(32,) * 3]), _BA((48,) * 3, [(32, 32, 32), (16, 32, 32)] * 4),
                              _BA((32,) * 3, [(32,) * 3])])
    assert many == "32x32x32/b1/e32:2,48x48x48/b8/e32:1"
    k = tuning.make_key("gfx950", "batch", "f32-in-f64", "const", many, "PPP", ("libabc",))
    assert k.split("|") == ["gfx950", "batch", "f32-in-f64", "const", many, "PPP", "libabc"]
    assert tuning._arith({"precision": 1}) == "f32-in-f64" and tuning._arith({}) == "f64"


def test_fingerprint_follows_the_library():
    if not os.path.exists(tuning.L.LIB_PATH):
        pytest.skip("library not built")
    fp = tuning.lib_fingerprint()
    assert len(fp) == 12 and int(fp, 16) >= 0


def test_unwritable_cache_keeps_entry_in_memory(tmp_path):
    blocker = tmp_path / "file"
    blocker.write_text("not a folder")
    tc = tuning.TuneCache(str(blocker / "sub" / "tune.json"))  # parent is a file: cannot be created
    assert tc.put("k", dict(tuning.DEFAULT_SHAPE)) is False
    assert tc.get("k")["planes_per_thread"] == 4
