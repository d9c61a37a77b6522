"""Host-side logic of the multi-view tuner: candidate set, workload
signature, cache location and tolerance of a damaged cache file."""

import json

from paper_2601_17354_amd import autotune


def test_candidates_cover_every_shape_and_batch():
    c = autotune.candidates()
    assert len(c) == 20 and len(set(c)) == 20
    assert {t for t, _ in c} == {(16, 16), (8, 8), (16, 8), (32, 8), (8, 32)}
    assert {b for _, b in c} == {32, 64, 128, 256}


def test_signature_names_the_workload():
    cams = [dict(width=640, height=480), dict(width=1920, height=1440)]
    a = autotune.signature(1000, 3, cams, True)
    assert a == "n1000-sh3-cached-640x480-1920x1440"
    assert autotune.signature(1000, 3, cams, False) != a
    assert autotune.signature(1000, 3, cams[::-1], True) != a


def test_cache_path_and_damaged_cache(tmp_path, monkeypatch):
    p = tmp_path / "tune.json"
    monkeypatch.setenv("PGS_TUNE_CACHE", str(p))
    assert autotune.cache_path() == str(p)
    p.write_text("{not json")
    assert autotune._load(str(p)) == {}
    p.write_text(json.dumps({"k": {"tile": [8, 8]}}))
    assert autotune._load(str(p)) == {"k": {"tile": [8, 8]}}
