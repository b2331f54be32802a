"""Host logic of the window autotuner (no GPU): candidate delays and the JSON cache."""
from __future__ import annotations

import json

import pytest

autotune = pytest.importorskip("paper_2602_05255_amd.autotune", reason="liblrx.so not built")


def test_delay_candidates_follow_the_byte_model():
    # K* = sqrt(2 n / kbar): n = 128, k = 1 gives 16 (the paper's measured det optimum, Sec. IV)
    c = autotune.delay_candidates(128, 1, (1,))
    assert 16 in c and min(c) >= 2
    # every candidate respects the C ABI limit K * k_max <= 256 and the delay maximum
    for n in (64, 256, 1024):
        for km, ranks in ((1, (1,)), (4, (1, 2, 4)), (8, (1, 2, 4, 8))):
            for K in autotune.delay_candidates(n, km, ranks):
                assert K * km <= 256 and K <= 64
            assert autotune.delay_candidates(n, km, ranks)


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("LRX_TUNE_CACHE", str(path))
    assert autotune.cache_path() == str(path)
    autotune._store(str(path), {"k": {"delay": 8}})
    assert json.loads(path.read_text()) == {"k": {"delay": 8}}
    assert autotune._load(str(path / "missing")) == {}
