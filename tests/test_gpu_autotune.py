"""The autotuner times every tile/map candidate, returns the fastest, caches
it, and never changes results (integer and Life bodies are tile-invariant)."""
import numpy as np
import pytest

from gpu_helpers import note

pytestmark = pytest.mark.gpu


def _tm():
    from paper_1609_01490_amd import trimap
    return trimap


@pytest.mark.parametrize("workload,n,d", [(0, 4096, 0), (1, 2048, 0), (2, 2048, 0),
                                          (3, 700, 32), (4, 700, 32)])
def test_autotune_picks_the_fastest_candidate(workload, n, d, tmp_path):
    tm = _tm()
    tm.tune_cache_clear()
    note("autotune", workload, n, d)
    best, allc = tm.autotune(workload, n, d, reps=2, use_cache=False)
    assert allc, "no candidate timed"
    assert best["ms"] == min(c["ms"] for c in allc)
    assert all(c["ms"] > 0 for c in allc)
    maps = {c["map"] for c in allc}
    assert "lambda" in maps and "bb" in maps
    # a cached answer comes back unchanged without timing
    again, allc2 = tm.autotune(workload, n, d, reps=2, use_cache=True)
    assert again == best and allc2 == []
    # save / load round trip
    f = str(tmp_path / "tune.json")
    tm.tune_cache_save(f)
    tm.tune_cache_clear()
    tm.tune_cache_load(f)
    third, allc3 = tm.autotune(workload, n, d, reps=2, use_cache=True)
    assert allc3 == [] and third["tile"] == best["tile"] and third["map"] == best["map"]
